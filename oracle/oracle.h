/*
 * oracle.h -- declarations of the CPU reference (test infrastructure only;
 * see oracle.c).  Column-major storage, 0-based bucket indices, signs +-1.
 */
#ifndef MSKETCH_ORACLE_H
#define MSKETCH_ORACLE_H

#include <stdint.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG 1
#define ORACLE_ERR_RANGE 2
#define ORACLE_ERR_NOMEM 3
#define ORACLE_ERR_SINGULAR 4

int or_countsketch_f64(int64_t d, int64_t n, int64_t k, const double *A,
                       int64_t lda, const int32_t *h, const int8_t *s,
                       double *Y, int64_t ldy);
int or_countsketch_f32(int64_t d, int64_t n, int64_t k, const float *A,
                       int64_t lda, const int32_t *h, const int8_t *s,
                       float *Y, int64_t ldy);
int or_countsketch_f32_acc64(int64_t d, int64_t n, int64_t k, const float *A,
                             int64_t lda, const int32_t *h, const int8_t *s,
                             double *Y, int64_t ldy);
/* or_countsketch_f64 with its columns split over nthreads host threads
 * (bit-identical: each column is folded in the canonical order) */
int or_countsketch_f64_cols(int64_t d, int64_t n, int64_t k, const double *A,
                            int64_t lda, const int32_t *h, const int8_t *s,
                            double *Y, int64_t ldy, int nthreads);
int or_bucket_hist(int64_t d, int64_t k, const int32_t *h, int64_t *cnt);
int or_bucket_plan(int64_t d, int64_t k, const int32_t *h, int64_t *off,
                   int64_t *perm);
void or_gemm_f64(int64_t M, int64_t N, int64_t K, const double *G, int64_t ldg,
                 const double *Y, int64_t ldy, double *Z, int64_t ldz);
void or_householder_qr(int64_t m, int64_t n, double *W, int64_t ldw,
                       double *tau);
void or_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *W,
                 int64_t ldw, const double *tau, double *B, int64_t ldb);
int or_trsv_upper(int64_t n, int64_t nrhs, const double *R, int64_t ldr,
                  double *B, int64_t ldb);
int or_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W,
                int64_t ldw, const double *Bm, int64_t ldb, double *X,
                int64_t ldx);
int or_normal_equations(int64_t d, int64_t n, int64_t nrhs, const double *A,
                        int64_t lda, const double *B, int64_t ldb, double *X,
                        int64_t ldx);
int or_sketch_lstsq_f64(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                        int64_t k2, const double *A, int64_t lda,
                        const double *B, int64_t ldb, const int32_t *h,
                        const int8_t *s, const double *G, int64_t ldg,
                        double *X, int64_t ldx, double *Ys, double *Zs);
float or_round_bf16(float x);
void or_round_bf16_array(int64_t count, const float *x, float *out);
/* flags of or_sketch_lstsq_f32: round the FP32 sketch to BF16 before the
 * Gaussian stage; form the FP32 sketch as Def. 3's sums in FP64 rounded once
 * to FP32 (else folded in FP32, the canonical order) */
#define ORACLE_Y_BF16 1
#define ORACLE_Y_ACC64 2
#define ORACLE_Y_F16 4
int or_sketch_lstsq_f32(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                        int64_t k2, const float *A, int64_t lda,
                        const float *B, int64_t ldb, const int32_t *h,
                        const int8_t *s, const double *G, int64_t ldg,
                        int y_bf16, double *X, int64_t ldx, float *Ys,
                        double *Zs);
int or_rand_cholqr_from_sketch(int64_t d, int64_t n, int64_t nrhs, int64_t m,
                               const double *SA, int64_t lds, const double *A,
                               int64_t lda, const double *B, int64_t ldb, double *X,
                               int64_t ldx, double *Rout, int64_t ldr);

void or_splitmix64(uint64_t seed, int64_t count, uint64_t *out);
int or_hash_sketch(int64_t d, int64_t k, uint64_t seed, int32_t *h, int8_t *s);

int or_srht(int64_t mx, int64_t ncols, int64_t k, const double *X, int64_t ldx,
            const int8_t *dsign, const int32_t *r, double *Y, int64_t ldy);

float or_round_f16(float x);
int or_f16_col_exp(int64_t k, const float *y);
void or_round_f16_colscaled(int64_t k, int64_t nc, const float *Y, int64_t ldy,
                            double *out, int64_t ldo);

#endif
