"""Sec. 6.3's conditioning experiment on the GPU: with b = A e (a consistent
system) and A of 2^17 x 16 with condition number kappa from 1e2 to 1e12, the
normal equations lose accuracy once kappa passes about u^{-1/2} (the paper
sees them fail beyond 1e8), while multisketch sketch-and-solve behaves like
a Householder QR least-squares solve.

Both GPU solvers go through the C ABI; the QR comparator is LAPACK's
least-squares solve on the same data.  The reported quantity is the paper's
relative residual ||b - A x|| / ||b||.  Bars (as for the oracle's own
conditioning pin): sketch-and-solve and QR below 1e-10 at every kappa (a
backward-stable solve of a consistent system leaves a residual of a small
multiple of u ||A|| ||x||); the normal equations below 1e-12 at kappa = 1e2,
and at kappa >= 1e10 either a reported breakdown or a residual at least 1e3
times the other two solvers' (their forward error grows like kappa^2 u).
"""
import numpy as np
import pytest

import synth
from gpu_util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


KAPPAS = [1e2, 1e4, 1e6, 1e8, 1e10, 1e12]


def test_conditioning_sweep(ms, orc):
    d, n = 1 << 17, 16
    k, k2 = 2 * n * n, 2 * n
    h = synth.bucket_map(d, k, seed=17)
    s = synth.signs(d, seed=17)
    G = synth.gaussian_sketch(k2, k, seed=17)
    hd, sd, Gd = to_dev(h), to_dev(s), to_dev(G)
    for kappa in KAPPAS:
        A = synth.conditioned_matrix(d, n, kappa, seed=17)
        b = synth.paper_rhs(A, seed=17)
        Ad, bd = to_dev(A), to_dev(b)

        def relres(x):
            return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))

        Xs, ws = ms.sketch_lstsq(Ad, bd, hd, sd, Gd, k)
        ms.check_status(ws)
        r_ss = relres(to_host(Xs))
        Xn, _, wn = ms.normal_equations_lstsq(Ad, bd)
        try:
            ms.check_status(wn)
            r_ne = relres(to_host(Xn))
        except ms.MsketchError as e:
            assert e.code == ms.MS_ERR_SINGULAR
            r_ne = np.inf
        r_qr = relres(np.linalg.lstsq(A, b, rcond=None)[0])
        print("kappa %.0e: relative residual  normal equations %.3e  sketch-and-solve %.3e  "
              "QR %.3e" % (kappa, r_ne, r_ss, r_qr), flush=True)
        assert r_ss < 1e-10 and r_qr < 1e-10
        if kappa == 1e2:
            assert r_ne < 1e-12
            # and the GPU normal equations agree with the oracle's there
            assert rel(to_host(Xn), orc.normal_equations(A, b)) <= 1e-10
            # (kappa u = 1e-14: the FP64 bar binds for sketch-and-solve)
            Xso, _, _ = orc.sketch_lstsq(A, b, h, s, G, k)
            assert rel(to_host(Xs), Xso) <= 1e-12
        if kappa >= 1e10:
            assert r_ne > 1e3 * max(r_ss, r_qr)
