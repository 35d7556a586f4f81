"""Continuous-batching least-squares serving loop over the batched C-ABI call.

Requests (least-squares problems of uneven d, n and right-hand-side count)
arrive over time.  Each is generated into device memory when it arrives, on a
generator stream; it is admitted when its HBM footprint fits the budget next
to the requests already in flight and a slot is free; admitted requests wait
in a ready list until a solver stream is free, and then every ready request
(up to ``max_batch``) is solved by one batched multisketch sketch-and-solve
call (``sketch_lstsq_batched``) on that stream.  Several solver streams run
batches concurrently, and arrivals keep being generated and admitted while
batches run, so work of requests that arrived at different times overlaps on
the device (continuous batching).  A request's latency runs from its
scheduled arrival to the moment the host observes its batch's completion
event.

The solver is the library's; this module only schedules.  Inputs follow the
serving workload: A = Z diag(logspace(0, -log10 kappa, n)) Q (FP32; Q
orthogonal), B = A x* + 1e-6 N(0,1), h uniform, s Rademacher,
G ~ N(0, 1/k2), k = 2 n^2, k2 = 2 n.  Q is the product of two Householder
reflections I - 2 u u^T with Gaussian directions u: an orthogonal matrix that
mixes every column into every other.  The library's device generator makes a
request in one write pass over each input (a row of A is formed in registers
and both reflections applied there), so that generating an arriving request
costs little next to solving it.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import torch

import paper_2508_14209_amd as ms

@dataclass
class Request:
    id: int
    d: int
    n: int
    nrhs: int
    kappa: float
    k: int
    k2: int
    seed: int
    arrival: float = 0.0            # scheduled arrival, seconds from the start
    tensors: dict | None = None
    footprint: int = 0
    gen_event: object = None
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan
    status: int = -1
    batch: int = -1
    extra: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def footprint_bytes(d: int, n: int, nrhs: int, k: int, k2: int, w: int = 4,
                    refine: bool = False) -> int:
    """HBM a request holds while in flight: its inputs and output plus its
    share of the batched workspace (packed bucket/sign words, sketch,
    split-K partials, Z; with refinement also the QR factors, the FP64
    residual, its sketch and the Gaussian-stage partials of the residual)."""
    data = d * (n + nrhs) * w + d * 5 + k2 * k * w + n * nrhs * 8
    nsplit = (k + 1023) // 1024
    work = (d * 4 + k * (n + nrhs) * w + nsplit * k2 * (n + nrhs) * 4 + k2 * (n + nrhs) * 8
            + 1280)
    if refine:
        work += (k2 * n + n) * 8 + d * nrhs * 8 + k * nrhs * 8 + nsplit * k2 * nrhs * 8 + 1024
    return data + work


def generate(req: Request, device, g_dtype: str = "f32", a_dtype: str = "f32") -> dict:
    """Seeded synthetic inputs of one request, on the current stream, made by
    the library's device generator (ms_gen_lstsq_request: A = Z diag(D) Q with
    Q two Householder reflections, B = A x* + 1e-6 N(0,1), h, s, G in one
    write pass each).  A and B are FP32; a_dtype "f64" promotes them exactly
    for the plain FP64 path."""
    d, n, nrhs, k, k2 = req.d, req.n, req.nrhs, req.k, req.k2
    gdt = {"f32": ms.MS_F32, "bf16": ms.MS_BF16, "f64": ms.MS_F64}[g_dtype]
    t = ms.gen_lstsq_request(req.seed, d, n, nrhs, req.kappa, k, k2, g_dtype=gdt, device=device)
    A, B = t["A"], t["B"]
    if a_dtype == "f64":
        A64 = ms.empty_colmajor(d, n, torch.float64, device)
        A64.copy_(A)
        B64 = ms.empty_colmajor(d, nrhs, torch.float64, device)
        B64.copy_(B)
        A, B = A64, B64
    X = ms.empty_colmajor(n, nrhs, torch.float64, device)
    return dict(A=A, B=B, h=t["h"], s=t["s"], G=t["G"], X=X, k=k, xstar=t["xstar"])


class Admission:
    """HBM-budget admission: a request is admitted when a slot is free and its
    footprint fits the budget next to the requests in flight (a request larger
    than the whole budget is admitted alone, when nothing else is in flight).
    Host logic only."""

    def __init__(self, hbm_budget: int, max_inflight: int):
        self.hbm_budget = int(hbm_budget)
        self.max_inflight = int(max_inflight)
        self.bytes = 0
        self.count = 0
        self.peak_bytes = 0

    def try_admit(self, footprint: int) -> bool:
        if self.count >= self.max_inflight:
            return False
        if self.count and self.bytes + footprint > self.hbm_budget:
            return False
        self.count += 1
        self.bytes += footprint
        self.peak_bytes = max(self.peak_bytes, self.bytes)
        return True

    def release(self, footprint: int):
        self.count -= 1
        self.bytes -= footprint


class Server:
    """Continuous-batching scheduler (see the module docstring).

    hbm_budget: bytes the in-flight requests may hold together.
    max_inflight: request slots.  max_batch: requests per batched call.
    streams: solver streams running batches concurrently.
    """

    def __init__(self, hbm_budget: int = 64 << 30, max_inflight: int = 256, max_batch: int = 64,
                 streams: int = 4, g_dtype: str = "f32", rows_log2: int = 0,
                 kchunk_log2: int = 0, refine_steps: int = 0, tuned: bool = False,
                 a_dtype: str = "f32", single: bool = False, device="cuda",
                 persistent: bool = False, graphs: bool = True, max_shape=None,
                 deterministic: bool = False):
        self.device = torch.device(device)
        self.admission = Admission(hbm_budget, max_inflight)
        self.max_batch = max_batch
        self.g_dtype = g_dtype
        self.rows_log2 = rows_log2
        self.kchunk_log2 = kchunk_log2
        self.refine_steps = refine_steps
        self.tuned = tuned              # take rows/K per item from the autotuner's cache
        self.a_dtype = a_dtype          # "f64": A, B promoted exactly (the plain FP64 path)
        self.single = single            # one request per call of the single-problem solver
        # persistent: one BatchRunner per solver stream, its workspace sized
        # once for max_batch requests of the largest shape (d, n, nrhs) the
        # stream can send; a batch of fewer requests is padded with a 1-row
        # placeholder problem, so every call has the runner's count and its
        # launch sequence is captured once in a graph and replayed
        # deterministic: the batched CountSketch folds each bucket in row
        # order and the Gaussian stage's K split is fixed (no per-batch
        # tuning), so a request's solution does not depend on its batch
        self.deterministic = deterministic
        self.persistent = persistent and not single
        self.graphs = graphs
        self.max_shape = max_shape or (1 << 20, 128, 8)
        self.runners = {}
        self._pad = None
        self.gen_stream = torch.cuda.Stream(device=self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.busy = {}                # stream index -> (event, runner, requests)
        self.waiting = deque()        # arrived, not yet admitted (budget / slots)
        self.ready = deque()          # admitted, inputs being / been generated
        self.done = []
        self.nbatches = 0
        self.t0 = None

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- arrivals and admission ------------------------------------------------
    def arrive(self, req: Request):
        req.footprint = footprint_bytes(req.d, req.n, req.nrhs, req.k, req.k2,
                                        w=8 if self.a_dtype == "f64" else 4,
                                        refine=self.refine_steps > 0)
        self.waiting.append(req)
        self._admit()

    def _admit(self):
        while self.waiting:
            req = self.waiting[0]
            if not self.admission.try_admit(req.footprint):
                return
            self.waiting.popleft()
            req.t_admit = self.now()
            with torch.cuda.stream(self.gen_stream):
                req.tensors = generate(req, self.device, self.g_dtype, self.a_dtype)
                ev = torch.cuda.Event()
                ev.record(self.gen_stream)
            req.gen_event = ev
            self.ready.append(req)

    # -- batches -----------------------------------------------------------------
    def _launch(self):
        for si, st in enumerate(self.streams):
            if si in self.busy or not self.ready:
                continue
            batch = []
            cap = 1 if self.single else self.max_batch
            while self.ready and len(batch) < cap:
                batch.append(self.ready.popleft())
            probs = [r.tensors for r in batch]
            st.wait_stream(self.gen_stream)     # inputs generated before the solve
            for pr in probs:                    # memory of the generator stream used here
                for key in ("A", "B", "h", "s", "G", "X"):
                    pr[key].record_stream(st)
            if self.single:
                # the paper's path: one sketch_lstsq call per request
                pr = probs[0]
                with torch.cuda.stream(st):
                    _, ws = ms.sketch_lstsq(pr["A"], pr["B"], pr["h"], pr["s"], pr["G"], pr["k"],
                                            refine_steps=self.refine_steps, X=pr["X"], stream=st)
                    ev = torch.cuda.Event()
                    ev.record(st)
                runner = ("single", ws)
            elif self.persistent:
                runner = self._stream_runner(si, st, probs)
                padded = probs + [self._pad_problem()] * (self.max_batch - len(probs))
                with torch.cuda.stream(st):
                    runner.set_problems(padded, stream=st)
                    if self.graphs:
                        runner.replay()
                    else:
                        runner.launch(st)
                    ev = torch.cuda.Event()
                    ev.record(st)
            else:
                rl, kl = self.rows_log2, self.kchunk_log2
                if self.tuned and not (rl or kl) and not self.deterministic:
                    from paper_2508_14209_amd import autotune
                    rl, kl = autotune.batch_params(probs, self.device)
                with torch.cuda.stream(st):
                    runner = ms.BatchRunner(probs, rows_log2=rl, kchunk_log2=kl,
                                            refine_steps=self.refine_steps,
                                            deterministic=self.deterministic)
                    runner.launch(st)
                    ev = torch.cuda.Event()
                    ev.record(st)
            tl = self.now()
            for r in batch:
                r.t_launch = tl
                r.batch = self.nbatches
            self.nbatches += 1
            self.busy[si] = (ev, runner, batch)

    def _pad_problem(self) -> dict:
        """A 1-row, 1-column problem (k = k2 = 1) that fills unused batch slots."""
        if self._pad is None:
            dev = self.device
            adt = torch.float64 if self.a_dtype == "f64" else torch.float32
            gdt = {"f64": torch.float64, "bf16": torch.bfloat16}.get(self.g_dtype, torch.float32)
            A = ms.empty_colmajor(1, 1, adt, dev)
            A.fill_(1.0)
            B = ms.empty_colmajor(1, 1, adt, dev)
            B.fill_(1.0)
            G = ms.empty_colmajor(1, 1, gdt, dev)
            G.fill_(1.0)
            self._pad = dict(A=A, B=B, h=torch.zeros(1, dtype=torch.int32, device=dev),
                             s=torch.ones(1, dtype=torch.int8, device=dev), G=G,
                             X=ms.empty_colmajor(1, 1, torch.float64, dev), k=1)
        return self._pad

    def _capacity(self) -> list:
        """Shapes the persistent runners are sized for: max_batch copies of
        the largest request (d, n, nrhs, k, k2)."""
        d, n, nrhs = self.max_shape
        return [(d, n, nrhs, 2 * n * n, 2 * n)] * self.max_batch

    def _stream_runner(self, si, st, probs):
        r = self.runners.get(si)
        if r is None:
            rl, kl = self.rows_log2, self.kchunk_log2
            if self.tuned and not (rl or kl) and not self.deterministic:
                from paper_2508_14209_amd import autotune
                rl, kl = autotune.batch_params(probs, self.device)
            padded = probs + [self._pad_problem()] * (self.max_batch - len(probs))
            with torch.cuda.stream(st):
                r = ms.BatchRunner(padded, capacity=self._capacity(), rows_log2=rl,
                                   kchunk_log2=kl, refine_steps=self.refine_steps,
                                   deterministic=self.deterministic)
            if self.graphs:
                with torch.cuda.stream(st):
                    r.capture()
            self.runners[si] = r
        return r

    def warm_runners(self, requests):
        """Build every stream's persistent runner (workspace, graph capture)
        before a timed run, tuned for the shape class of ``requests``."""
        if not self.persistent:
            return
        probs = [generate(r, self.device, self.g_dtype, self.a_dtype) for r in requests]
        probs = probs[:self.max_batch]
        for si, st in enumerate(self.streams):
            runner = self._stream_runner(si, st, probs)
            padded = probs + [self._pad_problem()] * (self.max_batch - len(probs))
            with torch.cuda.stream(st):
                runner.set_problems(padded, stream=st)
                if self.graphs:
                    runner.replay()
                else:
                    runner.launch(st)
        torch.cuda.synchronize(self.device)

    def _complete(self):
        for si in list(self.busy):
            ev, runner, batch = self.busy[si]
            if not ev.query():
                continue
            t = self.now()
            if isinstance(runner, tuple):
                try:
                    ms.check_status(runner[1], self.streams[si])
                    per = [ms.MS_OK]
                except ms.MsketchError as e:
                    per = [e.code]
            else:
                st, per = runner.status(self.streams[si])
            for r, code in zip(batch, per):
                r.t_done = t
                r.status = code
                self.admission.release(r.footprint)
                self.done.append(r)
            del self.busy[si]
        self._admit()

    def step(self):
        self._complete()
        self._launch()

    def idle(self) -> bool:
        return not (self.busy or self.ready or self.waiting)

    # -- drivers -------------------------------------------------------------------
    def run(self, requests, keep_tensors: bool = False):
        """Open loop: request r arrives at r.arrival seconds after the start."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = time.perf_counter()
        while pending or not self.idle():
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.arrive(pending.popleft())
            self.step()
            if not keep_tensors:
                for r in self.done:
                    if r.tensors is not None and not r.extra.get("kept"):
                        r.tensors = None
            if pending and self.idle():
                time.sleep(max(0.0, min(pending[0].arrival - self.now(), 1e-3)))
        torch.cuda.synchronize(self.device)
        return self.done


def make_requests(count: int, rate: float, seed: int = 14209, **kw):
    """The serving stream: synth's request descriptors with Poisson arrivals."""
    import synth
    desc = synth.serving_requests(count, seed, **kw)
    times = synth.poisson_arrivals(count, rate, seed) if rate > 0 else [0.0] * count
    return [Request(id=dd["id"], d=dd["d"], n=dd["n"], nrhs=dd["nrhs"], kappa=dd["kappa"],
                    k=dd["k"], k2=dd["k2"], seed=dd["seed"], arrival=float(t))
            for dd, t in zip(desc, times)]


def summarize(done, wall: float) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in done if r.status == ms.MS_OK]) * 1e3
    ok = len(lat)
    return {"requests": len(done), "ok": ok,
            "solves_per_s": ok / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if ok else None,
            "p99_ms": float(np.percentile(lat, 99)) if ok else None,
            "mean_ms": float(lat.mean()) if ok else None}
