"""Serving loop: many independent AltGDmin-LR+S problems on one GPU.

Requests arrive over time (a Poisson process); each one brings its sizes and
the seed of its data.  The scheduler

  * admits waiting requests in arrival order while the sum of their device
    footprints (stored A, Y, X*, and the exact workspace of
    altgdmin_workspace_bytes) stays within an HBM budget; a request larger than
    the whole budget is rejected;
  * on admission, writes the request's A and y on the device
    (altgdmin_op_make_a, altgdmin_op_measure) and enqueues the initialisation of
    Alg. 1 (altgdmin_init);
  * advances every admitted problem together, `poll_every` GDmin iterations per
    round, with altgdmin_step_many (the column, gradient and QR kernels of all
    problems share launches); the round's launches go out before the host
    admits new requests, so admission overlaps the GPU work, and a request
    admitted during a round joins the next one;
  * after each round reads every active problem's status with one
    synchronisation (altgdmin_status_many) and retires those whose relative
    residual is at or below `tol`, that reached `max_iters` iterations, whose
    kernels raised an error flag (a non-finite value, an indefinite Gram
    matrix, invalid state), that diverge (the residual, above `diverge_floor`,
    rose by more than `diverge_rise` at `diverge_polls` polls in a row, or is not
    finite), or that stall (no new minimum by 1 % for `stall_polls` polls: above
    `diverge_floor` a failure -- the period-2 oscillation of a step that is too
    long looks flat when the polls fall on iterations of one parity -- and at or
    below it the FP32 rounding floor of a request whose `tol` sits just under
    it, retired as `at_floor`), recording the latency (completion minus
    arrival) and the error against X*;
  * optionally (`retry_step_limit`) re-queues a diverged or stalled request, at
    the head of the queue, when its step is too long: the fixed step of Sec. 2.6
    scales the error along direction i by about 1 - eta m sigma_i(B)^2 (Gaussian
    A_k, E[A_k^T A_k] = m I), so with an initialisation that is already accurate
    eta m sigma_max^2 exceeds 2 and the iteration cannot settle.  The executor's
    step_diagnostic(job) gives eta m sigma_max(B_t)^2 from the current iterate
    (no knowledge of X*); above the limit, the retry scales eta_c by 1 over it.
    Requests that stall for other reasons are not retried;
  * honours cancel(idx), from any thread: a request still waiting is dropped,
    an admitted one is released (its handle destroyed, its footprint returned to
    the budget) before the next round.

The scheduling logic is host-only and takes an executor object, so it can be
exercised without a GPU; GpuExecutor is the one that drives the library.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import itertools
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import instances as inst
from . import roofline


@dataclasses.dataclass
class Outcome:
    idx: int
    arrival: float
    admitted: float
    done: float
    iterations: int
    resid: float
    converged: bool
    error: float            # ||X - X*||_F / ||X*||_F of the consistent pair
    rejected: bool = False
    error_flags: int = 0    # the kernels' error bits when the request was retired
    cancelled: bool = False
    diverged: bool = False
    stalled: bool = False
    at_floor: bool = False  # stalled at or below diverge_floor: the rounding floor, not a failure
    attempts: int = 1       # 1 + retries with a shorter step
    eta_m_sigma2: float = float("nan")   # eta m sigma_max(B*)^2 of the last attempt, when the executor reports it
    step_diag: float = float("nan")      # eta m sigma_max(B_t)^2 from the iterate, when a failure was checked
    bytes_per_iteration: float = 0.0     # algorithmic HBM bytes of one GDmin iteration (A_k U + column kernel)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class ServeReport:
    outcomes: List[Outcome]
    makespan: float
    budget_bytes: int
    peak_bytes: int
    rounds: int
    host_seconds: dict = dataclasses.field(default_factory=dict)

    def summary(self, err_bound: float = 1e-6) -> dict:
        """Counts, throughput and latency.  A completed request is one the scheduler
        retired (converged, at the iteration cap, diverged, or with an error flag);
        rejected and cancelled requests are counted apart.  Only converged ones
        count as solves in converged_solves_per_s; error_violations counts every
        completed request whose error exceeds err_bound, converged or not."""
        done = [o for o in self.outcomes if not o.rejected and not o.cancelled]
        lat = np.array([o.latency for o in done]) if done else np.zeros(1)
        conv = [o for o in done if o.converged]
        unconv = [o for o in done if not o.converged]
        return {
            "requests": len(self.outcomes),
            "completed": len(done),
            "rejected": sum(1 for o in self.outcomes if o.rejected),
            "cancelled": sum(1 for o in self.outcomes if o.cancelled),
            "solves_per_s": len(done) / self.makespan if self.makespan > 0 else 0.0,
            "converged_solves_per_s": len(conv) / self.makespan if self.makespan > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "converged_fraction": len(conv) / max(1, len(done)),
            "max_error_converged": max((o.error for o in conv), default=float("nan")),
            "not_converged": len(unconv),
            "max_error_not_converged": max((o.error for o in unconv), default=float("nan")),
            "retired_with_error_flags": sum(1 for o in done if o.error_flags),
            "diverged": sum(1 for o in done if o.diverged),
            "stalled": sum(1 for o in done if o.stalled),
            "at_floor": sum(1 for o in done if o.at_floor),
            "retried": sum(1 for o in done if o.attempts > 1),
            "converged_after_retry": sum(1 for o in done if o.attempts > 1 and o.converged),
            "not_converged_detail": [{"idx": o.idx, "iterations": o.iterations, "resid": o.resid, "error": o.error,
                                      "attempts": o.attempts, "eta_m_sigma2": o.eta_m_sigma2,
                                      "step_diag": o.step_diag,
                                      "why": "diverged" if o.diverged else "stalled" if o.stalled else
                                      "at floor" if o.at_floor else "error flag" if o.error_flags else
                                      "iteration cap"} for o in unconv][:16],
            "error_violations": sum(1 for o in done if not (o.error <= err_bound)),
            "mean_iterations": float(np.mean([o.iterations for o in done])) if done else 0.0,
            # algorithmic bytes of the GDmin iterations run (last attempt of each request;
            # initialisations not counted) over the makespan: a lower bound of the HBM rate
            "iteration_GBps": (sum(o.iterations * o.bytes_per_iteration for o in done) / self.makespan / 1e9
                               if self.makespan > 0 else 0.0),
            "makespan_s": self.makespan,
            "budget_gib": self.budget_bytes / 2**30,
            "peak_admitted_gib": self.peak_bytes / 2**30,
            "rounds": self.rounds,
            "host_seconds": {k: round(v, 4) for k, v in self.host_seconds.items()},
        }


@dataclasses.dataclass
class _Active:
    req: object
    job: object
    footprint: int
    admitted: float
    iterations: int = 0
    resid: float = float("nan")
    rises: int = 0          # consecutive polls at which the residual rose
    best: float = float("inf")
    since_best: int = 0     # polls since the residual last reached a new minimum (by 1 %)


class Scheduler:
    """FIFO admission by footprint, batched stepping, retire on residual, cap,
    error flag or divergence; cancellation from any thread."""

    def __init__(self, executor, budget_bytes: int, poll_every: int = 10, tol: float = 1e-7,
                 max_iters: int = 300, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, prefetch: int = 16,
                 max_active: Optional[int] = None, diverge_polls: int = 3, diverge_rise: float = 0.01,
                 diverge_floor: float = 1e-5, stall_polls: int = 6, retry_step_limit: Optional[float] = None,
                 max_retries: int = 1):
        if poll_every < 1 or max_iters < 1:
            raise ValueError("poll_every and max_iters must be >= 1")
        if diverge_polls < 0 or diverge_rise < 0 or stall_polls < 0 or max_retries < 0:
            raise ValueError("diverge_polls, diverge_rise, stall_polls and max_retries must be >= 0")
        if retry_step_limit is not None and not retry_step_limit >= 1.0:
            raise ValueError("retry_step_limit must be >= 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.poll_every = poll_every
        self.tol = tol
        self.max_iters = max_iters
        self.clock = clock
        self.sleep = sleep
        self.prefetch = prefetch
        self.max_active = max_active   # None: limited by the budget only; 1: one request at a time
        self.diverge_polls = diverge_polls   # 0: never retire for divergence
        self.diverge_rise = diverge_rise
        self.diverge_floor = diverge_floor
        self.stall_polls = stall_polls       # 0: never retire for a stall
        self.retry_step_limit = retry_step_limit
        self.max_retries = max_retries
        self._lock = threading.Lock()
        self._cancel = set()

    def cancel(self, idx: int) -> None:
        """Ask for request `idx` to be dropped (waiting) or released (admitted)
        before the next round.  Thread-safe; a request already retired, or an
        unknown index, is ignored."""
        with self._lock:
            self._cancel.add(int(idx))

    def _take_cancels(self) -> set:
        with self._lock:
            out, self._cancel = self._cancel, set()
        return out

    def _diverging(self, a: _Active, resid: float) -> bool:
        """Updates the rise count of `a` with the new residual; True once it diverges."""
        if not np.isfinite(resid):
            return True
        if self.diverge_polls == 0:
            return False
        rose = np.isfinite(a.resid) and resid > self.diverge_floor and resid > a.resid * (1.0 + self.diverge_rise)
        a.rises = a.rises + 1 if rose else 0
        return a.rises >= self.diverge_polls

    def _stalled(self, a: _Active, resid: float) -> bool:
        """Updates the poll count since the last new minimum; True once it reaches stall_polls."""
        if resid < a.best * 0.99:
            a.best, a.since_best = resid, 0
            return False
        a.since_best += 1
        return self.stall_polls > 0 and a.since_best >= self.stall_polls

    def run(self, requests) -> ServeReport:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.idx)))
        waiting = collections.deque()
        active: List[_Active] = []
        outcomes = []
        used = peak = 0
        rounds = 0
        spent = collections.Counter()     # wall time inside each executor call
        attempts = collections.defaultdict(lambda: 1)
        prepare = getattr(self.ex, "prepare", None)
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731

        def timed(name, fn, *args):
            a = self.clock()
            out = fn(*args)
            spent[name] += self.clock() - a
            return out

        def release(a: _Active):
            rel = getattr(self.ex, "release", None)
            timed("release", rel if rel is not None else self.ex.finish, a.job)

        while pending or waiting or active:
            t = now()
            cancels = self._take_cancels()
            if cancels:
                for q in (pending, waiting):
                    for req in [r for r in q if r.idx in cancels]:
                        q.remove(req)
                        outcomes.append(Outcome(req.idx, req.arrival, t, t, 0, float("nan"), False, float("nan"),
                                                cancelled=True))
                        if hasattr(self.ex, "forget"):
                            self.ex.forget(req)
                keep = []
                for a in active:
                    if a.req.idx in cancels:
                        release(a)
                        used -= a.footprint
                        outcomes.append(Outcome(a.req.idx, a.req.arrival, a.admitted, now(), a.iterations, a.resid,
                                                False, float("nan"), cancelled=True))
                    else:
                        keep.append(a)
                active = keep
                if not (pending or waiting or active):
                    break
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            # the round's batched step goes out first (asynchronous on the GPU), and the
            # host admits waiting requests while it runs; they join the next round
            stepped = list(active)
            if stepped:
                timed("step", self.ex.step, [a.job for a in stepped], self.poll_every)
                rounds += 1
            if prepare is not None:          # host-side payloads of the next few, made in the background
                for req in itertools.islice(waiting, self.prefetch):
                    prepare(req)
            while waiting:
                req = waiting[0]
                fp = self.ex.footprint(req)
                if fp > self.budget:
                    waiting.popleft()
                    outcomes.append(Outcome(req.idx, req.arrival, t, t, 0, float("nan"), False,
                                            float("nan"), rejected=True))
                    continue
                if used + fp > self.budget:
                    break
                if self.max_active is not None and len(active) >= self.max_active:
                    break
                waiting.popleft()
                job = timed("start", self.ex.start, req)
                used += fp
                peak = max(peak, used)
                active.append(_Active(req, job, fp, now()))
            if not stepped:
                if not active and pending:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            admitted = active[len(stepped):]
            status = timed("poll", self.ex.poll, [a.job for a in stepped])
            keep = []
            retry = []
            for a, st in zip(stepped, status):
                iters, resid = st[0], st[1]
                flags = st[2] if len(st) > 2 else 0
                conv = resid <= self.tol and not flags
                diverged = not conv and not flags and self._diverging(a, resid)
                stalled = not conv and not flags and not diverged and self._stalled(a, resid)
                at_floor = stalled and resid <= self.diverge_floor
                stalled = stalled and not at_floor
                a.iterations, a.resid = iters, resid
                diag = float("nan")
                if (diverged or stalled) and self.retry_step_limit and attempts[a.req.idx] <= self.max_retries \
                        and hasattr(self.ex, "step_diagnostic"):
                    diag = timed("diagnose", self.ex.step_diagnostic, a.job)
                if diag > (self.retry_step_limit or float("inf")):
                    release(a)
                    used -= a.footprint
                    attempts[a.req.idx] += 1
                    retry.append(dataclasses.replace(a.req, eta_scale=a.req.eta_scale / diag))
                elif conv or iters >= self.max_iters or flags or diverged or stalled or at_floor:
                    out = timed("finish", self.ex.finish, a.job)
                    err, info = out if isinstance(out, tuple) else (out, {})
                    bpi = self.ex.iteration_bytes(a.req) if hasattr(self.ex, "iteration_bytes") else 0.0
                    outcomes.append(Outcome(a.req.idx, a.req.arrival, a.admitted, now(), iters, resid, conv, err,
                                            error_flags=int(flags), diverged=diverged, stalled=stalled,
                                            at_floor=at_floor,
                                            attempts=attempts[a.req.idx], step_diag=diag,
                                            eta_m_sigma2=info.get("eta_m_sigma2", float("nan")),
                                            bytes_per_iteration=bpi))
                    used -= a.footprint
                else:
                    keep.append(a)
            active = keep + admitted
            waiting.extendleft(reversed(retry))     # retries go first, in their original order
        makespan = max((o.done for o in outcomes), default=0.0) - min((o.arrival for o in outcomes), default=0.0)
        outcomes.sort(key=lambda o: o.idx)
        return ServeReport(outcomes, makespan, self.budget, peak, rounds, dict(spent))


class GpuExecutor:
    """Runs requests through the HIP library (torch for device memory).

    Two streams of default priority: a request's data (A, y) and its
    initialisation -- the tau_0 IHT iterations and the subspace iteration, mostly
    small latency-bound launches -- go on the init stream, so they overlap the
    batched GDmin iterations of the admitted problems on the step stream; the
    step stream waits on an event recorded after a request's initialisation
    before its first step.  BF16 requests run the mixed form (hi plane for the
    transposed products, hi + lo for every residual) unless bf16_mixed is False.
    """

    def __init__(self, tol: float = 1e-7, max_iters: int = 300, device: str = "cuda", bf16_mixed: bool = True):
        import torch
        from . import altgdmin as lib
        if not torch.cuda.is_available():
            raise RuntimeError("GpuExecutor needs a ROCm GPU")
        lib.load()
        self.torch, self.lib, self.device = torch, lib, device
        self.table = torch.from_numpy(inst.normal_table()).to(device)
        self.params = lib.default_params(tol_resid=tol, t_max=max_iters)
        self.params_bf16 = lib.default_params(tol_resid=tol, t_max=max_iters,
                                              flags=lib.FLAG_BF16_MIXED if bf16_mixed else 0)
        self.bf16_mixed = bf16_mixed
        self.group_ws = None
        self.init_stream = torch.cuda.Stream(device=device)
        self.step_stream = torch.cuda.Stream(device=device)
        self._ws_cache = {}
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=4)
        self._truth = {}

    def _make_truth(self, req):
        """X*^T, pinned for the upload, and sigma_min(B*)^2, sigma_max(B*)^2 (step diagnostic)."""
        t = inst.request_truth(req)
        sv = np.linalg.svd(t["B_star"], compute_uv=False)
        return self.torch.from_numpy(t["Xt"]).pin_memory(), (float(sv[-1]) ** 2, float(sv[0]) ** 2)

    def _params(self, req):
        base = self.params if req.a_format == "f32" else self.params_bf16
        if req.eta_scale == 1.0:
            return base
        par = self.lib.Params.from_buffer_copy(base)
        par.eta_c = base.eta_c * req.eta_scale
        return par

    def prepare(self, req) -> None:
        """Start drawing X* of a request on a host thread (pinned for the upload)."""
        if req.idx not in self._truth:
            self._truth[req.idx] = self._pool.submit(self._make_truth, req)

    # -- sizes
    def _problem_for_size(self, req):
        p = self.lib.Problem()
        p.n, p.q, p.m, p.r, p.rho = req.n, req.q, req.m, req.r, req.rho
        p.a_format = self.lib.ALTGDMIN_A_F32 if req.a_format == "f32" else self.lib.ALTGDMIN_A_BF16X2
        # placeholder addresses: only the layout is validated by the size query
        p.A, p.A_lo, p.Y = 1 << 20, 1 << 21, 1 << 24
        p.lda, p.a_stride_k, p.ldy = req.lda, req.lda * req.n, req.m
        return p

    def workspace_bytes(self, req) -> int:
        key = (req.n, req.q, req.m, req.r, req.rho, req.a_format)
        if key not in self._ws_cache:
            self._ws_cache[key] = self.lib.altgdmin_workspace_bytes(self._problem_for_size(req), self.params)
        return self._ws_cache[key]

    def footprint(self, req) -> int:
        return req.a_bytes() + 4 * req.q * req.m + 8 * req.q * req.n + self.workspace_bytes(req)

    def iteration_bytes(self, req) -> float:
        """Algorithmic HBM bytes of one GDmin iteration of the request (its form's A reads)."""
        return roofline.iteration_bytes(req.n, req.q, req.m, req.r, req.rho, 3,
                                        mixed=req.a_format != "f32" and self.bf16_mixed)

    # -- lifecycle
    def start(self, req):
        torch, lib = self.torch, self.lib
        fut = self._truth.pop(req.idx, None)
        Xt_host, sv2 = fut.result() if fut is not None else self._make_truth(req)
        with torch.cuda.stream(self.init_stream):
            Xt = Xt_host.to(self.device, non_blocking=True)
            shape = (req.q, req.n, req.lda)
            if req.a_format == "f32":
                A, A_lo = torch.empty(shape, dtype=torch.float32, device=self.device), None
            else:
                A = torch.empty(shape, dtype=torch.int16, device=self.device)
                A_lo = torch.empty(shape, dtype=torch.int16, device=self.device)
            Y = torch.empty((req.q, req.m), dtype=torch.float32, device=self.device)
            lib.altgdmin_op_make_a(req.a_seed, self.table, req.q, req.n, req.m, A, A_lo)
            prob = lib.make_problem(A, Y, req.r, req.rho, A_lo=A_lo, m=req.m)
            lib.altgdmin_op_measure(prob, Xt, Y)
            ws = torch.empty(self.workspace_bytes(req), dtype=torch.uint8, device=self.device)
            h = lib.altgdmin_init(prob, self._params(req), ws)
            ready = torch.cuda.Event()
            ready.record(self.init_stream)
        # the step stream reads these too: the allocator must not reuse them before it is done
        for t in (Xt, A, A_lo, Y, ws):
            if t is not None:
                t.record_stream(self.step_stream)
        return dict(req=req, A=A, A_lo=A_lo, Y=Y, Xt=Xt, Xt_host=Xt_host, ws=ws, prob=prob, h=h, sv2=sv2,
                    ready=ready)

    def step(self, jobs, iters: int) -> None:
        torch = self.torch
        hs = [j["h"] for j in jobs]
        with torch.cuda.stream(self.step_stream):
            for j in jobs:   # a newly admitted job: its initialisation first
                ev = j.pop("ready", None)
                if ev is not None:
                    self.step_stream.wait_event(ev)
            need = self.lib.altgdmin_group_bytes(hs)
            if self.group_ws is None or self.group_ws.numel() < need:
                self.group_ws = torch.empty(max(need, 1 << 20), dtype=torch.uint8, device=self.device)
            self.lib.altgdmin_step_many(hs, iters, self.group_ws)

    def poll(self, jobs):
        """(iterations, residual, error flags) of every job, with one synchronisation."""
        with self.torch.cuda.stream(self.step_stream):
            reps = self.lib.altgdmin_status_many([j["h"] for j in jobs])
        return [(int(st["iterations"]), float(st["resid"]), int(st["error_flags"])) for st in reps]

    def finish(self, job):
        """(error against X*, {"eta_m_sigma2": eta m sigma_max(B*)^2}) of a retired job."""
        torch, req = self.torch, job["req"]
        with torch.cuda.stream(self.step_stream):
            U = torch.empty((req.n, req.r), dtype=torch.float32, device=self.device)
            Bt = torch.empty((req.q, req.r), dtype=torch.float32, device=self.device)
            rho = max(req.rho, 1)
            Si = torch.zeros((req.q, rho), dtype=torch.int32, device=self.device)
            Sv = torch.zeros((req.q, rho), dtype=torch.float32, device=self.device)
            self.lib.altgdmin_get(job["h"], U, Bt, Si if req.rho else None, Sv if req.rho else None)
            # error of the consistent pair in FP64 (measurement harness, not the method)
            Xt = Bt.double() @ U.double().T
            if req.rho:
                Xt.scatter_add_(1, Si.long(), Sv.double())
            err = float(torch.linalg.norm(Xt - job["Xt"]) / torch.linalg.norm(job["Xt"]))
            eta = self.lib.altgdmin_status(job["h"])["eta"]
        diag = eta * req.m * job["sv2"][1]
        self.release(job)
        return err, {"eta_m_sigma2": diag}

    def step_diagnostic(self, job) -> float:
        """eta m sigma_max(B_t)^2 from the iterate's B_t (an estimate of B*); above 2 the
        fixed step is too long (Gaussian A_k, E[A_k^T A_k] = m I)."""
        req = job["req"]
        with self.torch.cuda.stream(self.step_stream):
            Bt = self.torch.empty((req.q, req.r), dtype=self.torch.float32, device=self.device)
            self.lib.altgdmin_get(job["h"], None, Bt)
            eta = self.lib.altgdmin_status(job["h"])["eta"]
        sv = np.linalg.svd(Bt.double().cpu().numpy(), compute_uv=False)
        return float(eta * req.m * sv[0] ** 2)

    def release(self, job) -> None:
        """Destroy the handle and drop the job's device buffers (cancellation)."""
        ready = job.get("ready")
        if ready is not None:   # never stepped: its initialisation may still be running
            ready.synchronize()
        if job.get("h") is not None:
            self.lib.altgdmin_destroy(job["h"])
        job.clear()

    def forget(self, req) -> None:
        """Drop the host-side payload prepared for a request that will not run."""
        fut = self._truth.pop(req.idx, None)
        if fut is not None:
            fut.cancel()


def calibrate_rate(executor, requests, budget_bytes: int, poll_every: int = 10, tol: float = 1e-7,
                   max_iters: int = 300, max_active: Optional[int] = None, **policy) -> float:
    """Closed-loop throughput (all requests present at t = 0), in solves/s.  With
    max_active = 1 the requests are solved one after the other (no batching).
    `policy`: the Scheduler's retirement and retry arguments."""
    reqs = [dataclasses.replace(r, arrival=0.0) for r in requests]
    rep = Scheduler(executor, budget_bytes, poll_every, tol, max_iters, max_active=max_active, **policy).run(reqs)
    return rep.summary()["solves_per_s"]


def load_sweep(executor, requests, saturated: float, loads: Sequence[float], budget_bytes: int, seed: int,
               poll_every: int = 10, tol: float = 1e-7, max_iters: int = 300,
               clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
               log=None, **policy) -> Dict[str, dict]:
    """The same requests under seeded Poisson arrivals at each load x the closed-loop
    throughput `saturated`; per load: the rate, solves/s, p50 / p99 latency and the
    converged fraction."""
    out = {}
    for ld in loads:
        rate = ld * saturated
        arr = inst.poisson_arrivals(len(requests), rate, seed)
        reqs = [dataclasses.replace(r, arrival=float(a)) for r, a in zip(requests, arr)]
        s = Scheduler(executor, budget_bytes, poll_every, tol, max_iters, clock=clock, sleep=sleep,
                      **policy).run(reqs).summary()
        out[f"{ld:g}"] = {"arrival_rate_per_s": rate, "solves_per_s": s["solves_per_s"],
                          "p50_latency_s": s["p50_latency_s"], "p99_latency_s": s["p99_latency_s"],
                          "converged_fraction": s["converged_fraction"], "error_violations": s["error_violations"]}
        if log:
            log(f"load {ld:g}: arrivals {rate:.2f}/s, {s['solves_per_s']:.2f} solves/s, "
                f"p50 {s['p50_latency_s']:.3f} s, p99 {s['p99_latency_s']:.3f} s")
    return out


def serve(count: int = 512, seed: int = 231103828, budget_gib: float = 32.0, load: float = 0.8,
          rate: Optional[float] = None, poll_every: int = 10, tol: float = 1e-7, max_iters: int = 300,
          calibration_count: Optional[int] = None, sequential: bool = True, bf16_mixed: bool = True,
          sweep: Sequence[float] = (), log=None, retry_step_limit: Optional[float] = 2.0) -> dict:
    """Serve `count` seeded requests on the GPU and return the summary.

    Without an explicit `rate`, the arrival rate is `load` times the closed-loop
    throughput of the first `calibration_count` requests (default: all of them);
    `sweep` adds runs at those other multiples of it.  A request that diverges or
    stalls with a step diagnostic above retry_step_limit is retried once with the
    step scaled to a diagnostic of 1 (None: no retries).
    """
    policy = {"retry_step_limit": retry_step_limit}
    ex = GpuExecutor(tol=tol, max_iters=max_iters, bf16_mixed=bf16_mixed)
    reqs = inst.serving_requests(count, seed)
    budget = int(budget_gib * 2**30)
    sat = None
    if rate is None:
        cal = reqs[: calibration_count or count]
        sat = calibrate_rate(ex, cal, budget, poll_every, tol, max_iters, **policy)
        rate = load * sat
        if log:
            log(f"closed-loop throughput {sat:.2f} solves/s over {len(cal)} requests; arrival rate {rate:.2f}/s")
    arr = inst.poisson_arrivals(count, rate, seed)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    rep = Scheduler(ex, budget, poll_every, tol, max_iters, **policy).run(reqs)
    out = rep.summary()
    out.update({"arrival_rate_per_s": rate, "closed_loop_solves_per_s": sat, "load": load if sat else None,
                "tol_resid": tol, "max_iters": max_iters, "poll_every": poll_every, "seed": seed,
                "bf16_form": "mixed" if bf16_mixed else "hi+lo", "retry_step_limit": retry_step_limit})
    if sequential and sat:
        # the same requests solved one at a time through the same executor (no batching)
        seq = calibrate_rate(ex, reqs[: calibration_count or count], budget, poll_every, tol, max_iters, max_active=1,
                             **policy)
        out["sequential_solves_per_s"] = seq
        out["batching_speedup"] = sat / seq if seq > 0 else None
        if log:
            log(f"one request at a time: {seq:.2f} solves/s (batching speedup {sat / seq:.2f}x)")
    if sweep and sat:
        out["load_sweep"] = load_sweep(ex, reqs, sat, sweep, budget, seed, poll_every, tol, max_iters, log=log,
                                       **policy)
    return out
