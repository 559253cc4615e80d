"""Host logic of the serving loop: request draws, arrivals, and the scheduler
driven by a mock executor on a virtual clock (no GPU)."""
import dataclasses

import numpy as np
import pytest

from paper_2311_03824_amd import instances as inst
from paper_2311_03824_amd.serve import Scheduler, load_sweep


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class MockExecutor:
    """Each request converges after `conv_at[idx]` iterations (never if None);
    a round of `iters` iterations costs `cost` virtual seconds per active job."""

    def __init__(self, clock, conv_at, cost=1e-3, fp=None):
        self.clock, self.conv_at, self.cost = clock, conv_at, cost
        self.fp = fp or (lambda r: r.a_bytes())
        self.in_use = 0
        self.max_in_use = 0
        self.admit_order = []
        self.rounds = []

    def footprint(self, req):
        return self.fp(req)

    def start(self, req):
        self.in_use += self.fp(req)
        self.max_in_use = max(self.max_in_use, self.in_use)
        self.admit_order.append(req.idx)
        return {"req": req, "it": 0}

    def step(self, jobs, iters):
        self.rounds.append(len(jobs))
        for j in jobs:
            j["it"] += iters
        self.clock.t += self.cost * len(jobs)

    def poll(self, jobs):
        out = []
        for j in jobs:
            c = self.conv_at[j["req"].idx]
            resid = 1e-9 if (c is not None and j["it"] >= c) else 1e-3
            out.append((j["it"], resid))
        return out

    def finish(self, job):
        self.in_use -= self.fp(job["req"])
        return 1e-9


def _reqs(count=40, seed=5):
    return inst.serving_requests(count, seed)


def test_request_sizes_follow_the_laws():
    rs = inst.serving_requests(2000, 11)
    a = np.array([[r.n, r.q, r.m, r.r, r.rho] for r in rs], dtype=float)
    n, q, m, r, rho = a.T
    assert n.min() >= 256 and n.max() <= 2048 and q.min() >= 128 and q.max() <= 1024
    assert r.min() >= 2 and r.max() <= 16
    assert np.all(m >= np.floor(0.3 * n)) and np.all(m <= np.ceil(0.5 * n))
    assert np.all(rho >= np.floor(0.01 * n)) and np.all(rho <= np.ceil(0.05 * n))
    # log-uniform: the median of log n sits mid-way between log 256 and log 2048
    assert abs(np.median(np.log(n)) - 0.5 * (np.log(256) + np.log(2048))) < 0.1
    assert [x.a_format for x in rs[:4]] == ["f32", "bf16x2", "f32", "bf16x2"]
    again = inst.serving_requests(2000, 11)
    assert [dataclasses.astuple(x) for x in again] == [dataclasses.astuple(x) for x in rs]


def test_poisson_arrivals_rate():
    t = inst.poisson_arrivals(20000, rate=50.0, seed=3)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 50.0) < 0.05 / 50.0
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05     # exponential: CV = 1


def test_request_truth_structure():
    req = inst.ServeRequest(idx=0, n=300, q=50, m=100, r=3, rho=7, a_format="f32", seed=9)
    t = inst.request_truth(req)
    U, B, supp, vals, Xt = t["U_star"], t["B_star"], t["supp"], t["vals"], t["Xt"]
    assert np.allclose(U.T @ U, np.eye(3), atol=1e-13)
    assert supp.shape == (50, 7) and np.all(np.diff(supp, axis=1) > 0)
    S = Xt - (U @ B).T
    nz = np.abs(S) > 0
    assert np.all(nz.sum(axis=1) == 7)
    assert np.array_equal(np.sort(np.nonzero(nz)[1].reshape(50, 7), axis=1), supp)
    assert np.allclose(S[np.arange(50)[:, None], supp], vals, rtol=0, atol=1e-12)


def test_scheduler_completes_everything_within_budget():
    clk = Clock()
    reqs = _reqs()
    for i, r in enumerate(reqs):
        r.arrival = 0.01 * i
    conv = {r.idx: 10 * (1 + r.idx % 5) for r in reqs}
    budget = 8 * 2**30
    ex = MockExecutor(clk, conv)
    rep = Scheduler(ex, budget, poll_every=10, tol=1e-7, max_iters=300, clock=clk, sleep=clk.sleep).run(reqs)
    s = rep.summary()
    assert s["completed"] + s["rejected"] == len(reqs)
    big = [r.idx for r in reqs if r.a_bytes() > budget]
    assert s["rejected"] == len(big)
    assert ex.max_in_use <= budget and rep.peak_bytes <= budget
    for o in rep.outcomes:
        if o.rejected:
            assert o.idx in big
            continue
        assert o.converged and o.iterations == conv[o.idx]
        assert o.done >= o.admitted >= o.arrival
    # FIFO: admission order is arrival order (ties by index), skipping rejected requests
    expect = [r.idx for r in sorted(reqs, key=lambda r: (r.arrival, r.idx)) if r.idx not in big]
    assert ex.admit_order == expect


def test_scheduler_caps_iterations_and_reports_non_convergence():
    clk = Clock()
    reqs = _reqs(6)
    conv = {r.idx: (None if r.idx == 2 else 20) for r in reqs}
    ex = MockExecutor(clk, conv)
    rep = Scheduler(ex, 1 << 50, poll_every=7, tol=1e-7, max_iters=50, clock=clk, sleep=clk.sleep,
                    stall_polls=0).run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert not o[2].converged and o[2].iterations == 56          # first poll at or past the cap
    assert all(o[i].converged and o[i].iterations == 21 for i in o if i != 2)
    assert rep.summary()["converged_fraction"] == pytest.approx(5 / 6)


def test_scheduler_waits_for_arrivals():
    clk = Clock()
    reqs = _reqs(3)
    for r, a in zip(reqs, [0.0, 5.0, 9.0]):
        r.arrival = a
    ex = MockExecutor(clk, {r.idx: 10 for r in reqs})
    rep = Scheduler(ex, 1 << 50, poll_every=10, clock=clk, sleep=clk.sleep).run(reqs)
    adm = {o.idx: o.admitted for o in rep.outcomes}
    assert adm[1] >= 5.0 and adm[2] >= 9.0
    assert rep.rounds == 3 and ex.rounds == [1, 1, 1]


def test_scheduler_batches_concurrent_requests():
    clk = Clock()
    reqs = _reqs(8)
    ex = MockExecutor(clk, {r.idx: 30 for r in reqs})
    rep = Scheduler(ex, 1 << 50, poll_every=10, clock=clk, sleep=clk.sleep).run(reqs)
    assert ex.rounds == [8, 8, 8]
    assert rep.summary()["solves_per_s"] > 0


def test_scheduler_rejects_bad_arguments():
    with pytest.raises(ValueError):
        Scheduler(None, 1, poll_every=0)


def test_scheduler_one_at_a_time():
    clk = Clock()
    reqs = _reqs(5)
    ex = MockExecutor(clk, {r.idx: 20 for r in reqs})
    rep = Scheduler(ex, 1 << 50, poll_every=10, clock=clk, sleep=clk.sleep, max_active=1).run(reqs)
    assert ex.rounds == [1] * 10 and ex.max_in_use == max(r.a_bytes() for r in reqs)
    assert rep.summary()["completed"] == 5


def test_load_sweep_runs_each_load_on_the_same_requests():
    clk = Clock()
    reqs = _reqs(12)
    ex = MockExecutor(clk, {r.idx: 20 for r in reqs}, cost=0.01)
    sw = load_sweep(ex, reqs, saturated=50.0, loads=(0.5, 1.2), budget_bytes=1 << 50, seed=9,
                    clock=clk, sleep=clk.sleep)
    assert list(sw) == ["0.5", "1.2"]
    assert sw["0.5"]["arrival_rate_per_s"] == pytest.approx(25.0)
    assert sw["1.2"]["arrival_rate_per_s"] == pytest.approx(60.0)
    for v in sw.values():
        assert v["converged_fraction"] == 1.0 and v["error_violations"] == 0
        assert 0.0 < v["p50_latency_s"] <= v["p99_latency_s"]
    # the caller's requests keep their own arrival times
    assert all(r.arrival == 0.0 for r in reqs)


def test_requests_with_error_flags_are_retired_at_once_and_counted():
    """A job whose kernels report an error flag is retired after the round that
    raised it (not run to max_iters), counted as not converged and as a violation."""
    clock = Clock()

    class Flagging(MockExecutor):
        def poll(self, jobs):
            out = super().poll(jobs)
            return [(it, res, 1 if j["req"].idx == 2 else 0) for (it, res), j in zip(out, jobs)]

    ex = Flagging(clock, {i: None for i in range(4)} | {0: 30, 1: 30, 3: 30})
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(4)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-7, max_iters=300,
                    clock=clock, sleep=clock.sleep).run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert o[2].error_flags == 1 and not o[2].converged and o[2].iterations == 10
    assert all(o[i].converged and o[i].iterations == 30 for i in (0, 1, 3))
    s = rep.summary()
    assert s["retired_with_error_flags"] == 1 and s["not_converged"] == 1
    assert s["converged_solves_per_s"] < s["solves_per_s"]


def test_unconverged_requests_count_as_error_violations():
    clock = Clock()

    class BadFinish(MockExecutor):
        def finish(self, job):
            super().finish(job)
            return 1e-9 if self.conv_at[job["req"].idx] is not None else 0.5

    ex = BadFinish(clock, {0: 20, 1: None})
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(2)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-7, max_iters=50,
                    clock=clock, sleep=clock.sleep).run(reqs)
    s = rep.summary()
    assert s["not_converged"] == 1 and s["max_error_not_converged"] == 0.5
    assert s["error_violations"] == 1


class Releasing(MockExecutor):
    """Counts releases apart from finishes (a cancelled job is released, not finished)."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.released, self.finished = [], []

    def release(self, job):
        self.in_use -= self.fp(job["req"])
        self.released.append(job["req"].idx)

    def finish(self, job):
        self.finished.append(job["req"].idx)
        return super().finish(job)


def test_cancel_drops_waiting_and_releases_active_requests():
    """cancel(idx) before the run drops a request that never starts; cancel during
    the run releases an admitted job before the next round and returns its
    footprint to the budget; the rest complete as usual."""
    clock = Clock()
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(5)]
    sched = None

    class CancelMid(Releasing):
        def step(self, jobs, iters):
            super().step(jobs, iters)
            if len(self.rounds) == 2:
                sched.cancel(1)       # an active request, after two rounds
                sched.cancel(99)      # unknown: ignored

    ex = CancelMid(clock, {i: 40 for i in range(5)} | {1: None})
    sched = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-7, max_iters=300,
                      clock=clock, sleep=clock.sleep)
    sched.cancel(3)                   # waiting: never admitted
    rep = sched.run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert len(o) == 5
    assert o[3].cancelled and 3 not in ex.admit_order and o[3].iterations == 0
    assert o[1].cancelled and o[1].iterations == 20 and np.isnan(o[1].error)
    assert ex.released == [1] and 1 not in ex.finished and 3 not in ex.finished
    assert ex.rounds == [4, 4, 3, 3]                 # request 1 is gone from the third round on
    assert all(o[i].converged and not o[i].cancelled for i in (0, 2, 4))
    assert ex.in_use == 0
    s = rep.summary()
    assert s["cancelled"] == 2 and s["completed"] == 3 and s["rejected"] == 0
    assert s["converged_fraction"] == 1.0 and s["error_violations"] == 0


def test_cancel_from_another_thread():
    import threading

    clock = Clock()
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(3)]
    started = threading.Event()
    sched = None

    def canceller():
        started.wait(10)
        sched.cancel(0)

    th = threading.Thread(target=canceller)

    class Signal(Releasing):
        def step(self, jobs, iters):
            super().step(jobs, iters)
            if len(self.rounds) == 1:
                started.set()
                th.join(10)

    ex = Signal(clock, {0: None, 1: 30, 2: 30})
    sched = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, clock=clock, sleep=clock.sleep)
    th.start()
    rep = sched.run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert o[0].cancelled and o[0].iterations == 10 and ex.released == [0]
    assert o[1].converged and o[2].converged


def test_cancelling_the_last_request_ends_the_run():
    clock = Clock()
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(1)]
    sched = None

    class CancelFirst(Releasing):
        def step(self, jobs, iters):
            super().step(jobs, iters)
            sched.cancel(0)

    ex = CancelFirst(clock, {0: None})
    sched = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, max_iters=10**6, clock=clock, sleep=clock.sleep)
    rep = sched.run(reqs)
    assert rep.outcomes[0].cancelled and ex.rounds == [1] and ex.in_use == 0


class Trajectory(MockExecutor):
    """Residual of request idx at its p-th poll: traj[idx](p)."""

    def __init__(self, clock, traj):
        super().__init__(clock, {i: None for i in traj})
        self.traj = traj
        self.polls = {}

    def poll(self, jobs):
        out = []
        for j in jobs:
            i = j["req"].idx
            p = self.polls.get(i, 0) + 1
            self.polls[i] = p
            out.append((j["it"], self.traj[i](p)))
        return out


def test_diverging_requests_are_retired():
    """A residual that rises by more than diverge_rise at diverge_polls polls in a row
    retires the request as diverged; one that rises only below diverge_floor, or
    rises and falls again, runs to the cap; a NaN residual retires at once."""
    clock = Clock()
    traj = {
        0: lambda p: 1e-3 * 1.5 ** p,                          # grows: rises at polls 2, 3, 4
        1: lambda p: 1e-8 * 1.5 ** p,                          # grows, but below the floor up to poll 12
        2: lambda p: 1e-3 * (1.5 if p % 3 else 0.5),           # two rises, then a fall, repeating
        3: lambda p: float("nan") if p == 2 else 1e-3,
        4: lambda p: 1e-3 * 1.005 ** p,                        # rises by less than 1 %
    }
    ex = Trajectory(clock, traj)
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(5)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-12, max_iters=100, stall_polls=0,
                    clock=clock, sleep=clock.sleep).run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert o[0].diverged and o[0].iterations == 40 and not o[0].converged
    assert o[3].diverged and o[3].iterations == 20
    for i in (1, 2, 4):
        assert not o[i].diverged and o[i].iterations == 100
    s = rep.summary()
    assert s["diverged"] == 2 and s["completed"] == 5 and s["not_converged"] == 5


def test_divergence_check_can_be_switched_off():
    clock = Clock()
    ex = Trajectory(clock, {0: lambda p: 1e-3 * 2.0 ** p, 1: lambda p: float("inf")})
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(2)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-12, max_iters=60, diverge_polls=0,
                    stall_polls=0, clock=clock, sleep=clock.sleep).run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert not o[0].diverged and o[0].iterations == 60
    assert o[1].diverged and o[1].iterations == 10        # a non-finite residual always ends the request
    with pytest.raises(ValueError):
        Scheduler(None, 1, diverge_polls=-1)


def test_stalled_requests_are_retired():
    """A residual that reaches no new minimum (by 1 %) for stall_polls polls retires the
    request: as stalled above diverge_floor (a flat residual, and an oscillation whose
    polls see one phase only), as at_floor below it (the rounding floor); a slow but
    steady decrease runs on."""
    clock = Clock()
    traj = {
        0: lambda p: 3e-2,                                     # flat
        1: lambda p: 3e-2 * (1.0 if p % 2 else 0.9),           # oscillates: best at poll 2, then never beaten
        2: lambda p: 1e-2 * 0.98 ** p,                         # 2 % per poll: keeps going
        3: lambda p: 1e-6,                                     # flat below the floor
    }
    ex = Trajectory(clock, traj)
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(4)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-12, max_iters=200, stall_polls=6,
                    clock=clock, sleep=clock.sleep).run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert o[0].stalled and o[0].iterations == 70            # best at poll 1, six polls without a new one
    assert o[1].stalled and o[1].iterations == 80            # best at poll 2
    assert not o[2].stalled and o[2].iterations == 200
    assert not o[3].stalled and o[3].at_floor and o[3].iterations == 70
    s = rep.summary()
    assert s["stalled"] == 2 and s["at_floor"] == 1 and s["not_converged"] == 4
    assert {d["idx"]: d["why"] for d in s["not_converged_detail"]} == {0: "stalled", 1: "stalled", 2: "iteration cap",
                                                                      3: "at floor"}


class StepSensitive(MockExecutor):
    """Requests with an odd index start with a step diagnostic of 3 (too long): they
    oscillate until the step is scaled below 2 / 3 of the original; every request with a
    diagnostic below 2 converges after 30 iterations, except index 2, which stalls
    whatever its step (a failure the retry cannot mend)."""

    def __init__(self, clock):
        super().__init__(clock, {})
        self.started = []

    def _diag(self, req):
        return (3.0 if req.idx % 2 else 0.8) * req.eta_scale

    def start(self, req):
        self.started.append((req.idx, req.eta_scale))
        return super().start(req)

    def poll(self, jobs):
        out = []
        for j in jobs:
            ok = self._diag(j["req"]) < 2.0 and j["req"].idx != 2
            out.append((j["it"], 1e-9 if ok and j["it"] >= 30 else (3e-2 if (j["it"] // 10) % 2 else 2e-2)))
        return out

    def step_diagnostic(self, job):
        return self._diag(job["req"])

    def finish(self, job):
        super().finish(job)
        return 1e-9, {"eta_m_sigma2": self._diag(job["req"])}


def test_too_long_steps_are_retried_with_a_shorter_step():
    clock = Clock()
    ex = StepSensitive(clock)
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(4)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, tol=1e-7, max_iters=300, stall_polls=4,
                    retry_step_limit=2.0, clock=clock, sleep=clock.sleep).run(reqs)
    o = {x.idx: x for x in rep.outcomes}
    assert len(o) == 4 and o[0].converged and o[0].attempts == 1
    assert o[1].converged and o[3].converged and o[1].attempts == 2 and o[3].attempts == 2
    assert o[1].iterations == 30 and o[1].eta_m_sigma2 == pytest.approx(1.0)    # scaled by 1 / 3
    assert (1, pytest.approx(1 / 3)) in ex.started and (3, pytest.approx(1 / 3)) in ex.started
    # index 2 stalls with a diagnostic of 0.8: not a long step, so no retry
    assert o[2].stalled and o[2].attempts == 1 and o[2].step_diag == pytest.approx(0.8)
    assert ex.in_use == 0
    s = rep.summary()
    assert s["retried"] == 2 and s["converged_after_retry"] == 2 and s["stalled"] == 1
    # without retries the odd requests end as stalled too
    ex2 = StepSensitive(Clock())
    rep2 = Scheduler(ex2, budget_bytes=1 << 50, poll_every=10, tol=1e-7, max_iters=300, stall_polls=4,
                     clock=ex2.clock, sleep=ex2.clock.sleep).run(reqs)
    s2 = rep2.summary()
    assert s2["stalled"] == 3 and s2["converged_fraction"] == 0.25 and s2["retried"] == 0
    with pytest.raises(ValueError):
        Scheduler(None, 1, retry_step_limit=0.5)


def test_iteration_bytes_enter_the_summary():
    """The summary's iteration_GBps is the sum over completed requests of iterations x
    bytes per iteration, over the makespan."""
    clock = Clock()

    class Sized(MockExecutor):
        def iteration_bytes(self, req):
            return 1e9 * (1 + req.idx)

    ex = Sized(clock, {0: 20, 1: 30}, cost=0.01)
    reqs = [dataclasses.replace(r, arrival=0.0) for r in _reqs(2)]
    rep = Scheduler(ex, budget_bytes=1 << 50, poll_every=10, clock=clock, sleep=clock.sleep).run(reqs)
    s = rep.summary()
    want = (20 * 1e9 + 30 * 2e9) / rep.makespan / 1e9
    assert s["iteration_GBps"] == pytest.approx(want)
    assert {o.idx: o.bytes_per_iteration for o in rep.outcomes} == {0: 1e9, 1: 2e9}


def test_iteration_bytes_formula():
    from paper_2311_03824_amd import roofline
    # the benchmark workload: 6.743e9 B in the column kernel, 1.6 GB + P_k, G^{-1} in A_k U
    assert roofline.column_kernel_bytes(1000, 1000, 400, 10, 50, 3) == 6743248000.0
    assert roofline.au_kernel_bytes(1000, 1000, 400, 10) == 1000 * (1.6e6 + 16000 + 800) + 40000
    full = roofline.iteration_bytes(1000, 1000, 400, 10, 50)
    mixed = roofline.iteration_bytes(1000, 1000, 400, 10, 50, mixed=True)
    assert full == pytest.approx(8.36e9, rel=1e-3) and mixed == pytest.approx(5.16e9, rel=2e-3)


def test_fourier_column_flops_formula():
    from paper_2311_03824_amd import roofline
    # a 2 x 2 frame: one transform is 5 * 4 * log2(4) = 40 flops; the Gram 8 m r^2
    assert roofline.fourier_column_flops(2, 2, 1, 3, 1, transforms=1) == 40.0 + 24.0
    # the benchmark's 64 frames of 96 x 96, m = 1536, r = 6: 8 transforms each
    f = roofline.fourier_column_flops(96, 96, 64, 1536, 6)
    assert f == pytest.approx(64 * (8 * 5 * 9216 * 13.1699 + 8 * 1536 * 36), rel=1e-5)
