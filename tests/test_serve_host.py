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
    rep = Scheduler(ex, 1 << 50, poll_every=7, tol=1e-7, max_iters=50, clock=clk, sleep=clk.sleep).run(reqs)
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
