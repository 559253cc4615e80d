"""GPU tests of the serving path: device-made instances against the host
generator, and a small mixed-size serving run (errors against X*, and the
batched result of one request equal to its solo result)."""
import dataclasses

import numpy as np
import pytest

from paper_2311_03824_amd import instances as inst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return torch


@pytest.mark.parametrize("q,n,m", [(3, 37, 29), (2, 130, 260), (1, 5, 1)])
def test_make_a_matches_host_generator(lib, torch_dev, q, n, m):
    torch = torch_dev
    lda = inst.round_up(m, 8)
    seed = 0x1234_5678_9ABC_DEF0 + m
    table = inst.normal_table()
    tab = torch.from_numpy(table).cuda()
    hi, lo, canon = inst.canonical_philox_A(seed, range(q), n, m, lda, table)
    A = torch.full((q, n, lda), float("nan"), dtype=torch.float32, device="cuda")
    lib.altgdmin_op_make_a(seed, tab, q, n, m, A)
    Ah = torch.full((q, n, lda), -1, dtype=torch.int16, device="cuda")
    Al = torch.full((q, n, lda), -1, dtype=torch.int16, device="cuda")
    lib.altgdmin_op_make_a(seed, tab, q, n, m, Ah, Al)
    torch.cuda.synchronize()
    got = A.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), canon.view(np.uint32))       # bit-exact, padding rows zero
    assert np.array_equal(Ah.cpu().numpy().view(np.uint16), hi)
    assert np.array_equal(Al.cpu().numpy().view(np.uint16), lo)


def _ulp_diff(a, b):
    ai = a.view(np.int32).astype(np.int64)
    bi = b.view(np.int32).astype(np.int64)
    return np.abs(ai - bi)


@pytest.mark.parametrize("fmt", ["f32", "bf16x2", "philox"])
def test_measure_matches_fp64_products(lib, torch_dev, fmt):
    torch = torch_dev
    q, n, m = 5, 300, 123
    lda = inst.round_up(m, 8)
    seed = 77
    table = inst.normal_table()
    tab = torch.from_numpy(table).cuda()
    rng = np.random.default_rng(1)
    Xt = rng.standard_normal((q, n)) * 3.0
    Xd = torch.from_numpy(Xt).cuda()
    Y = torch.full((q, m), float("nan"), dtype=torch.float32, device="cuda")
    if fmt == "philox":
        A_host = inst.philox_A(seed, range(q), n, m, lda, table)
        prob = lib.make_problem(None, Y, 2, 3, m=m, philox_seed=seed, normal_table=tab, n=n)
    else:
        hi, lo, A_host = inst.canonical_philox_A(seed, range(q), n, m, lda, table)
        if fmt == "f32":
            A = torch.from_numpy(A_host).cuda()
            prob = lib.make_problem(A, Y, 2, 3, m=m)
        else:
            A = torch.from_numpy(hi.view(np.int16)).cuda()
            A_lo = torch.from_numpy(lo.view(np.int16)).cuda()
            prob = lib.make_problem(A, Y, 2, 3, A_lo=A_lo, m=m)
    lib.altgdmin_op_measure(prob, Xd, Y)
    torch.cuda.synchronize()
    ref = np.einsum("kji,kj->ki", A_host[:, :, :m].astype(np.float64), Xt).astype(np.float32)
    got = Y.cpu().numpy()
    # FP64 sums in different orders agree to far below FP32 resolution; allow one
    # ulp for a sum that lands next to an FP32 rounding boundary
    assert _ulp_diff(got, ref).max() <= 1


def _small_requests(count, seed):
    return inst.serving_requests(count, seed, n_range=(256, 420), q_range=(128, 200), r_range=(2, 4))


def test_small_serving_run(lib, torch_dev):
    from paper_2311_03824_amd.serve import GpuExecutor, Scheduler
    reqs = _small_requests(6, 424242)
    for i, r in enumerate(reqs):
        r.arrival = 0.002 * i
    ex = GpuExecutor(tol=1e-7, max_iters=300)
    budget = 3 * max(ex.footprint(r) for r in reqs)          # forces queueing
    rep = Scheduler(ex, budget, poll_every=5, tol=1e-7, max_iters=300).run(reqs)
    s = rep.summary()
    print(s, [(o.idx, o.iterations, o.resid, o.error) for o in rep.outcomes])
    assert s["completed"] == 6 and s["rejected"] == 0
    assert s["converged_fraction"] == 1.0
    assert s["max_error_converged"] <= 1e-6
    assert rep.peak_bytes <= budget
    # the same request alone gives the same iterations and the same error, bit for bit
    solo = dataclasses.replace(reqs[3], arrival=0.0)
    rep1 = Scheduler(GpuExecutor(tol=1e-7, max_iters=300), budget, poll_every=5, tol=1e-7,
                     max_iters=300).run([solo])
    mixed = [o for o in rep.outcomes if o.idx == reqs[3].idx][0]
    assert rep1.outcomes[0].iterations == mixed.iterations
    assert rep1.outcomes[0].error == mixed.error


def test_too_long_step_is_caught_and_retried(lib, torch_dev):
    """A request whose initialisation is so accurate that the fixed step of Sec. 2.6 is
    too long (n = 128, q = 2048, m = 128, r = 2: eta m sigma_max(B*)^2 near 3, so the
    error grows and then oscillates) is retired as diverged or stalled; the retry, with
    the step scaled by the diagnostic read from the iterate, converges."""
    from paper_2311_03824_amd.serve import GpuExecutor, Scheduler
    req = inst.ServeRequest(idx=0, n=128, q=2048, m=128, r=2, rho=1, a_format="f32", seed=20231103)
    ex = GpuExecutor(tol=1e-7, max_iters=300)
    budget = 2 * ex.footprint(req)
    print("\ncase: one request, no retry", flush=True)
    rep = Scheduler(ex, budget, poll_every=10, tol=1e-7, max_iters=300).run([req])
    o = rep.outcomes[0]
    print(o, flush=True)
    assert not o.converged and (o.diverged or o.stalled) and o.eta_m_sigma2 > 2.0
    assert o.iterations < 300
    print("case: one request, retry when the step diagnostic exceeds 2", flush=True)
    rep = Scheduler(ex, budget, poll_every=10, tol=1e-7, max_iters=300, retry_step_limit=2.0).run([req])
    o = rep.outcomes[0]
    print(o, flush=True)
    # the retry scales the step by 1 / (eta m sigma_max(B_t)^2), B_t from the stalled iterate
    assert o.converged and o.attempts == 2 and 0.5 < o.eta_m_sigma2 < 1.5 and o.error <= 1e-6
