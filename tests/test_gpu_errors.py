"""Failure paths of the solve on the GPU, forced from the host (every kernel
still runs to its normal end; all loops in the kernels have fixed trip counts):

  * a NaN in the measurements reaches the HardThreshold selection; the kernels
    raise error bit 0 (and bit 1 once the non-finite gradient reaches the QR
    step, which then leaves U unchanged), the residual is NaN, `converged` stays
    0, and altgdmin_solve returns ALTGDMIN_ENONFINITE instead of a result (FP32
    plane, mixed BF16, partial Fourier);
  * a tolerance that cannot be reached exhausts t_max: altgdmin_solve returns
    the ALTGDMIN_ENOTCONV warning with the iterate of the last iteration in the
    outputs (the binding passes the warning through);
  * a problem's bad values do not leak into other problems stepped in the same
    batched launches (altgdmin_step_many).
"""
import numpy as np
import pytest

from paper_2311_03824_amd import instances as I

pytestmark = pytest.mark.gpu

SHAPE = dict(n=100, q=24, m=40, r=2, rho=2)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return _t


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _outputs(torch, n, q, r, rho):
    return (torch.zeros((n, r), dtype=torch.float32, device="cuda"),
            torch.zeros((q, r), dtype=torch.float32, device="cuda"),
            torch.zeros((q, rho), dtype=torch.int32, device="cuda"),
            torch.zeros((q, rho), dtype=torch.float32, device="cuda"))


def _problem(lib, torch, inst, form, Y32):
    Y = dev(torch, Y32)
    if form == "f32":
        A = dev(torch, inst.At)
        return lib.make_problem(A, Y, inst.r, inst.rho, m=inst.m), [A, Y], 0
    hi = dev(torch, inst.A_hi.view(np.int16))
    lo = dev(torch, inst.A_lo.view(np.int16))
    return lib.make_problem(hi, Y, inst.r, inst.rho, A_lo=lo, m=inst.m), [hi, lo, Y], lib.FLAG_BF16_MIXED


@pytest.mark.parametrize("form", ["f32", "bf16_mixed"])
def test_nan_in_measurements_is_reported(lib, torch, form):
    inst = I.make_instance(**SHAPE, seed=231103824, bf16_planes=(form != "f32"))
    Y32 = inst.Y32.copy()
    Y32[3, 5] = np.nan
    print(f"\ncase: NaN in y_3, {form}", flush=True)
    p, keep, flags = _problem(lib, torch, inst, form, Y32)
    par = lib.default_params(t_max=40, tol_resid=1e-7, poll_every=5, flags=flags)
    ws = torch.empty(lib.altgdmin_workspace_bytes(p, par), dtype=torch.uint8, device="cuda")
    outs = _outputs(torch, inst.n, inst.q, inst.r, inst.rho)
    with pytest.raises(lib.AltGDminError) as e:
        lib.altgdmin_solve(p, par, ws, *outs)
    assert e.value.code == lib.ALTGDMIN_ENONFINITE
    # the same through a handle: the flag is up after the initialisation already
    h = lib.altgdmin_init(p, par, ws)
    try:
        lib.altgdmin_step(h, 2)
        st = lib.altgdmin_status(h)
        assert st["error_flags"] & 1 and st["iterations"] == 2
        assert st["converged"] == 0 and np.isnan(st["resid"])
        # the failed QR steps left U as it was: finite, orthonormal
        U = torch.empty((inst.n, inst.r), dtype=torch.float32, device="cuda")
        lib.altgdmin_get(h, U)
        Uh = U.double().cpu().numpy()
        assert np.all(np.isfinite(Uh)) and np.abs(Uh.T @ Uh - np.eye(inst.r)).max() < 1e-5
    finally:
        lib.altgdmin_destroy(h)


def test_nan_in_fourier_measurements_is_reported(lib, torch):
    fi = I.make_fourier_instance(12, 12, 8, 60, 2, 3, 7)
    Y = fi.Y.copy()
    Y[2, 4] = np.nan
    print("\ncase: NaN in y_2, partial Fourier 12 x 12", flush=True)
    s = lib.FourierSolver(fi.mask, Y, 12, 12, 2, 3, lib.default_params(t_max=10)).init()
    try:
        s.step(3)
        st = s.status()
        assert st["error_flags"] & 1 and np.isnan(st["resid"]) and st["iterations"] == 3
    finally:
        s.close()


def test_tmax_exhaustion_returns_the_warning_and_the_last_iterate(lib, torch):
    inst = I.make_instance(**SHAPE, seed=231103824)
    print("\ncase: tol 1e-30, t_max 7", flush=True)
    p, keep, _ = _problem(lib, torch, inst, "f32", inst.Y32)
    par = lib.default_params(t_max=7, tol_resid=1e-30, poll_every=3)
    ws = torch.empty(lib.altgdmin_workspace_bytes(p, par), dtype=torch.uint8, device="cuda")
    U, Bt, Si, Sv = _outputs(torch, inst.n, inst.q, inst.r, inst.rho)
    rc, rep = lib.altgdmin_solve(p, par, ws, U, Bt, Si, Sv)
    assert rc == lib.ALTGDMIN_ENOTCONV
    assert rep["iterations"] == 7 and rep["converged"] == 0 and rep["error_flags"] == 0
    assert 0.0 < rep["resid"] < 0.1
    # the outputs hold the iterate of iteration 7: the same as stepping a handle 7 times
    h = lib.altgdmin_init(p, par, ws)
    try:
        lib.altgdmin_step(h, 7)
        U2, Bt2, Si2, Sv2 = _outputs(torch, inst.n, inst.q, inst.r, inst.rho)
        lib.altgdmin_get(h, U2, Bt2, Si2, Sv2)
        torch.cuda.synchronize()
        for a, b in ((U, U2), (Bt, Bt2), (Si, Si2), (Sv, Sv2)):
            assert torch.equal(a, b)
    finally:
        lib.altgdmin_destroy(h)
    Uh = U.double().cpu().numpy()
    assert np.abs(Uh.T @ Uh - np.eye(inst.r)).max() < 1e-5


def test_bad_problem_does_not_leak_into_its_batch(lib, torch):
    """Two problems stepped together by altgdmin_step_many, one with a NaN in y:
    the healthy one ends bitwise where it ends when stepped alone."""
    inst = I.make_instance(**SHAPE, seed=231103825)
    Ybad = inst.Y32.copy()
    Ybad[0, 0] = np.nan
    print("\ncase: step_many with one NaN problem", flush=True)
    par = lib.default_params(t_max=20)
    pg, kg, _ = _problem(lib, torch, inst, "f32", inst.Y32)
    pb, kb, _ = _problem(lib, torch, inst, "f32", Ybad)
    wsg = torch.empty(lib.altgdmin_workspace_bytes(pg, par), dtype=torch.uint8, device="cuda")
    wsb = torch.empty_like(wsg)
    wss = torch.empty_like(wsg)
    hg = lib.altgdmin_init(pg, par, wsg)
    hb = lib.altgdmin_init(pb, par, wsb)
    hs = lib.altgdmin_init(pg, par, wss)
    try:
        need = lib.altgdmin_group_bytes([hg, hb])
        gws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        lib.altgdmin_step_many([hg, hb], 10, gws)
        lib.altgdmin_step(hs, 10)
        reps = lib.altgdmin_status_many([hg, hb, hs])
        assert reps[0]["error_flags"] == 0 and reps[1]["error_flags"] & 1 and reps[2]["error_flags"] == 0
        got, solo = _outputs(torch, inst.n, inst.q, inst.r, inst.rho), _outputs(torch, inst.n, inst.q, inst.r, inst.rho)
        lib.altgdmin_get(hg, *got)
        lib.altgdmin_get(hs, *solo)
        torch.cuda.synchronize()
        for a, b in zip(got, solo):
            assert torch.equal(a, b)
    finally:
        for h in (hg, hb, hs):
            lib.altgdmin_destroy(h)
