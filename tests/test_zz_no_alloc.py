"""The allocation-free entry point altgdmin_op_subspace_noalloc against
altgdmin_op_subspace (the same kernels with a caller scratch buffer): bitwise
equal U and iteration counts on two calls in a row, the second with smaller
sizes (the static scratch keeps the first call's contents), and the subspace
against the oracle's exact SVD."""
import numpy as np
import pytest

from oracle import altgdmin_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return _t


def _l0(n, q, r, seed):
    rng = np.random.default_rng(seed)
    Uf = O.qr_pos(rng.standard_normal((n, r + 4)))[0]
    Vf = O.qr_pos(rng.standard_normal((q, r + 4)))[0]
    sv = np.concatenate([np.linspace(40.0, 12.0, r), [4.0, 3.0, 2.0, 1.0]])
    return np.ascontiguousarray((Uf @ np.diag(sv) @ Vf.T).T, dtype=np.float32), Uf[:, :r]


def test_noalloc_subspace_equals_the_scratch_entry_point(lib, torch):
    for n, q, r, seed in ((1500, 900, 12, 1), (300, 200, 3, 2)):     # second call smaller
        L0t_h, U_true = _l0(n, q, r, seed)
        L0t = torch.from_numpy(L0t_h).cuda()
        Us = torch.from_numpy(np.random.default_rng(seed + 7).standard_normal((n, r)).astype(np.float32)).cuda()
        Ua = torch.zeros((n, r), dtype=torch.float32, device="cuda")
        Ub = torch.full((n, r), float("nan"), dtype=torch.float32, device="cuda")
        ia = torch.zeros(1, dtype=torch.int32, device="cuda")
        ib = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        lib.altgdmin_op_subspace(L0t, r, Us, 200, 1e-7, Ua, ia)
        lib.altgdmin_op_subspace_noalloc(L0t, r, Us, 200, 1e-7, Ub, ib)
        torch.cuda.synchronize()
        print(f"n={n} q={q} r={r}: {int(ia.item())} iterations")
        assert np.array_equal(Ua.cpu().numpy(), Ub.cpu().numpy())
        assert ia.item() == ib.item() and 1 <= ia.item() < 200
        U_ref = O.spectral_init(L0t_h.T.astype(np.float64), r)
        assert O.subspace_distance(U_ref, Ub.cpu().numpy().astype(np.float64)) <= 1e-5
        assert O.subspace_distance(U_true, U_ref) <= 1e-6


def test_noalloc_rejects_sizes_beyond_the_static_scratch(lib, torch):
    L0t = torch.zeros((2, 300000), dtype=torch.float32, device="cuda")
    U = torch.zeros((300000, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.AltGDminError) as e:
        lib.altgdmin_op_subspace_noalloc(L0t, 16, None, 1, 1e-7, U)
    assert e.value.code == -2
