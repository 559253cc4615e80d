"""Pins of the complex (partial Fourier) oracle against the DFT definition,
invariants, brute force and exact recovery -- never against itself."""
import numpy as np
import pytest

from oracle import fourier_oracle as F
from paper_2311_03824_amd import instances as I


def _op(N1, N2, q, m, seed=0):
    rng = np.random.default_rng(seed)
    mask = np.sort(np.stack([rng.choice(N1 * N2, m, replace=False) for _ in range(q)]), axis=1)
    return F.PartialFourier(N1, N2, mask)


def _cn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_operator_matches_dft_definition():
    """Sign, normalisation and row-major flattening against the explicit DFT sum."""
    op = _op(4, 6, 3, 10)
    rng = np.random.default_rng(1)
    X = _cn(rng, (3, 24))
    V = _cn(rng, (3, 10))
    for k in range(3):
        # written out term by term, independent of numpy.fft and of op.dense
        ref = np.zeros(10, np.complex128)
        for i, u in enumerate(op.mask[k]):
            u1, u2 = divmod(int(u), 6)
            for j in range(24):
                j1, j2 = divmod(j, 6)
                ref[i] += X[k, j] * np.exp(-2j * np.pi * (u1 * j1 / 4 + u2 * j2 / 6)) / np.sqrt(24)
        assert np.allclose(op.apply(X)[k], ref, atol=1e-12)
        D = op.dense(k)
        assert np.allclose(D @ X[k], ref, atol=1e-12)
        assert np.allclose(op.adjoint(V)[k], D.conj().T @ V[k], atol=1e-12)


def test_rows_are_orthonormal():
    op = _op(8, 12, 5, 30, seed=2)
    rng = np.random.default_rng(3)
    V = _cn(rng, (5, 30))
    assert np.allclose(op.apply(op.adjoint(V)), V, atol=1e-12)          # A A^H = I
    assert np.allclose(np.linalg.norm(op.adjoint(V), axis=1), np.linalg.norm(V, axis=1))
    U = np.linalg.qr(_cn(rng, (96, 3)))[0]
    P = op.apply_U(U)
    for c in range(3):
        assert np.allclose(P[:, :, c], op.apply(np.tile(U[:, c], (5, 1))), atol=1e-12)


def test_hard_threshold_brute_force_and_ties():
    rng = np.random.default_rng(4)
    V = _cn(rng, (50, 40))
    V[0, ::2] = V[0, 1::2] * 1j            # equal moduli in pairs: lower index wins
    V[1] = np.exp(1j * rng.uniform(0, 2 * np.pi, 40))   # all moduli 1 (up to rounding)
    V[2] = 0
    for rho in (0, 1, 7, 40):
        dense, idx = F.hard_threshold(V, rho)
        for k in range(50):
            a = np.abs(V[k])
            order = np.lexsort((np.arange(40), -a))[:rho]
            assert np.array_equal(idx[k], np.sort(order))
            keep = np.zeros(40, bool)
            keep[order] = True
            assert np.array_equal(dense[k][keep], V[k][keep]) and not dense[k][~keep].any()
    # hand-built ties: moduli 1, 1, 1, 0.5, 1 -> the lowest indices among equal moduli win
    v = np.array([[1.0, 1j, -1.0, 0.5, -1j]])
    for rho, want in [(1, [0]), (2, [0, 1]), (3, [0, 1, 2]), (4, [0, 1, 2, 4]), (5, [0, 1, 2, 3, 4])]:
        assert F.hard_threshold(v, rho)[1][0].tolist() == want


def test_iht_step_is_the_line_search_minimiser():
    """mu minimises ||M (s - alpha g_T) - z||^2 over real alpha (brute force)."""
    op = _op(8, 8, 4, 40, seed=5)
    rng = np.random.default_rng(6)
    z = _cn(rng, (4, 40))
    S0 = np.zeros((4, 64), np.complex128)
    trace = []
    F.iht(z, op.apply, op.adjoint, 5, 1, S0, trace=trace)
    G = trace[0]["G"]
    _, T = F.hard_threshold(G, 5)
    for k in range(4):
        gT = np.zeros(64, np.complex128)
        gT[T[k]] = G[k, T[k]]
        alphas = np.linspace(0, 2 * trace[0]["mu"][k], 200001)
        Mg = op.apply(np.tile(gT, (4, 1)))[k]
        vals = [np.linalg.norm(-a * Mg - z[k]) for a in alphas[::1000]]
        fine = alphas[np.argmin([np.linalg.norm(-a * Mg - z[k]) for a in alphas])]
        assert abs(fine - trace[0]["mu"][k]) <= 2e-5 * trace[0]["mu"][k]
        assert min(vals) >= np.linalg.norm(-trace[0]["mu"][k] * Mg - z[k]) - 1e-12


def test_iht_recovers_sparse_frames_exactly():
    """Compressive-sensing special case: partial Fourier, m >> rho log n, IHT from 0."""
    q, N, m, rho = 6, 16, 100, 6
    op = _op(N, N, q, m, seed=7)
    rng = np.random.default_rng(8)
    S = np.zeros((q, N * N), np.complex128)
    for k in range(q):
        S[k, rng.choice(N * N, rho, replace=False)] = _cn(rng, rho) * 3
    S_rec, _ = F.iht(op.apply(S), op.apply, op.adjoint, rho, 300, np.zeros_like(S))
    assert np.linalg.norm(S_rec - S) <= 1e-10 * np.linalg.norm(S)


def test_projector_and_ls():
    op = _op(8, 10, 3, 30, seed=9)
    rng = np.random.default_rng(10)
    U = np.linalg.qr(_cn(rng, (80, 4)))[0]
    P, G = F.projector_parts(op, U)
    V = _cn(rng, (3, 30))
    PV = F.project_out(P, G, V)
    assert np.allclose(F.project_out(P, G, PV), PV, atol=1e-12)                  # idempotent
    assert np.allclose(np.matmul(P.conj().transpose(0, 2, 1), PV[:, :, None]), 0, atol=1e-12)
    for k in range(3):
        Q = np.linalg.qr(P[k])[0]
        assert np.allclose(PV[k], V[k] - Q @ (Q.conj().T @ V[k]), atol=1e-12)
        b = F.pinv_apply(P, G, V)[k]
        assert np.allclose(b, np.linalg.lstsq(P[k], V[k], rcond=None)[0], atol=1e-12)


def test_gradient_central_differences():
    """d/de f(U + e E) at 0 equals 2 Re <E, grad> for the Wirtinger gradient without the factor 2."""
    op = _op(6, 8, 5, 20, seed=11)
    rng = np.random.default_rng(12)
    U, B, S, Y = _cn(rng, (48, 3)), _cn(rng, (5, 3)), _cn(rng, (5, 48)) * 0.1, _cn(rng, (5, 20))
    grad = F.grad_U(op, U, B, S, Y)
    for _ in range(3):
        E = _cn(rng, (48, 3))
        h = 1e-6
        fd = (F.cost(op, U + h * E, B, S, Y) - F.cost(op, U - h * E, B, S, Y)) / (2 * h)
        assert fd == pytest.approx(2 * np.real(np.vdot(E, grad)), rel=1e-6)


def test_qr_positive_real_diagonal():
    rng = np.random.default_rng(13)
    M = _cn(rng, (50, 5))
    Q, R = F.qr_pos(M)
    assert np.allclose(Q.conj().T @ Q, np.eye(5), atol=1e-14)
    assert np.allclose(Q @ R, M, atol=1e-12)
    assert np.allclose(np.tril(R, -1), 0)
    d = np.diag(R)
    assert np.all(d.real > 0) and np.allclose(d.imag, 0)


def test_eta_normalises_first_step():
    inst = I.make_fourier_instance(16, 16, 24, 120, 2, 4, seed=14)
    op = F.PartialFourier(16, 16, inst.mask)
    st = F.initialise(op, inst.Y, 2, 4)
    rec = {}
    F.gdmin_iteration(op, inst.Y, st, 4, record=rec)
    assert rec["eta"] * F.spectral_norm(rec["grad"]) == pytest.approx(0.14, rel=1e-12)


def test_spectral_init_left_singular_vectors():
    rng = np.random.default_rng(15)
    L0 = _cn(rng, (60, 20))
    U0 = F.spectral_init(L0, 3)
    w, V = np.linalg.eigh(L0 @ L0.conj().T)
    top = V[:, np.argsort(w)[::-1][:3]]
    assert F.subspace_distance(U0, top) < 1e-10


def test_exact_recovery_small_frames():
    """L + S recovery from partial Fourier data in FP64 (16 x 16 frames)."""
    inst = I.make_fourier_instance(16, 16, 32, 128, 2, 5, seed=7)
    op = F.PartialFourier(16, 16, inst.mask)
    st, hist = F.solve(op, inst.Y, 2, 5, t_max=300, X_star=inst.X_star, err_tol=1e-10)
    assert hist[-1] < 1e-10


def test_low_rank_only_reduces_to_altgdmin_lr():
    """rho = 0: S stays zero and the low-rank part is recovered."""
    inst = I.make_fourier_instance(16, 16, 32, 128, 2, 0, seed=16)
    op = F.PartialFourier(16, 16, inst.mask)
    st, hist = F.solve(op, inst.Y, 2, 0, t_max=300, X_star=inst.X_star, err_tol=1e-10)
    assert not st.S.any() and hist[-1] < 1e-10


def test_phase_equivariance():
    """Y -> e^{i theta} Y gives X -> e^{i theta} X (a dropped conjugate breaks this)."""
    inst = I.make_fourier_instance(12, 12, 16, 80, 2, 3, seed=17)
    op = F.PartialFourier(12, 12, inst.mask)
    c = np.exp(0.7j) * 2.5
    st1, _ = F.solve(op, inst.Y, 2, 3, t_max=15)
    st2, _ = F.solve(op, c * inst.Y, 2, 3, t_max=15, U0=None)
    X1, X2 = F.estimate(st1), F.estimate(st2)
    assert np.linalg.norm(X2 - c * X1) <= 1e-9 * np.linalg.norm(c * X1)


def test_generator_measurements_are_exact():
    inst = I.make_fourier_instance(10, 12, 5, 40, 2, 3, seed=18)
    op = F.PartialFourier(10, 12, inst.mask)
    assert np.allclose(op.apply(inst.X_star.T), inst.Y, atol=1e-12)
    assert np.all(np.diff(inst.mask, axis=1) > 0)
    assert np.allclose(inst.U_star.conj().T @ inst.U_star, np.eye(2), atol=1e-13)


def test_backprojection_is_minus_half_the_gradient_in_s():
    """Complex l_k = A_k^H (y_k - A_k s_k): for c(s) = ||y_k - A_k s||^2, the central
    differences of c along Re s_j and Im s_j are -2 Re l_k[j] and -2 Im l_k[j].
    Only the forward operator (pinned to the DFT definition) builds c."""
    op = _op(4, 5, 3, 9, seed=21)
    rng = np.random.default_rng(22)
    Y = _cn(rng, (3, 9))
    S = _cn(rng, (3, 20))
    L0 = F.backprojection(op, Y, S)                  # n x q
    h = 1e-4
    for k in range(3):
        def c(s):
            Sk = np.zeros((3, 20), np.complex128)
            Sk[k] = s
            return float(np.sum(np.abs(Y[k] - op.apply(Sk)[k]) ** 2))
        for j in range(20):
            e = np.zeros(20, np.complex128)
            e[j] = h
            d_re = (c(S[k] + e) - c(S[k] - e)) / (2 * h)
            d_im = (c(S[k] + 1j * e) - c(S[k] - 1j * e)) / (2 * h)
            assert abs(L0[j, k].real + d_re / 2) <= 1e-7 * max(1.0, abs(d_re))
            assert abs(L0[j, k].imag + d_im / 2) <= 1e-7 * max(1.0, abs(d_im))


def test_auto_rank_complex_equal_values():
    """Complex L_0 with r0 equal singular values: ceil(0.65 r0), as in the real form."""
    rng = np.random.default_rng(5)
    for r0, want in [(1, 1), (4, 3), (6, 4)]:
        Uf = np.linalg.qr(_cn(rng, (300, r0)))[0]
        Vf = np.linalg.qr(_cn(rng, (120, r0)))[0]
        L0 = Uf @ Vf.conj().T * 2.0
        r, sv = F.auto_rank(L0, 200)
        assert r == want and len(sv) == 12
