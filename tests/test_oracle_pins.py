"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one oracle function against something other than itself:
a closed form, an invariant, brute force on a tiny input, a special case that
reduces to a textbook result, or the paper's exact-recovery claims.
"""
import itertools

import numpy as np
import pytest

from oracle import altgdmin_oracle as O
from paper_2311_03824_amd import instances as I


def _small(n=40, q=12, m=24, r=3, rho=3, seed=7, **kw):
    inst = I.make_instance(n, q, m, r, rho, seed, **kw)
    return inst, inst.A64(), inst.Y64


# ---------------------------------------------------------------- HardThreshold

def _ht_brute(v, rho):
    """The unique rho-subset T with |v_j| > |v_l| or (equal and j < l) for all j in T, l not in T."""
    n = len(v)
    found = []
    for T in itertools.combinations(range(n), rho):
        Ts = set(T)
        ok = all((abs(v[j]) > abs(v[l])) or (abs(v[j]) == abs(v[l]) and j < l)
                 for j in Ts for l in range(n) if l not in Ts)
        if ok:
            found.append(T)
    assert len(found) == 1
    return np.array(found[0], dtype=np.int64)


def test_hard_threshold_brute_force_random():
    rng = np.random.default_rng(1)
    for trial in range(200):
        n = rng.integers(1, 9)
        rho = rng.integers(0, n + 1)
        # small integer values force many magnitude ties, with both signs and zeros
        v = rng.integers(-3, 4, size=n).astype(np.float64)
        dense, idx = O.hard_threshold(v[None, :], rho)
        T = _ht_brute(v, rho)
        assert np.array_equal(idx[0], T)
        ref = np.zeros(n)
        ref[T] = v[T]
        assert np.array_equal(dense[0], ref)


def test_hard_threshold_hand_ties():
    v = np.array([[1.0, -3.0, 3.0, 0.0, -1.0, 2.0]])
    assert O.hard_threshold(v, 1)[1].tolist() == [[1]]           # -3 and 3 tie: lower index
    assert O.hard_threshold(v, 2)[1].tolist() == [[1, 2]]
    assert O.hard_threshold(v, 4)[1].tolist() == [[0, 1, 2, 5]]  # 1 and -1 tie at |1|: index 0
    assert O.hard_threshold(v, 6)[1].tolist() == [[0, 1, 2, 3, 4, 5]]
    z = np.array([[0.0, -0.0, 0.0]])
    assert O.hard_threshold(z, 2)[1].tolist() == [[0, 1]]        # -0 equals +0
    with pytest.raises(ValueError):
        O.hard_threshold(np.array([[1.0, np.nan]]), 1)


# ---------------------------------------------------------------- projector and LS

def test_projector_invariants():
    inst, A, Y = _small()
    U = O.qr_pos(np.random.default_rng(3).standard_normal((inst.n, inst.r)))[0]
    P, G = O.projector_parts(A, U)
    V = np.random.default_rng(4).standard_normal((inst.q, inst.m))
    PV = O.project_out(P, G, V)
    assert np.allclose(O.project_out(P, G, PV), PV, atol=1e-12)          # idempotent
    PtPV = np.matmul(P.transpose(0, 2, 1), PV[:, :, None])[:, :, 0]
    assert np.abs(PtPV).max() < 1e-11                                   # annihilates range(P)
    for k in range(inst.q):                                             # = I - Q Q^T
        Qk, _ = np.linalg.qr(P[k])
        assert np.allclose(PV[k], V[k] - Qk @ (Qk.T @ V[k]), atol=1e-12)


def test_ls_b_normal_equations_and_lstsq():
    inst, A, Y = _small()
    U = O.qr_pos(np.random.default_rng(5).standard_normal((inst.n, inst.r)))[0]
    S = inst.S_star.T.copy()
    B = O.ls_b(A, U, Y, S)
    for k in range(inst.q):
        AU = A[k] @ U
        rhs = Y[k] - A[k] @ S[k]
        assert np.abs(AU.T @ (rhs - AU @ B[k])).max() < 1e-10 * np.abs(AU).sum()
        ref = np.linalg.lstsq(AU, rhs, rcond=None)[0]
        assert np.allclose(B[k], ref, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- IHT

def test_iht_step_is_line_search_minimiser():
    """mu must minimise ||M(s - a g_T) - z||^2 over a (brute-force 1-D search)."""
    inst, A, Y = _small(q=5)
    Mop = lambda S: O.apply_A(A, S)
    MTop = lambda V: O.apply_AT(A, V)
    trace = []
    S1, idx1 = O.iht(Y, Mop, MTop, inst.rho, 1, np.zeros((inst.q, inst.n)), trace=trace)
    S2, idx2 = O.iht(Y, Mop, MTop, inst.rho, 1, S1, idx1, trace=trace)
    G, mu = trace[1]["G"], trace[1]["mu"]
    for k in range(inst.q):
        gT = np.zeros(inst.n)
        gT[idx1[k]] = G[k, idx1[k]]
        f = lambda a: np.sum((A[k] @ (S1[k] - a * gT) - Y[k]) ** 2)
        lo, hi = 0.0, 10 * mu[k] + 1.0
        for _ in range(200):                                # golden-section search
            a1 = hi - (hi - lo) / 1.618033988749895
            a2 = lo + (hi - lo) / 1.618033988749895
            if f(a1) < f(a2):
                hi = a2
            else:
                lo = a1
        assert abs((lo + hi) / 2 - mu[k]) <= 1e-7 * mu[k]


def test_iht_recovers_sparse_vectors_exactly():
    """L* = 0 and m >> rho log(n/rho): IHT from 0 is plain compressive sensing and recovers s*."""
    inst = I.make_instance(120, 20, 60, 1, 4, 11)
    A = inst.A64()
    Y = O.apply_A(A, inst.S_star.T)
    S, idx = O.iht(Y, lambda S: O.apply_A(A, S), lambda V: O.apply_AT(A, V), 4, 40,
                   np.zeros((20, 120)))
    assert np.array_equal(idx, inst.supp)
    assert np.abs(S - inst.S_star.T).max() < 1e-9 * np.abs(inst.S_star).max()


def test_iht_scale_invariance():
    inst, A, Y = _small(q=6)
    run = lambda c: O.iht(c * Y, lambda S: O.apply_A(c * A, S), lambda V: O.apply_AT(c * A, V),
                          inst.rho, 5, np.zeros((inst.q, inst.n)))
    S1, i1 = run(1.0)
    S2, i2 = run(8.0)        # (M, z) -> (cM, cz) leaves the IHT iterates unchanged
    assert np.array_equal(i1, i2)
    assert np.allclose(S1, S2, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rule", ["literal", "full"])
def test_other_step_readings_fail_exact_recovery(rule):
    """Negative test: the printed unsquared ratio diverges; the unrestricted ratio stalls."""
    inst = I.make_instance(100, 100, 40, 1, 2, 231103824, s_zero=False)
    A = inst.A64()
    Y = O.apply_A(A, inst.S_star.T)
    S, idx = O.iht(Y, lambda S: O.apply_A(A, S), lambda V: O.apply_AT(A, V), 2, 30,
                   np.zeros((100, 100)), mu_rule=rule)
    assert np.mean([set(idx[k]) == set(inst.supp[k]) for k in range(100)]) < 0.9
    S, idx = O.iht(Y, lambda S: O.apply_A(A, S), lambda V: O.apply_AT(A, V), 2, 30,
                   np.zeros((100, 100)))
    assert np.array_equal(idx, inst.supp)


# ---------------------------------------------------------------- gradient, QR, eta

def test_grad_U_central_differences():
    inst, A, Y = _small(n=20, q=6, m=12, r=2, rho=2)
    rng = np.random.default_rng(9)
    U = rng.standard_normal((inst.n, inst.r))
    B = rng.standard_normal((inst.q, inst.r))
    S = inst.S_star.T
    g = O.grad_U(A, U, B, S, Y)
    h = 1e-5
    fd = np.zeros_like(U)
    for j in range(inst.n):
        for c in range(inst.r):
            E = np.zeros_like(U)
            E[j, c] = h
            fd[j, c] = (O.cost(A, U + E, B, S, Y) - O.cost(A, U - E, B, S, Y)) / (2 * h)
    assert np.abs(g - fd / 2).max() <= 1e-6 * np.abs(g).max()     # grad = (1/2) df/dU


def test_qr_positive_diagonal():
    M = np.random.default_rng(2).standard_normal((50, 6))
    Q, R = O.qr_pos(M)
    assert np.abs(Q.T @ Q - np.eye(6)).max() < 1e-14
    assert np.allclose(Q @ R, M, atol=1e-13)
    assert np.allclose(R, np.triu(R)) and (np.diag(R) > 0).all()


def test_eta_normalises_first_step():
    inst, A, Y = _small(n=60, q=30, m=30, r=2, rho=2)
    st = O.initialise(A, Y, inst.r, inst.rho)
    rec = {}
    st1 = O.gdmin_iteration(A, Y, st, inst.rho, record=rec)
    assert abs(np.linalg.svd(st1.eta * rec["grad"], compute_uv=False)[0] - O.ETA_C) < 1e-12
    assert abs(O.spectral_norm(rec["grad"]) - np.linalg.svd(rec["grad"], compute_uv=False)[0]) < 1e-9


def test_spectral_init_matches_eigenvectors():
    L0 = np.random.default_rng(4).standard_normal((30, 20))
    U0 = O.spectral_init(L0, 3)
    w, V = np.linalg.eigh(L0 @ L0.T)
    assert O.subspace_distance(V[:, -3:], U0) < 1e-10


# ---------------------------------------------------------------- whole algorithm

def test_exact_recovery_n100():
    inst = I.make_workload("gauss_n100_q100_m40_r2_rho2")
    st, hist = O.solve(inst.A64(), inst.Y64, inst.r, inst.rho, t_max=300,
                       X_star=inst.X_star, err_tol=1e-10)
    assert hist[-1] < 1e-10 and len(hist) <= 300
    assert np.array_equal(st.idx, inst.supp)


def test_low_rank_only_reduces_to_altgdmin_lr():
    """S* = 0 with rho = 0: S stays 0 and the method is AltGDmin for LRCCS; exact recovery."""
    inst = I.make_instance(100, 80, 80, 2, 0, 21, s_zero=True)
    st, hist = O.solve(inst.A64(), inst.Y64, 2, 0, t_max=200, X_star=inst.X_star, err_tol=1e-10)
    assert np.all(st.S == 0)
    assert hist[-1] < 1e-10


def test_measurement_scaling_equivariance():
    inst = I.make_workload("gauss_n100_q100_m40_r2_rho2")
    A = inst.A64()
    st1, _ = O.solve(A, inst.Y64, 2, 2, t_max=15)
    st2, _ = O.solve(A, 4.0 * inst.Y64, 2, 2, t_max=15)
    assert np.allclose(O.estimate(st2), 4.0 * O.estimate(st1), rtol=1e-9, atol=1e-9)


def test_rotation_invariance_of_U0():
    inst = I.make_workload("gauss_n100_q100_m40_r2_rho2")
    A = inst.A64()
    st0 = O.initialise(A, inst.Y64, 2, 2)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    st1, _ = O.solve(A, inst.Y64, 2, 2, t_max=10, U0=st0.U)
    st2, _ = O.solve(A, inst.Y64, 2, 2, t_max=10, U0=st0.U @ R)
    assert np.allclose(O.estimate(st1), O.estimate(st2), rtol=1e-9, atol=1e-9)


def test_column_permutation_equivariance():
    inst = I.make_workload("gauss_n100_q100_m40_r2_rho2")
    A = inst.A64()
    perm = np.random.default_rng(0).permutation(inst.q)
    st1, _ = O.solve(A, inst.Y64, 2, 2, t_max=10)
    st2, _ = O.solve(A[perm], inst.Y64[perm], 2, 2, t_max=10)
    assert np.allclose(O.estimate(st2), O.estimate(st1)[:, perm], rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- mixed-precision variant
# A_t (here the bf16 hi plane of A) replaces A in the transposed products and the
# IHT step length only; the products that form residuals keep A.


def _truth_state(inst):
    return O.State(U=inst.U_star.copy(), S=inst.S_star.T.copy(), idx=inst.supp.copy(), eta=0.1)


def test_mixed_variant_with_A_t_equal_A_is_the_plain_method():
    inst, A, Y = _small(bf16_planes=True)
    a, ha = O.solve(A, Y, inst.r, inst.rho, t_max=5, X_star=inst.X_star)
    b, hb = O.solve(A, Y, inst.r, inst.rho, t_max=5, X_star=inst.X_star, A_t=A)
    assert np.array_equal(a.U, b.U) and np.array_equal(a.idx, b.idx) and ha == hb


def test_mixed_variant_keeps_the_exact_fixed_point():
    """Noise-free data: from (U*, S*) one mixed iteration returns X* to rounding, because
    every residual is formed with the exact A; taking the hi plane for the residuals as
    well (the planted mistake) moves the iterate by about the bf16 relative error."""
    inst = I.make_instance(120, 30, 60, 3, 4, 17, bf16_planes=True)
    A, Y, Ahi = inst.A64(), inst.Y64, inst.A64_hi()
    assert 1e-4 < np.abs(A - Ahi).max() / np.abs(A).max() < 1e-2      # the planes differ
    st = O.gdmin_iteration(A, Y, _truth_state(inst), inst.rho, A_t=Ahi)
    assert O.rel_error(O.estimate(st), inst.X_star) < 1e-12
    assert O.subspace_distance(st.U, inst.U_star) < 1e-12
    assert np.array_equal(st.idx, inst.supp)
    bad = O.gdmin_iteration(Ahi, Y, _truth_state(inst), inst.rho)
    assert O.rel_error(O.estimate(bad), inst.X_star) > 1e-5


def test_mixed_variant_recovers_exactly_n100():
    """The paper's exact-recovery size with A_t = bf16 hi plane: Error < 1e-10 as in the
    plain method, within a few more iterations; the hi plane alone stalls far above."""
    inst = I.make_workload("gauss_n100_q100_m40_r2_rho2", bf16_planes=True)
    A, Y, Ahi = inst.A64(), inst.Y64, inst.A64_hi()
    _, h_plain = O.solve(A, Y, inst.r, inst.rho, t_max=300, X_star=inst.X_star, err_tol=1e-10)
    st, h_mix = O.solve(A, Y, inst.r, inst.rho, t_max=300, X_star=inst.X_star, err_tol=1e-10, A_t=Ahi)
    assert h_mix[-1] < 1e-10 and len(h_mix) <= len(h_plain) + 10
    assert np.array_equal(st.idx, inst.supp)
    _, h_hi = O.solve(Ahi, Y, inst.r, inst.rho, t_max=len(h_mix), X_star=inst.X_star)
    assert min(h_hi) > 1e-5


# ---------------------------------------------------------------- back-projection (Sec. 2.3)

def test_backprojection_is_minus_half_the_gradient_in_s():
    """l_k = A_k^T (y_k - A_k s_k) is -1/2 the gradient of c(s) = ||y_k - A_k s||^2 at
    s = s_k: central differences of c, built from the forward products alone.  Dropping
    the A_k s_k term, a sign or a transpose fails this."""
    inst, A, Y = _small(n=25, q=5, m=15, r=2, rho=3, seed=31)
    rng = np.random.default_rng(8)
    S = inst.S_star.T + rng.standard_normal((inst.q, inst.n))    # a dense s, away from the truth
    L0 = O.backprojection(A, Y, S)                               # n x q
    h = 1e-4
    for k in range(inst.q):
        c = lambda s: float(np.sum((Y[k] - A[k] @ s) ** 2))
        fd = np.empty(inst.n)
        for j in range(inst.n):
            e = np.zeros(inst.n)
            e[j] = h
            fd[j] = (c(S[k] + e) - c(S[k] - e)) / (2 * h)
        assert np.abs(L0[:, k] + fd / 2).max() <= 1e-7 * np.abs(fd).max()
    # at the truth (noise free) every l_k lies in the row space of A_k applied to L*
    L0_star = O.backprojection(A, Y, inst.S_star.T)
    want = O.apply_AT(A, O.apply_A(A, (inst.U_star @ inst.B_star).T)).T
    assert np.allclose(L0_star, want, rtol=1e-10, atol=1e-10 * np.abs(want).max())


# ---------------------------------------------------------------- Fig. 1 (Sec. 3)

@pytest.mark.slow
def test_fig1_exact_recovery_claim():
    """Sec. 3, Fig. 1: Gaussian A_k, n = q = 600, m = 80, r = 4, S1 values U[-6, 6],
    threshold budget rho_max = 7, T_max = 200; the paper reports the error reaching
    about 1e-15 in most cases.  With the restricted normalised step the oracle goes
    below 1e-10 within the 200 iterations (rho = 2); with the unrestricted step it is
    still above 1e-2 after 40 iterations, where the restricted one is below 1e-4."""
    inst = I.make_instance(600, 600, 80, 4, 2, 231103900, s_dist="uniform", s_scale=6.0)
    A, Y = inst.A64(), inst.Y64
    st, hist = O.solve(A, Y, 4, 7, t_max=200, X_star=inst.X_star, err_tol=1e-10)
    assert hist[-1] < 1e-10 and len(hist) <= 200
    assert hist[39] < 1e-4
    _, hist_full = O.solve(A, Y, 4, 7, t_max=40, X_star=inst.X_star, mu_rule="full")
    assert min(hist_full) > 1e-2


# ---------------------------------------------------------------- the fixed step size (Sec. 2.6)

def _first_eta_and_errors(inst, c, iters):
    A, Y = inst.A64(), inst.Y64
    st = O.initialise(A, Y, inst.r, inst.rho)
    errs = []
    for _ in range(iters):
        st = O.gdmin_iteration(A, Y, st, inst.rho, eta_c=c)
        errs.append(O.rel_error(O.estimate(st), inst.X_star))
    return st.eta, np.array(errs)


def test_fixed_step_contracts_by_one_minus_eta_m_sigma_squared():
    """Near the solution, with B refitted by least squares and E[A_k^T A_k] = m I,
    one projected GD step scales the error of U along the i-th direction by about
    1 - eta m sigma_i(B*)^2 (the gradient of Sec. 2.1 without its factor 2).  The
    fixed eta = c / ||grad_U f(U_0, B_1, S_1)||_2 is proportional to 1 / SD(U_0),
    so with the paper's c = 0.14 a start that is already accurate (here SD(U_0) =
    0.06, from q = 3000 columns) gives eta m sigma^2 near 3 > 2: the error doubles
    per step instead of shrinking.  With c = 0.05 the same start gives about 1.1
    and the error falls by the predicted factor.  On the paper's own shapes (the
    n = q = 100 instance below; also the Fig. 1 shape and n = q = 1000, m = 400)
    eta m sigma^2 lies in [0.5, 0.92]."""
    inst = I.make_instance(60, 3000, 60, 2, 1, 5)
    sv = np.linalg.svd(inst.B_star, compute_uv=False)
    m = inst.m
    eta, e = _first_eta_and_errors(inst, 0.14, 4)
    lo, hi = eta * m * sv[-1] ** 2, eta * m * sv[0] ** 2
    assert 2.5 < lo <= hi < 3.5
    ratios = e[1:] / e[:-1]
    assert np.all(ratios > 1.5)                                        # diverges
    assert ratios[0] == pytest.approx(lo - 1.0, rel=0.15)              # |1 - eta m sigma^2|, slowest mode
    eta, e = _first_eta_and_errors(inst, 0.05, 8)
    lo, hi = eta * m * sv[-1] ** 2, eta * m * sv[0] ** 2
    assert 0.9 < lo <= hi < 1.3
    ratios = e[1:] / e[:-1]
    assert np.all(ratios < 1.1 * max(abs(1 - lo), abs(1 - hi)))
    assert e[-1] < 1e-8
    paper = I.make_instance(100, 100, 40, 2, 2, 231103824)
    eta, _ = _first_eta_and_errors(paper, 0.14, 1)
    svp = np.linalg.svd(paper.B_star, compute_uv=False)
    assert 0.4 < eta * paper.m * svp[-1] ** 2 <= eta * paper.m * svp[0] ** 2 < 1.0


# ---------------------------------------------------------------- automatic rank (Sec. 2.6)

def _with_spectrum(n, q, sv, seed=0):
    rng = np.random.default_rng(seed)
    Uf = O.qr_pos(rng.standard_normal((n, len(sv))))[0]
    Vf = O.qr_pos(rng.standard_normal((q, len(sv))))[0]
    return Uf @ np.diag(sv) @ Vf.T


def test_rank_budget_is_a_tenth_of_the_smallest_size():
    assert O.rank_budget(600, 600, 80) == 8          # Fig. 1 and Fig. 2 shapes
    assert O.rank_budget(400, 400, 40) == 4          # Table 1, m = 40
    assert O.rank_budget(1000, 1000, 400) == 40
    assert O.rank_budget(30, 25, 9) == 1             # never below one


@pytest.mark.parametrize("r0,want", [(1, 1), (2, 2), (4, 3), (7, 5), (10, 7)])
def test_auto_rank_equal_singular_values(r0, want):
    """r0 equal singular values hold k / r0 of the energy after k of them, so the 65 %
    rule gives ceil(0.65 r0) (budget 10 at n = q = 200, m = 100)."""
    L0 = _with_spectrum(200, 200, np.full(r0, 3.0), seed=r0)
    r, sv = O.auto_rank(L0, 100)
    assert r == want and len(sv) == 10


def test_auto_rank_geometric_spectrum_and_budget():
    # sigma_i^2 = 2^-i: 50 % of the energy after one value, 75 % after two
    L0 = _with_spectrum(300, 200, np.sqrt(2.0 ** -np.arange(1, 16)), seed=3)
    assert O.auto_rank(L0, 150)[0] == 2
    # 30 equal values but a budget of 10: only the first 10 count, so ceil(6.5) = 7
    L0 = _with_spectrum(300, 200, np.ones(30), seed=4)
    assert O.auto_rank(L0, 100)[0] == 7
    # one dominant value: 1 regardless of the small ones
    L0 = _with_spectrum(300, 200, np.array([10.0, 1.0, 1.0, 1.0, 1.0]), seed=5)
    assert O.auto_rank(L0, 100)[0] == 1


def test_auto_rank_against_eigenvalues_and_invariances():
    """The singular values are the square roots of the eigenvalues of L_0^T L_0
    (a library eigen-solver); scaling, transposing and rotating L_0 keep r."""
    rng = np.random.default_rng(12)
    L0 = _with_spectrum(250, 180, np.array([9.0, 7.0, 6.0, 2.0, 1.5, 1.0]), seed=6)
    L0 += 0.05 * rng.standard_normal(L0.shape)
    r, sv = O.auto_rank(L0, 120)
    ev = np.sort(np.linalg.eigvalsh(L0.T @ L0))[::-1][: len(sv)]
    assert np.allclose(sv ** 2, ev, rtol=1e-10)
    cum = np.cumsum(ev)
    assert cum[r - 1] >= 0.65 * cum[-1] and (r == 1 or cum[r - 2] < 0.65 * cum[-1])
    Q = O.qr_pos(rng.standard_normal((250, 250)))[0]
    assert O.auto_rank(7.5 * L0, 120)[0] == r
    assert O.auto_rank(L0.T, 120)[0] == r
    assert O.auto_rank(Q @ L0, 120)[0] == r


def test_auto_rank_initialisation_uses_the_chosen_rank():
    """r = None in the initialisation: U_0 gets auto_rank(L_0) columns."""
    inst = I.make_instance(200, 150, 100, 3, 2, 41)
    A, Y = inst.A64(), inst.Y64
    st = O.initialise(A, Y, None, inst.rho)
    S, _ = O.init_sparse(A, Y, inst.rho)
    r, _ = O.auto_rank(O.backprojection(A, Y, S), inst.m)
    assert st.U.shape == (inst.n, r)
