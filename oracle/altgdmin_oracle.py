"""FP64 CPU oracle of AltGDmin-LR+S.

Source: S. Babu, N. Vaswani, "A Fast Algorithm for Low Rank + Sparse column-wise
Compressive Sensing", arXiv 2311.03824.  Alg. 1 (altGDmin-L+S) and Alg. 2
(IHT), with the definitions of Sec. 1.1 (notation, pseudo-inverse), Sec. 2
(cost), Sec. 2.1 (gradient in U), Sec. 2.2 (decoupled minimisation over B and
S, eq. (bk_LS)), Sec. 2.3 (initialisation) and Sec. 2.6 (parameters).

TEST INFRASTRUCTURE.  This module is the correctness reference for the HIP
path.  Only tests/, the smoke check and the benchmark's CPU-baseline leg may
import it.  It imports nothing from the product package and shares no code with
it.  Everything is NumPy FP64, vectorised over the column index k but
otherwise written in the order the paper states it.

Arrays: A is (q, m, n) with A[k] = A_k; Y is (q, m) with Y[k] = y_k; S is kept
dense as (q, n) with S[k] = s_k; U is (n, r); B is returned as (q, r) with
B[k] = b_k (the transpose of the paper's r x q B).

Readings where the paper is garbled, ambiguous or silent (each is listed in the
design notes as well):
  * IHT step (Alg. 2): the normalised-IHT step of Blumensath and Davies,
    mu = ||g_T||^2 / ||M g_T||^2 with g = M^T (M s - z) restricted to the
    current support T.  The printed ratio of unsquared, unrestricted norms is
    not invariant to scaling (M, z) -> (cM, cz) and diverges; the unrestricted
    squared ratio stalls on wrong supports.  Both are kept as ``mu_rule``
    variants for negative tests only.
  * Factor 2 of the gradients is dropped, as in the paper's own grad_U.
  * ||grad_U f|| in eta is the induced 2-norm (Sec. 1.1 notation); eta is set
    once, inside iteration t = 1, from grad_U f(U_0, B_1, S_1) (Sec. 2.6).
  * QR: thin QR with a positive diagonal R (unique Q).
  * HardThreshold: exactly rho entries; larger |v| first, lower index on ties.
  * The b_k of the initialisation block is dead (overwritten in iteration 1
    before any use) and is skipped.
  * The output pairs U with the B and S fitted to it ("consistent pair").
  * mu = 0 when ||M g|| is 0 or not finite; eta = 0 when grad_U f = 0.
  * Automatic rank (Sec. 2.6): "energy" is the sum of squared singular values;
    r is the smallest k whose first k values reach 65 % of the energy of the
    first floor(min(n, q, m) / 10) (at least one).

Mixed-precision variant (not in the paper; an option of the GPU path whose
A_k is stored as a BF16 hi + lo pair): every function that takes ``A_t`` uses
it in place of A for the transposed products A_k^T v (the IHT gradient, h_k of
grad_U f, the back-projection L_0) and for the IHT step-length product M g_T,
while every product that forms a residual (A_k U, A_k s_k) keeps A.  With
A_t = A (the default) this is the paper's algorithm unchanged.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

ETA_C = 0.14     # step-size constant of Sec. 2.6
TAU0 = 10        # IHT iterations in the initialisation (Alg. 1, Sec. 2.6)
TAU = 3          # IHT iterations per GDmin iteration (Alg. 1, Sec. 2.6)
T_MAX = 200      # GDmin iterations (Sec. 2.6; Alg. 1 prints 120)
ENERGY = 0.65    # energy threshold of the automatic rank (Sec. 2.6)


# ---------------------------------------------------------------------------
# Helpers of Alg. 2
# ---------------------------------------------------------------------------

def hard_threshold(V: np.ndarray, rho: int):
    """HardThreshold(v, rho) of Alg. 2, row by row.

    Keeps the rho entries of largest magnitude of each row of V (q x n), the
    lower index winning a tie in magnitude; zeroes the rest.  Returns the dense
    result and the kept indices, ascending, as a (q, rho) int64 array.
    """
    V = np.asarray(V, dtype=np.float64)
    if np.isnan(V).any():
        raise ValueError("HardThreshold: NaN input")
    q, n = V.shape
    order = np.argsort(-np.abs(V), axis=1, kind="stable")   # stable: ties keep index order
    idx = np.sort(order[:, :rho], axis=1)
    out = np.zeros_like(V)
    rows = np.arange(q)[:, None]
    out[rows, idx] = V[rows, idx]
    return out, idx


def iht(z: np.ndarray, Mop: Callable, MTop: Callable, rho: int, tau: int,
        S0: np.ndarray, idx0: Optional[np.ndarray] = None, mu_rule: str = "support",
        trace: Optional[list] = None, Dop: Optional[Callable] = None):
    """IHT(z, M, rho, tau, s) of Alg. 2 for all columns at once.

    For t = 1..tau: gradient g of L(s) = ||M s - z||^2 (factor 2 dropped),
    step size mu, gradient step s - mu g, HardThreshold to rho entries.

    The step size is the normalised-IHT step of the IHT the paper builds on
    (Blumensath and Davies): mu = ||g_T||^2 / ||M g_T||^2, where g_T is g
    restricted to the support T kept by the previous HardThreshold (idx0 on
    entry), or, when there is none yet (s = 0), to the support of
    HardThreshold(g, rho).  It is the exact line-search minimiser of L along
    g_T.  mu_rule="full" uses all of g and mu_rule="literal" the printed ratio
    of unsquared norms; both are kept for negative tests only.

    Mop maps (q, n) -> (q, m) column by column; MTop maps (q, m) -> (q, n).
    Dop, if given, replaces Mop in the step-length product M g_T only (the
    mixed-precision variant); the residual M s - z always uses Mop.
    Returns the dense (q, n) result and its kept indices (q, rho), ascending.
    """
    S = np.array(S0, dtype=np.float64, copy=True)
    q = S.shape[0]
    rows = np.arange(q)[:, None]
    idx = None if idx0 is None else np.asarray(idx0, dtype=np.int64)
    for _ in range(tau):
        R = Mop(S) - z                      # M s - z
        G = MTop(R)                         # gradient w.r.t. s, without the factor 2
        if mu_rule == "support":
            T = idx if idx is not None else hard_threshold(G, rho)[1]
            D = np.zeros_like(G)
            D[rows, T] = G[rows, T]         # g restricted to T
        elif mu_rule in ("full", "literal"):
            D = G
        else:
            raise ValueError(mu_rule)
        W = (Dop or Mop)(D)                 # M * (restricted) gradient
        gg = np.einsum("kn,kn->k", D, D)
        ww = np.einsum("km,km->k", W, W)
        if mu_rule == "literal":
            gg, ww = np.sqrt(gg), np.sqrt(ww)
        ok = (ww > 0) & np.isfinite(ww) & np.isfinite(gg)
        mu = np.where(ok, gg / np.where(ok, ww, 1.0), 0.0)
        S, idx = hard_threshold(S - mu[:, None] * G, rho)
        if trace is not None:
            trace.append(dict(G=G, W=W, mu=mu, S=S, idx=idx))
    return S, idx


# ---------------------------------------------------------------------------
# Column-wise linear algebra (Sec. 2.2)
# ---------------------------------------------------------------------------

def apply_A(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """(q, n) -> (q, m): A_k x_k for every k."""
    return np.matmul(A, X[:, :, None])[:, :, 0]


def apply_AT(A: np.ndarray, V: np.ndarray) -> np.ndarray:
    """(q, m) -> (q, n): A_k^T v_k for every k."""
    return np.matmul(V[:, None, :], A)[:, 0, :]


def projector_parts(A: np.ndarray, U: np.ndarray):
    """P_k = A_k U and G_k = P_k^T P_k (the pieces of (A_k U)^dagger, Sec. 1.1)."""
    P = np.matmul(A, U)                               # (q, m, r)
    G = np.matmul(P.transpose(0, 2, 1), P)            # (q, r, r)
    return P, G


def pinv_apply(P: np.ndarray, G: np.ndarray, V: np.ndarray) -> np.ndarray:
    """(A_k U)^dagger v_k = (P_k^T P_k)^{-1} P_k^T v_k for every k, (q, m) -> (q, r)."""
    PtV = np.matmul(P.transpose(0, 2, 1), V[:, :, None])
    return np.linalg.solve(G, PtV)[:, :, 0]


def project_out(P: np.ndarray, G: np.ndarray, V: np.ndarray) -> np.ndarray:
    """v_k - A_k U (A_k U)^dagger v_k, the map that defines z_k and M_k in Sec. 2.2."""
    return V - np.matmul(P, pinv_apply(P, G, V)[:, :, None])[:, :, 0]


def ls_b(A: np.ndarray, U: np.ndarray, Y: np.ndarray, S: np.ndarray) -> np.ndarray:
    """eq. (bk_LS): b_k = (A_k U)^dagger (y_k - A_k s_k); returns (q, r)."""
    P, G = projector_parts(A, U)
    return pinv_apply(P, G, Y - apply_A(A, S))


def grad_U(A: np.ndarray, U: np.ndarray, B: np.ndarray, S: np.ndarray, Y: np.ndarray,
           A_t: Optional[np.ndarray] = None) -> np.ndarray:
    """Sec. 2.1: grad_U f = sum_k A_k^T (A_k (U b_k + s_k) - y_k) b_k^T, an (n, r) matrix."""
    X = B @ U.T + S                                    # rows are (U b_k + s_k)^T
    Rres = apply_A(A, X) - Y                           # r_k = A_k (U b_k + s_k) - y_k
    H = apply_AT(A if A_t is None else A_t, Rres)      # rows h_k^T = (A_k^T r_k)^T
    return H.T @ B


def cost(A, U, B, S, Y) -> float:
    """Sec. 2: f(U, B, S) = sum_k ||y_k - A_k (U b_k + s_k)||^2."""
    X = B @ U.T + S
    return float(np.sum((Y - apply_A(A, X)) ** 2))


def qr_pos(M: np.ndarray):
    """Thin QR of M (n x r) with a positive diagonal R (Householder, then sign fix)."""
    Q, R = np.linalg.qr(M)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


def spectral_norm(M: np.ndarray) -> float:
    """Induced 2-norm (largest singular value), the norm of Sec. 1.1."""
    return float(np.linalg.norm(M, 2))


def subspace_distance(U1: np.ndarray, U2: np.ndarray) -> float:
    """||(I - U1 U1^T) U2||_F for orthonormal U1, U2."""
    return float(np.linalg.norm(U2 - U1 @ (U1.T @ U2)))


def rel_error(X: np.ndarray, X_star: np.ndarray) -> float:
    """Error(X*, X) = ||X* - X||_F / ||X*||_F (Sec. 3)."""
    return float(np.linalg.norm(X_star - X) / np.linalg.norm(X_star))


# ---------------------------------------------------------------------------
# Alg. 1
# ---------------------------------------------------------------------------

def init_sparse(A: np.ndarray, Y: np.ndarray, rho: int, tau0: int = TAU0, mu_rule="support",
                A_t: Optional[np.ndarray] = None, trace: Optional[list] = None):
    """Alg. 1 initialisation, first step: s_k = IHT(y_k, A_k, rho, tau0, 0).  Returns (S, idx)."""
    q, m, n = A.shape
    At = A if A_t is None else A_t
    return iht(Y, lambda S: apply_A(A, S), lambda V: apply_AT(At, V), rho, tau0,
               np.zeros((q, n)), mu_rule=mu_rule, trace=trace, Dop=lambda S: apply_A(At, S))


def backprojection(A: np.ndarray, Y: np.ndarray, S: np.ndarray, A_t: Optional[np.ndarray] = None) -> np.ndarray:
    """Alg. 1 / Sec. 2.3: L_0 = [A_k^T (y_k - A_k s_k)]_k, an n x q matrix."""
    return apply_AT(A if A_t is None else A_t, Y - apply_A(A, S)).T


def spectral_init(L0: np.ndarray, r: int) -> np.ndarray:
    """Alg. 1: U_0 = top r left singular vectors of L_0 (exact SVD)."""
    Uf, _, _ = np.linalg.svd(L0, full_matrices=False)
    return Uf[:, :r]


def rank_budget(n: int, q: int, m: int) -> int:
    """Sec. 2.6: the energy threshold looks at the first min(n/10, q/10, m/10)
    singular values of L_0 (rounded down; at least one)."""
    return max(1, min(n, q, m) // 10)


def auto_rank(L0: np.ndarray, m: int, energy: float = ENERGY):
    """Sec. 2.6, automatic rank: the b% energy threshold on the leading singular
    values of L_0 (b = 65 in the paper's experiments).

    With sigma_1 >= sigma_2 >= ... the singular values of L_0 (n x q) and
    K = rank_budget(n, q, m), the rank is the smallest k such that the energy of
    the first k values, sum_{i <= k} sigma_i^2, is at least `energy` times the
    energy of the first K.  Returns (r, sigma_1..sigma_K).
    """
    n, q = L0.shape
    K = rank_budget(n, q, m)
    sv = np.linalg.svd(L0, compute_uv=False)[:K]
    cum = np.cumsum(sv ** 2)
    r = int(np.searchsorted(cum, energy * cum[-1], side="left")) + 1
    return min(r, K), sv


@dataclasses.dataclass
class State:
    U: np.ndarray                 # (n, r) current U (the one the next iteration uses)
    S: np.ndarray                 # (q, n) dense S
    idx: Optional[np.ndarray] = None  # (q, rho) kept support of each column, ascending
    B: Optional[np.ndarray] = None  # (q, r)
    U_fit: Optional[np.ndarray] = None  # the U that B and S were fitted with
    eta: Optional[float] = None
    t: int = 0


def initialise(A, Y, r, rho, tau0=TAU0, mu_rule="support", A_t=None) -> State:
    """Initialisation block of Alg. 1 (Sec. 2.3): sparse part first with B = 0, then
    spectral init.  r = None takes the automatic rank of Sec. 2.6 from L_0."""
    S, idx = init_sparse(A, Y, rho, tau0, mu_rule, A_t)
    L0 = backprojection(A, Y, S, A_t)
    if r is None:
        r = auto_rank(L0, A.shape[1])[0]
    U0 = spectral_init(L0, r)
    return State(U=U0, S=S, idx=idx)


def gdmin_iteration(A, Y, st: State, rho: int, tau: int = TAU, eta_c: float = ETA_C,
                    mu_rule="support", record: Optional[dict] = None, A_t=None,
                    trace: Optional[list] = None) -> State:
    """One GDmin iteration of Alg. 1.

    z_k, M_k from the current U; warm-started IHT for s_k; LS for b_k
    (eq. (bk_LS)); gradient in U (Sec. 2.1); eta fixed at t = 1 (Sec. 2.6);
    projected GD step U+ = QR(U - eta grad).
    """
    U = st.U
    At = A if A_t is None else A_t
    P, G = projector_parts(A, U)                             # A_k U and its Gram
    Z = project_out(P, G, Y)                                 # z_k
    Mop = lambda S: project_out(P, G, apply_A(A, S))         # s -> M_k s
    MTop = lambda V: apply_AT(At, project_out(P, G, V))      # v -> M_k^T v (projector is symmetric)
    Dop = lambda S: project_out(P, G, apply_A(At, S))        # step-length product
    S, idx = iht(Z, Mop, MTop, rho, tau, st.S, st.idx, mu_rule=mu_rule, trace=trace, Dop=Dop)
    B = pinv_apply(P, G, Y - apply_A(A, S))                  # b_k
    grad = grad_U(A, U, B, S, Y, A_t)
    eta = st.eta
    if eta is None:
        nrm = spectral_norm(grad)
        eta = eta_c / nrm if nrm > 0 else 0.0
    U_new, _ = qr_pos(U - eta * grad)
    if record is not None:
        record.update(P=P, G=G, Z=Z, S=S, idx=idx, B=B, grad=grad, eta=eta, U_tilde=U - eta * grad)
    return State(U=U_new, S=S, idx=idx, B=B, U_fit=U, eta=eta, t=st.t + 1)


def estimate(st: State) -> np.ndarray:
    """Output of Alg. 1 from the consistent pair: x_k = U b_k + s_k, U being the one b_k was fitted with."""
    return st.U_fit @ st.B.T + st.S.T


def solve(A, Y, r, rho, t_max: int = T_MAX, tau0: int = TAU0, tau: int = TAU,
          eta_c: float = ETA_C, X_star: Optional[np.ndarray] = None,
          err_tol: Optional[float] = None, mu_rule="support", U0: Optional[np.ndarray] = None,
          A_t: Optional[np.ndarray] = None):
    """Alg. 1 end to end.  Returns (state, history of Error(X*, X_t) when X_star is given)."""
    st = initialise(A, Y, r, rho, tau0, mu_rule, A_t)
    if U0 is not None:
        st.U = np.array(U0, dtype=np.float64)
    hist = []
    for _ in range(t_max):
        st = gdmin_iteration(A, Y, st, rho, tau, eta_c, mu_rule, A_t=A_t)
        if X_star is not None:
            hist.append(rel_error(estimate(st), X_star))
            if err_tol is not None and hist[-1] < err_tol:
                break
    return st, hist
