"""FP64 (complex128) CPU oracle of AltGDmin-LR+S with partial Fourier measurements.

Source: S. Babu, N. Vaswani, "A Fast Algorithm for Low Rank + Sparse column-wise
Compressive Sensing", arXiv 2311.03824: Alg. 1 and Alg. 2 with the measurement
operators of Sec. 1.1 taken as partial Fourier matrices (the Fourier setting the
paper names next to the Gaussian one, and its Table 1 experiment).  Complex
data: every transpose of the real algorithm is a conjugate transpose, the
magnitude of HardThreshold is the modulus, norms are Euclidean.

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It imports nothing from the product
package and shares no code with it.

Operator.  A frame x (N1 x N2, flattened row-major, n = N1 N2) is mapped by the
unitary 2D DFT, (F x)[u1, u2] = (N1 N2)^(-1/2) sum_{j1, j2} x[j1, j2]
exp(-2 pi i (u1 j1 / N1 + u2 j2 / N2)), and A_k keeps the frequencies
mask[k] (indices u = u1 N2 + u2).  A_k A_k^H = I_m.

Arrays: Y (q, m) with Y[k] = y_k; S dense (q, n) with S[k] = s_k; U (n, r);
B (q, r) with B[k] = b_k.

Readings (as in the real oracle, plus the complex ones):
  * IHT step: mu = ||g_T||^2 / ||M g_T||^2 (normalised IHT on the previous
    support T; supp H_rho(g) when s = 0), g = M^H (M s - z).
  * HardThreshold: exactly rho entries; larger modulus first, lower index on ties.
  * grad_U f = sum_k A_k^H r_k b_k^H (Wirtinger gradient without the factor 2);
    eta = 0.14 / ||grad_U f(U_0, B_1, S_1)||_2 at t = 1.
  * QR: thin QR with R_ii real and positive.
  * Output from the consistent pair (the U that B and S were fitted with).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

ETA_C = 0.14
TAU0 = 10
TAU = 3
T_MAX = 200
ENERGY = 0.65    # energy threshold of the automatic rank (Sec. 2.6)


class PartialFourier:
    """A_k = rows mask[k] of the unitary 2D DFT of N1 x N2 frames."""

    def __init__(self, N1: int, N2: int, mask: np.ndarray):
        self.N1, self.N2 = int(N1), int(N2)
        self.mask = np.asarray(mask, dtype=np.int64)
        self.q, self.m = self.mask.shape
        self.n = self.N1 * self.N2
        self._rows = np.arange(self.q)[:, None]

    def apply(self, X: np.ndarray) -> np.ndarray:
        """(q, n) -> (q, m): A_k x_k for every k."""
        F = np.fft.fft2(np.asarray(X).reshape(self.q, self.N1, self.N2), norm="ortho")
        return F.reshape(self.q, self.n)[self._rows, self.mask]

    def adjoint(self, V: np.ndarray) -> np.ndarray:
        """(q, m) -> (q, n): A_k^H v_k for every k (zero-filled inverse unitary DFT)."""
        grid = np.zeros((self.q, self.n), np.complex128)
        grid[self._rows, self.mask] = V
        return np.fft.ifft2(grid.reshape(self.q, self.N1, self.N2), norm="ortho").reshape(self.q, self.n)

    def apply_U(self, U: np.ndarray) -> np.ndarray:
        """(n, r) -> (q, m, r): P_k = A_k U for every k (the DFT of U's columns, then each mask)."""
        r = U.shape[1]
        FU = np.fft.fft2(U.T.reshape(r, self.N1, self.N2), norm="ortho").reshape(r, self.n).T
        return FU[self.mask]

    def dense(self, k: int) -> np.ndarray:
        """A_k as an explicit m x n matrix, written from the DFT definition (small sizes only)."""
        j1, j2 = np.divmod(np.arange(self.n), self.N2)
        u1, u2 = np.divmod(self.mask[k], self.N2)
        ph = np.outer(u1, j1) / self.N1 + np.outer(u2, j2) / self.N2
        return np.exp(-2j * np.pi * ph) / np.sqrt(self.n)


def hard_threshold(V: np.ndarray, rho: int):
    """Keep the rho entries of largest modulus of each row (lower index first on ties)."""
    V = np.asarray(V, dtype=np.complex128)
    if np.isnan(V).any():
        raise ValueError("HardThreshold: NaN input")
    q = V.shape[0]
    order = np.argsort(-np.abs(V), axis=1, kind="stable")
    idx = np.sort(order[:, :rho], axis=1)
    out = np.zeros_like(V)
    rows = np.arange(q)[:, None]
    out[rows, idx] = V[rows, idx]
    return out, idx


def _sq(V: np.ndarray) -> np.ndarray:
    return np.sum(V.real ** 2 + V.imag ** 2, axis=1)


def iht(z, Mop: Callable, MHop: Callable, rho: int, tau: int, S0, idx0=None, trace=None):
    """Alg. 2 for all columns, complex: g = M^H (M s - z), mu on the previous support, HardThreshold."""
    S = np.array(S0, dtype=np.complex128, copy=True)
    q = S.shape[0]
    rows = np.arange(q)[:, None]
    idx = None if idx0 is None else np.asarray(idx0, dtype=np.int64)
    for _ in range(tau):
        R = Mop(S) - z
        G = MHop(R)
        T = idx if idx is not None else hard_threshold(G, rho)[1]
        D = np.zeros_like(G)
        D[rows, T] = G[rows, T]
        W = Mop(D)
        gg, ww = _sq(D), _sq(W)
        ok = (ww > 0) & np.isfinite(ww) & np.isfinite(gg)
        mu = np.where(ok, gg / np.where(ok, ww, 1.0), 0.0)
        S, idx = hard_threshold(S - mu[:, None] * G, rho)
        if trace is not None:
            trace.append(dict(G=G, W=W, mu=mu, S=S, idx=idx))
    return S, idx


def projector_parts(op: PartialFourier, U: np.ndarray):
    """P_k = A_k U and G_k = P_k^H P_k."""
    P = op.apply_U(U)
    G = np.matmul(P.conj().transpose(0, 2, 1), P)
    return P, G


def pinv_apply(P, G, V):
    """(A_k U)^dagger v_k = G_k^{-1} P_k^H v_k, (q, m) -> (q, r)."""
    PhV = np.matmul(P.conj().transpose(0, 2, 1), V[:, :, None])
    return np.linalg.solve(G, PhV)[:, :, 0]


def project_out(P, G, V):
    """v_k - P_k G_k^{-1} P_k^H v_k."""
    return V - np.matmul(P, pinv_apply(P, G, V)[:, :, None])[:, :, 0]


def grad_U(op: PartialFourier, U, B, S, Y):
    """sum_k A_k^H (A_k (U b_k + s_k) - y_k) b_k^H, an (n, r) matrix."""
    X = B @ U.T + S
    H = op.adjoint(op.apply(X) - Y)
    return H.T @ B.conj()


def cost(op, U, B, S, Y) -> float:
    X = B @ U.T + S
    return float(np.sum(np.abs(Y - op.apply(X)) ** 2))


def qr_pos(M: np.ndarray):
    """Thin QR with R_ii real and positive."""
    Q, R = np.linalg.qr(M)
    d = np.diag(R)
    ad = np.abs(d)
    ph = np.where(ad > 0, d / np.where(ad > 0, ad, 1.0), 1.0)
    return Q * ph, R * ph.conj()[:, None]


def spectral_norm(M) -> float:
    return float(np.linalg.norm(M, 2))


def subspace_distance(U1, U2) -> float:
    """||(I - U1 U1^H) U2||_F for orthonormal U1, U2."""
    return float(np.linalg.norm(U2 - U1 @ (U1.conj().T @ U2)))


def rel_error(X, X_star) -> float:
    return float(np.linalg.norm(X_star - X) / np.linalg.norm(X_star))


def init_sparse(op, Y, rho, tau0=TAU0):
    return iht(Y, op.apply, op.adjoint, rho, tau0, np.zeros((op.q, op.n), np.complex128))


def backprojection(op, Y, S):
    """L_0 = [A_k^H (y_k - A_k s_k)]_k, n x q."""
    return op.adjoint(Y - op.apply(S)).T


def spectral_init(L0, r):
    Uf, _, _ = np.linalg.svd(L0, full_matrices=False)
    return Uf[:, :r]


def auto_rank(L0, m, energy=ENERGY):
    """Sec. 2.6 automatic rank on a complex L_0: the smallest k whose leading
    singular values hold `energy` of the energy sum_i sigma_i^2 of the first
    K = max(1, floor(min(n, q, m) / 10)).  Returns (r, sigma_1..sigma_K)."""
    n, q = L0.shape
    K = max(1, min(n, q, m) // 10)
    sv = np.linalg.svd(L0, compute_uv=False)[:K]
    cum = np.cumsum(sv ** 2)
    r = int(np.searchsorted(cum, energy * cum[-1], side="left")) + 1
    return min(r, K), sv


@dataclasses.dataclass
class State:
    U: np.ndarray
    S: np.ndarray
    idx: Optional[np.ndarray] = None
    B: Optional[np.ndarray] = None
    U_fit: Optional[np.ndarray] = None
    eta: Optional[float] = None
    t: int = 0


def initialise(op, Y, r, rho, tau0=TAU0) -> State:
    """Initialisation of Alg. 1; r = None takes the automatic rank of Sec. 2.6."""
    S, idx = init_sparse(op, Y, rho, tau0)
    L0 = backprojection(op, Y, S)
    if r is None:
        r = auto_rank(L0, op.m)[0]
    U0 = spectral_init(L0, r)
    return State(U=U0, S=S, idx=idx)


def gdmin_iteration(op, Y, st: State, rho, tau=TAU, eta_c=ETA_C, record=None) -> State:
    U = st.U
    P, G = projector_parts(op, U)
    Z = project_out(P, G, Y)
    Mop = lambda S: project_out(P, G, op.apply(S))        # noqa: E731
    MHop = lambda V: op.adjoint(project_out(P, G, V))     # noqa: E731  (the projector is Hermitian)
    S, idx = iht(Z, Mop, MHop, rho, tau, st.S, st.idx)
    B = pinv_apply(P, G, Y - op.apply(S))
    grad = grad_U(op, U, B, S, Y)
    eta = st.eta
    if eta is None:
        nrm = spectral_norm(grad)
        eta = eta_c / nrm if nrm > 0 else 0.0
    U_new, _ = qr_pos(U - eta * grad)
    if record is not None:
        record.update(P=P, G=G, Z=Z, S=S, idx=idx, B=B, grad=grad, eta=eta)
    return State(U=U_new, S=S, idx=idx, B=B, U_fit=U, eta=eta, t=st.t + 1)


def estimate(st: State) -> np.ndarray:
    """x_k = U b_k + s_k from the consistent pair; (n, q)."""
    return st.U_fit @ st.B.T + st.S.T


def solve(op, Y, r, rho, t_max=T_MAX, tau0=TAU0, tau=TAU, eta_c=ETA_C, X_star=None, err_tol=None, U0=None):
    st = initialise(op, Y, r, rho, tau0)
    if U0 is not None:
        st.U = np.array(U0, dtype=np.complex128)
    hist = []
    for _ in range(t_max):
        st = gdmin_iteration(op, Y, st, rho, tau, eta_c)
        if X_star is not None:
            hist.append(rel_error(estimate(st), X_star))
            if err_tol is not None and hist[-1] < err_tol:
                break
    return st, hist
