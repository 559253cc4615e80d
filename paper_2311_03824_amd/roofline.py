"""Algorithmic HBM bytes of the two streaming kernels of a GDmin iteration, and the
algorithmic FLOPs of the partial Fourier column kernel.

These are the bytes the algorithm must move (each element of A read once per
pass, the small per-column vectors once), not what the hardware moved; the
benchmark divides them by measured kernel durations to place a kernel against
the 8 TB/s HBM roofline, and the serving loop sums them over the iterations it
ran.  Host-side bookkeeping only: no arithmetic of the method.
"""
from __future__ import annotations


def column_kernel_bytes(n, q, m, r, rho, tau, a_bytes=4.0, gather_bytes=None):
    """Algorithmic HBM bytes of one launch of the column kernel (tau IHT iterations + LS/gradient tail).

    Per column: (tau + 1) streaming passes over A_k (m n elements), (tau + 1)
    gathers of the rho support columns (rho m elements), y_k, P_k (m r FP32),
    G_k^{-1} (r^2 FP64), the support in and out (2 rho (4 + 4) bytes), h_k
    (n FP32), b_k (r FP32) and ||r_k||^2.  a_bytes: bytes per element of the
    streaming passes; gather_bytes: of the support gathers (default a_bytes;
    the mixed BF16 form streams 2 bytes and gathers 4).
    """
    gb = a_bytes if gather_bytes is None else gather_bytes
    per_col = ((tau + 1) * m * n * a_bytes + (tau + 1) * rho * m * gb + 4 * m + 4 * m * r
               + 8 * r * r + 16 * rho + 4 * n + 4 * r + 8)
    return per_col * q


def au_kernel_bytes(n, q, m, r, a_bytes=4.0):
    """Per column: one pass over A_k, U (n r, L2-resident after the first column), P_k written, G^{-1} written."""
    return q * (m * n * a_bytes + 4 * m * r + 8 * r * r) + 4 * n * r


def iteration_bytes(n, q, m, r, rho, tau=3, mixed=False):
    """A_k U plus the column kernel of one GDmin iteration.  FP32 plane and BF16 hi + lo:
    4 bytes per element everywhere; the mixed BF16 form: 2 in the column passes."""
    return (au_kernel_bytes(n, q, m, r, 4.0)
            + column_kernel_bytes(n, q, m, r, rho, tau, 2.0 if mixed else 4.0, 4.0))


def fourier_column_flops(n1, n2, q, m, r, transforms=8):
    """Algorithmic FLOPs of one launch of the partial Fourier column kernel (real
    flops, a complex multiply-add counted as 8).

    Per frame: `transforms` unitary 2D DFTs of n = n1 n2 points at the
    conventional 5 n log2 n of a radix-2 FFT (8 per GDmin call once the supports
    hold: per IHT step the adjoint of the residual and the forward transform of
    the step on the support, plus the LS / gradient tail), and the Gram
    G_k = P_k^H P_k (m r^2 multiply-adds).  The projections and the IHT updates
    (O(m r) and O(n) per step) are left out: under 2 % of the total here.
    """
    import math
    n = n1 * n2
    return q * (transforms * 5.0 * n * math.log2(n) + 8.0 * m * r * r)
