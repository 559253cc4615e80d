"""Support comparison under the near-tie rule of the parity contract.

The FP32 path and the FP64 oracle may keep different supports only where the
oracle's HardThreshold input nearly ties at the cut: a column must agree
exactly whenever every IHT step it went through had an oracle gap
|v|_(rho) - |v|_(rho+1) above 64 * 2^-24 * max|v| (and, at a start with no
support, the same gap of the gradient whose HardThreshold picks the support
of the first step length).  Columns below the bound are counted, not failed.
"""
import numpy as np

U32 = 2.0 ** -24
GAP_BOUND = 64 * U32


def ht_gap(V, rho):
    """Per row: (|v|_(rho) - |v|_(rho+1)) / max|v| (inf when rho is 0 or n)."""
    a = -np.sort(-np.abs(np.asarray(V)), axis=1)
    q, n = a.shape
    if rho <= 0 or rho >= n:
        return np.full(q, np.inf)
    mx = np.where(a[:, 0] > 0, a[:, 0], 1.0)
    return (a[:, rho - 1] - a[:, rho]) / mx


def iht_gaps(trace, S0, rho, no_start):
    """Smallest normalised gap over the IHT steps recorded by the oracle's `trace`,
    from the start S0 (v_t = s_{t-1} - mu_t g_t)."""
    gaps = np.full(S0.shape[0], np.inf)
    S_prev = S0
    for t, tr in enumerate(trace):
        if t == 0 and no_start:
            gaps = np.minimum(gaps, ht_gap(tr["G"], rho))
        v = S_prev - tr["mu"][:, None] * tr["G"]
        gaps = np.minimum(gaps, ht_gap(v, rho))
        S_prev = tr["S"]
    return gaps


def check_supports(gpu_idx, ref_idx, gaps, what="", bound=GAP_BOUND):
    """Exact agreement on every column whose smallest oracle gap exceeds the bound.
    Returns the boolean mask of agreeing columns."""
    same = np.array([np.array_equal(a, b) for a, b in zip(gpu_idx, ref_idx)])
    near = gaps <= bound
    bad = ~same & ~near
    print(f"{what}: {int((~same).sum())} of {len(same)} columns differ; "
          f"{int(near.sum())} below the near-tie bound; smallest gap {float(np.min(gaps)):.3e}")
    assert not bad.any(), (what, np.nonzero(bad)[0][:10], gaps[bad][:10])
    return same
