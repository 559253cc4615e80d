"""Writes study_oracle.json: the FP64 oracle's relative error ||X - X*||_F / ||X*||_F
after T_max iterations on the first two seeded runs of every cell of the studies of
Sec. 3, on the same seeded instances as the GPU studies:

  * Fig. 1: Gaussian A_k, n = q = 600, m = 80, r = 4, rho in {2, 5, 6, 7}, threshold
    budget rho_max = 7, S1 values U[-6, 6], T_max = 200;
  * Fig. 2: the same sizes with rho = 2, rho_max = 5, laws S1 and S2 ({+-1, +-10, +-100});
  * Table 1: partial Fourier, n = q = 400 as 20 x 20 and 1 x 400 frames, r = 4, rho = 2,
    rho_max = 5, S1 values, real X*, T_max = 10, m in {40, 60, 80, 100, 150, 200, 250, 300}.

Gaussian A_k is the canonical Philox draw of the request's key (bit-exact with the
device generator), and y_k = A_k x*_k is formed in FP64 and rounded to FP32, as the
device measures it.  Only oracle/ and the seeded input generators are called.
Run from the repository root: python tests/golden/make_study_oracle.py (about 15 min).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import altgdmin_oracle as O      # noqa: E402
from oracle import fourier_oracle as F       # noqa: E402
from paper_2311_03824_amd import instances as I   # noqa: E402

SEED = 231103900
RUNS = 2
FIG1 = dict(n=600, q=600, m=80, r=4, rho_max=7, rhos=(2, 5, 6, 7), s_dist="uniform", s_scale=6.0, t_max=200)
FIG2 = dict(n=600, q=600, m=80, r=4, rho=2, rho_max=5, laws=(("S1", "uniform", 6.0), ("S2", "pm_powers", 1.0)),
            t_max=200)
TABLE1 = dict(n=400, q=400, r=4, rho=2, rho_max=5, ms=(40, 60, 80, 100, 150, 200, 250, 300),
              frames=((20, 20), (1, 400)), s_dist="uniform", s_scale=6.0, t_max=10)


def gaussian_error(n, q, m, r, rho, rho_max, s_dist, s_scale, t_max, seed, table):
    req = I.ServeRequest(idx=0, n=n, q=q, m=m, r=r, rho=rho, a_format="f32", seed=seed)
    truth = I.request_truth(req, s_scale=s_scale, s_dist=s_dist)
    _, _, At = I.canonical_philox_A(req.a_seed, range(q), n, m, req.lda, table)
    A = np.ascontiguousarray(At[:, :, :m].transpose(0, 2, 1), dtype=np.float64)
    Y = np.einsum("kij,kj->ki", A, truth["Xt"]).astype(np.float32).astype(np.float64)
    _, hist = O.solve(A, Y, r, rho_max, t_max=t_max, X_star=truth["Xt"].T)
    return hist[-1]


def fourier_error(n1, n2, q, m, r, rho, rho_max, s_dist, s_scale, t_max, seed):
    fi = I.make_fourier_instance(n1, n2, q, m, r, rho, seed, real_signal=True, s_dist=s_dist, s_scale=s_scale)
    op = F.PartialFourier(n1, n2, fi.mask)
    _, hist = F.solve(op, fi.Y, r, rho_max, t_max=t_max, X_star=fi.X_star)
    return hist[-1]


def main():
    table = I.normal_table()
    out = {"runs_per_cell": RUNS, "fig1": {}, "fig2": {}, "table1": {}}
    t0 = time.time()
    c = FIG1
    for rho in c["rhos"]:
        out["fig1"][f"rho={rho}"] = [
            {"seed": SEED + 1000 * rho + i,
             "error": gaussian_error(c["n"], c["q"], c["m"], c["r"], rho, c["rho_max"], c["s_dist"], c["s_scale"],
                                     c["t_max"], SEED + 1000 * rho + i, table)} for i in range(RUNS)]
        print(f"fig1 rho={rho}: {out['fig1'][f'rho={rho}']}  ({time.time() - t0:.0f} s)", flush=True)
    c = FIG2
    for li, (name, dist, scale) in enumerate(c["laws"]):
        seeds = [SEED + 50000 + 20000 * li + i for i in range(RUNS)]
        out["fig2"][name] = [{"seed": s, "error": gaussian_error(c["n"], c["q"], c["m"], c["r"], c["rho"], c["rho_max"],
                                                                  dist, scale, c["t_max"], s, table)} for s in seeds]
        print(f"fig2 {name}: {out['fig2'][name]}  ({time.time() - t0:.0f} s)", flush=True)
    c = TABLE1
    for n1, n2 in c["frames"]:
        key = f"{n1}x{n2}"
        out["table1"][key] = {}
        for m in c["ms"]:
            seeds = [SEED + 90000 + 100 * m + i for i in range(RUNS)]
            out["table1"][key][f"m={m}"] = [
                {"seed": s, "error": fourier_error(n1, n2, c["q"], m, c["r"], c["rho"], c["rho_max"], c["s_dist"],
                                                   c["s_scale"], c["t_max"], s)} for s in seeds]
        print(f"table1 {key}: done  ({time.time() - t0:.0f} s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "study_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
