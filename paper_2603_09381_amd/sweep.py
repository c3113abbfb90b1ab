"""Frequency sweep of the compressed size (the frequency half of the paper's O(omega D)
claim, Sec. 4.3 and its Table of conditions): 64 inclusions (an 8 x 8 grid of stars, 200
nodes each, 25,600 unknowns), eps+ = 1, eps- = 5, angular frequency omega in {1, 2, 4, 8}
(k+ = omega, k- = omega sqrt 5), CPQR thresholds {1e-12, 1e-9, 1e-6}, self blocks by the
zeta-corrected trapezoid rule with 41 correction points as in the paper (Sec. 2.2).  The paper's own
shapes are given only as figures; the seeded stars of `workloads.star_grid` stand in.

Per (omega, threshold): the size of the top compressed system, the mean rank per level,
factor and solve times (synchronised host clock around the library calls), and the
relative 2-norm error (Sec. 4.2) against the plain FP64 solve at threshold 1e-14 of the
same system, whose own residual the caller may check on sampled rows with the oracle.

    python -m paper_2603_09381_amd.sweep [--omega 1 2 4 8] [--tol 1e-12 1e-9 1e-6]
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import pmx, workloads as W

REF_TOL = 1e-14


def sweep_workload(omega, g=8, n=200, eps_int=5.0, seed=2, quadrature="zeta"):
    """The sweep's 8 x 8 grid at frequency omega, with the paper's self-interaction rule
    (the zeta-corrected trapezoid, Sec. 2.2) unless told otherwise."""
    w = W.star_grid(g, n=n, k_ext=float(omega), k_int=float(omega) * math.sqrt(eps_int), seed=seed,
                    angles=[0.0])
    w.quadrature = quadrature
    return w


def _run(w, id_tol):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = pmx.Factor(w, pmx.options(w, precision=0, id_tol=id_tol))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = fac.info()
    fac.close()
    ranks = [float(info.rank_mean[l]) for l in range(info.levels)]
    return x, {"root_size": int(info.root_size), "mean_rank_per_level": ranks,
               "factor_s": t1 - t0, "solve_s": t2 - t1}


def frequency_sweep(omegas=(1, 2, 4, 8), tols=(1e-12, 1e-9, 1e-6), g=8, n=200, eps_int=5.0):
    """One row per (omega, threshold); the reference densities are returned per omega."""
    import torch
    rows, refs = [], {}
    for om in omegas:
        w = sweep_workload(om, g=g, n=n, eps_int=eps_int)
        xr, _ = _run(w, REF_TOL)
        refs[om] = (w, xr)
        for tol in tols:
            x, r = _run(w, tol)
            r.update({"omega": om, "id_tol": tol, "n_unknowns": w.n_unknowns,
                      "rel_error_vs_ref": float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr))})
            rows.append(r)
    return rows, refs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--omega", type=float, nargs="+", default=[1, 2, 4, 8])
    ap.add_argument("--tol", type=float, nargs="+", default=[1e-12, 1e-9, 1e-6])
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    rows, _ = frequency_sweep(a.omega, a.tol)
    for r in rows:
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
