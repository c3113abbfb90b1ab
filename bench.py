"""Benchmark: factor + solve of the proxy fast direct solver on one MI355X.

Workload (default): 16x16 grid of rotated stars r(t) = 0.3(1 + 0.2 cos 5t), unit spacing,
128 nodes each (N = 65536 unknowns), k+ = 10, k- = 15, ID tolerance 1e-10, four plane
waves at angles 2 pi j / 4, FP64.  One step = factorisation + solve of the four
right-hand sides, inputs (boundary samples) on the host, densities left in HBM.
The JSON line reports unknowns per second over the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor+solve seconds & unknowns/s at 1e-8 rel error: tuned vs plain, 1 GPU"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--grid", type=int, default=16, help="stars per side (16 = the 65536-unknown workload)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-check", action="store_true")
    return p.parse_args()


def cpu_baseline(w_full):
    """The oracle's dense solve (assembly, LU, solve) of the 4x4 corner of the same grid."""
    from oracle import dense
    from paper_2603_09381_amd import workloads as W
    sub = W.sub_grid(w_full, 4)
    t0 = time.perf_counter()
    dense.solve(sub)
    t = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": sub.n_unknowns / t, "unit": "unknowns/s", "cores": min(cores, threads),
            "kind": "oracle",
            "sample": f"dense PMCHWT-Omit Nystrom solve (Kress self blocks, LAPACK LU) of the 4x4 corner "
                      f"of the same star grid, N={sub.n_unknowns}, {len(sub.angles)} right-hand sides, "
                      f"{t:.2f} s"}


def accuracy(w, x):
    """Relative residual on sampled rows (oracle row evaluation) and the energy defect."""
    from oracle import dense
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(w.n_unknowns, size=48, replace=False))
    r = dense.residual_rows(w, x, rows)
    f = dense.rhs(dense.Geometry(w), w.angles)[rows]
    rel = float(np.linalg.norm(r) / np.linalg.norm(f))
    ed = float(np.max(np.abs(dense.energy_defect(dense.Geometry(w), x))))
    return rel, ed


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the solver is not sharded "
              f"across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_09381_amd import pmx, workloads as W
    torch.cuda.set_device(0)
    w = W.config2(a.grid)
    N = w.n_unknowns
    fac = None
    for _ in range(a.warmup):
        fac = pmx.Factor(w)
        fac.solve_plane_waves(w.angles)
        fac.close()
    torch.cuda.synchronize()
    times = []
    dens = None
    for _ in range(a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = pmx.Factor(w)
        dens = fac.solve_plane_waves(w.angles)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if _ != a.steps - 1:
            fac.close()
    total = sum(times)
    info = fac.info()
    res = {"metric": METRIC, "value": N * a.steps / total, "unit": "unknowns/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * total / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64)",
           "data": "synthetic",
           "config": {"workload": f"{a.grid}x{a.grid} rotated stars, 128 nodes, k+=10, k-=15, tol 1e-10, "
                                  f"4 plane waves (plain FP64 method)",
                      "n_unknowns": N, "nrhs": len(w.angles), "root_size": info.root_size,
                      "levels": info.levels, "precision": "fp64"},
           "roofline": None}
    if not a.no_check:
        x = pmx.dens_to_numpy(dens, w)
        rel, ed = accuracy(w, x)
        res["accuracy"] = {"sampled_row_rel_residual": rel, "max_energy_defect": ed}
    fac.close()
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
