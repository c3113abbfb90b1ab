"""Benchmark: factor + solve of the proxy fast direct solver on one MI355X.

Workload (default): 16x16 grid of rotated stars r(t) = 0.3(1 + 0.2 cos 5t), unit spacing,
128 nodes each (N = 65536 unknowns), k+ = 10, k- = 15, ID tolerance 1e-10, four plane
waves at angles 2 pi j / 4, FP64.  One step = factorisation + solve of the four
right-hand sides; the boundary samples are host inputs, the densities stay in HBM.
The JSON line reports unknowns per second over the timed steps, the roofline of the
dominant kernel (device time from HIP events around its launches in the timed steps,
algorithmic bytes counted by the library) and the CPU oracle's rate on a sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor+solve seconds & unknowns/s at 1e-8 rel error: tuned vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFS = 78.6           # MI355X FP64 vector and matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_ts_update_stars16.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--grid", type=int, default=16, help="stars per side (16 = the 65536-unknown workload)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-check", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a 256 MiB device copy first (reference kernel for HBM counters)")
    p.add_argument("--no-timing", action="store_true", help="no HIP events around kernels")
    return p.parse_args()


def cpu_baseline(w_full):
    """The oracle's dense solve (assembly, LU, solve) of the 6x6 corner of the same grid."""
    from oracle import dense
    from paper_2603_09381_amd import workloads as W
    sub = W.sub_grid(w_full, 6)
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
            "sample": f"dense PMCHWT-Omit Nystrom solve (Kress self blocks, LAPACK partial-pivot LU) of the "
                      f"6x6 corner of the same star grid, N={sub.n_unknowns}, {len(sub.angles)} right-hand "
                      f"sides, {t:.2f} s"}


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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("la_kernels.hip", "la.h"):
        h.update(open(os.path.join(ROOT, "paper_2603_09381_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch(kname):
    """HBM bytes per launch from the committed PMC summary, if taken on this kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("kernel") != kname or d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def roofline(info_list, names):
    """Dominant kernel among those whose algorithmic work the library counts."""
    ms = np.zeros(16)
    nl = np.zeros(16)
    by = np.zeros(16)
    fl = np.zeros(16)
    for info in info_list:
        ms += np.array(info.t_kernel_ms[:16])
        nl += np.array(info.n_kernel_launch[:16])
        by += np.array(info.kernel_bytes[:16])
        fl += np.array(info.kernel_flops[:16])
    counted = [k for k in range(len(names)) if by[k] > 0 and ms[k] > 0]
    if not counted:
        return None, {}
    k = max(counted, key=lambda i: ms[i])
    t = ms[k] * 1e-3
    per_launch_us = 1e3 * ms[k] / nl[k]
    tr = traffic_per_launch(names[k])
    # the bound follows the kernel's algorithmic intensity against the FP64 ridge point
    ridge = FP64_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if fl[k] / by[k] > ridge:
        roof = {"bound": "mfma", "achieved": fl[k] / t / 1e12, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                "frac": fl[k] / t / 1e12 / FP64_PEAK_TFS}
    else:
        roof = {"bound": "hbm", "achieved": by[k] / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": by[k] / t / 1e9 / HBM_PEAK_GBS}
    roof.update({"traffic": tr, "kernel": names[k], "avg_launch_us": per_launch_us,
            "algorithmic_flops_per_launch": fl[k] / nl[k],
            "algorithmic_bytes_per_launch": by[k] / nl[k],
            "launches_per_step": nl[k] / len(info_list),
            "algorithmic_bytes_per_step": by[k] / len(info_list),
            "hbm_gbs_algorithmic": by[k] / t / 1e9})
    share = {names[i]: round(float(ms[i] / max(ms.sum(), 1e-9)), 4) for i in range(len(names)) if ms[i] > 0}
    return roof, share


def summarize_pmc(fetch_csv, write_csv, kname="k_ts_update"):
    """HBM bytes per launch of `kname` from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE,
    KiB per dispatch), each scaled by what the same counter reads for the 256 MiB device
    copy that --copy-calibration runs first (expected 256 MiB fetched and 256 MiB written)."""
    import csv

    def load(path, counter):
        per, copy = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            name = r["Kernel_Name"]
            if name.startswith(kname + "("):
                per.append(v)
            elif "copy" in name.lower() and int(r["Grid_Size"]) > 1 << 20 and not copy:
                copy.append(v)
        return per, copy

    fetch, cf = load(fetch_csv, "FETCH_SIZE")
    write, cw = load(write_csv, "WRITE_SIZE")
    ref = float(256 << 20)
    ff = cf[0] / ref if cf else 1.0
    fw = cw[0] / ref if cw else 1.0
    per_launch = (np.mean(fetch) / ff + np.mean(write) / fw)
    out = {"kernel": kname, "source_hash": kernel_source_hash(), "bytes_per_launch": per_launch,
           "launches": len(fetch), "fetch_scale": ff, "write_scale": fw,
           "fetch_bytes_per_launch": np.mean(fetch) / ff, "write_bytes_per_launch": np.mean(write) / fw}
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        summarize_pmc(sys.argv[2], sys.argv[3])
        return
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the solver is not sharded "
              f"across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_09381_amd import pmx, workloads as W
    torch.cuda.set_device(0)
    if a.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.config2(a.grid)
    N = w.n_unknowns
    opts = pmx.options(w, timing=0 if a.no_timing else 1)
    for _ in range(a.warmup):
        fac = pmx.Factor(w, opts)
        fac.solve_plane_waves(w.angles)
        fac.close()
    torch.cuda.synchronize()
    times, infos = [], []
    dens = None
    fac = None
    for i in range(a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = pmx.Factor(w, opts)
        dens = fac.solve_plane_waves(w.angles)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(fac.info())
        if i != a.steps - 1:
            fac.close()
    total = sum(times)
    info = infos[-1]
    res = {"metric": METRIC, "value": N * a.steps / total, "unit": "unknowns/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * total / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64)",
           "data": "synthetic",
           "config": {"workload": f"{a.grid}x{a.grid} rotated stars, 128 nodes, k+=10, k-=15, tol 1e-10, "
                                  f"4 plane waves (plain FP64 method)",
                      "n_unknowns": N, "nrhs": len(w.angles), "root_size": info.root_size,
                      "levels": info.levels, "precision": "fp64"}}
    if not a.no_timing:
        roof, share = roofline(infos, pmx.KERNEL_NAMES)
        res["roofline"] = roof
        res["kernel_time_share"] = share
    else:
        res["roofline"] = None
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
