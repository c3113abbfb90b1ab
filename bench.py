"""Benchmark: factor + solve of the proxy fast direct solver on one MI355X, tuned vs plain.

Workload (default): 16x16 grid of rotated stars r(t) = 0.3(1 + 0.2 cos 5t), unit spacing,
128 nodes each (N = 65536 unknowns), k+ = 10, k- = 15, four plane waves at angles
2 pi j / 4.  One step = factorisation + solve of the four right-hand sides (boundary samples
are host inputs; densities stay in HBM).

Forms, both held to a relative residual of 1e-10 / field error of 1e-8:
  plain: FP64 throughout, ID tolerance 1e-10;
  tuned: the factor in complex FP32 (FP32 MFMA QR, LU and Schur products, FP64 pivots) at
         ID tolerance 1e-3, refined against the FP64 operator (near pairs directly, far
         inclusions through multipole expansions) to a relative residual of 1e-10; solves
         replay captured HIP graphs.
Before the timed steps each form gets a launch-parameter table from the library's autotuner
(pmx_autotune on this workload; --no-autotune keeps the built-in rules, --tune-dir keeps
the tables and reuses them in later runs).
`value` is the tuned form's unknowns per second over the timed steps.  The roofline object
covers the tuned form's dominant kernel (found in the warm-up steps, which time every
kernel; in the timed steps HIP events bracket that kernel's launches only), with the
algorithmic work counted by the library; kernel_time_share comes from the warm-up steps.
cpu_baseline times the CPU oracle (dense solve) on a sample of the same workload.
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
PEAK_TFS = {("mfma", 8): 78.6, ("mfma", 4): 157.3, ("alu", 8): 78.6, ("alu", 4): 157.3}
# kernels whose algorithmic work the library counts: bound kind and element size (bytes of
# the real type: 8 in the FP64 form, the factor's type otherwise; the apply is always FP64)
COUNTED = {"k_ts_update": "mfma", "k_ts_leaf": "alu", "k_getrf_panel": "alu", "k_apply_off": "alu"}
TRAFFIC_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = {"k_ts_update": ("la_kernels.hip", "la.h"), "k_ts_leaf": ("la_kernels.hip", "la.h"),
                  "k_getrf_panel": ("la_kernels.hip", "la.h"),
                  "k_apply_off": ("apply_kernels.hip", "assemble.h", "hankel_fast.h", "bessel.h")}
FORMS = {"plain": dict(precision=0, id_tol=1e-10),
         "tuned": dict(precision=1, id_tol=1e-3, ir_tol=1e-10, solve_graph=1)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--grid", type=int, default=16, help="stars per side (16 = the 65536-unknown workload)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-check", action="store_true")
    p.add_argument("--no-plain", action="store_true", help="time the tuned form only")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a 256 MiB device copy first (reference kernel for HBM counters)")
    p.add_argument("--no-timing", action="store_true", help="no HIP events around kernels")
    p.add_argument("--tune-dir", default=None,
                   help="keep the launch tables in this folder; a form whose table is already there "
                        "loads it instead of tuning (a profiled run then uses the bench run's choices)")
    p.add_argument("--no-autotune", action="store_true",
                   help="built-in launch rules instead of a launch-parameter table tuned before the timed steps")
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


def kernel_source_hash(kname):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kname, ("la_kernels.hip", "la.h")):
        h.update(open(os.path.join(ROOT, "paper_2603_09381_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_file(kname, workload_tag):
    return os.path.join(TRAFFIC_DIR, f"traffic_{kname}_{workload_tag}.json")


def traffic_per_launch(kname, workload_tag):
    """HBM bytes per launch from the committed PMC summary, if taken on this kernel source."""
    try:
        d = json.load(open(traffic_file(kname, workload_tag)))
    except Exception:
        return None
    if d.get("kernel") != kname or d.get("source_hash") != kernel_source_hash(kname):
        return None
    return d.get("bytes_per_launch")


def _sums(info_list):
    ms, nl, by, fl = (np.zeros(16) for _ in range(4))
    for info in info_list:
        ms += np.array(info.t_kernel_ms[:16])
        nl += np.array(info.n_kernel_launch[:16])
        by += np.array(info.kernel_bytes[:16])
        fl += np.array(info.kernel_flops[:16])
    return ms, nl, by, fl


def dominant_kernel(info_list, names):
    """From steps that timed every kernel: the index of the dominant kernel whose work the
    library counts (largest summed device time), the overall dominant one, and the time
    shares."""
    ms, _, _, fl = _sums(info_list)
    live = [k for k in range(len(names)) if ms[k] > 0]
    if not live:
        return None, None, {}
    top = max(live, key=lambda i: ms[i])
    counted = [k for k in live if names[k] in COUNTED and fl[k] > 0]
    k = None if not counted else (top if top in counted else max(counted, key=lambda i: ms[i]))
    share = {names[i]: round(float(ms[i] / max(ms.sum(), 1e-9)), 4) for i in live}
    return k, top, share


def roofline(info_list, k, top, names, real_bytes, workload_tag):
    """Kernel k over the timed steps: algorithmic work counted by the library divided by
    the device time of its launches (HIP events on its launch stream)."""
    if k is None:
        return None
    ms, nl, by, fl = _sums(info_list)
    if ms[k] <= 0 or nl[k] <= 0:
        return None
    name = names[k]
    t = ms[k] * 1e-3
    kind = COUNTED[name]
    rb = 8 if name == "k_apply_off" else real_bytes
    peak = PEAK_TFS[(kind, rb)]
    roof = {"bound": kind, "achieved": fl[k] / t / 1e12, "peak": peak, "unit": "TFLOP/s",
            "frac": fl[k] / t / 1e12 / peak, "traffic": traffic_per_launch(name, workload_tag),
            "kernel": name, "avg_launch_us": 1e3 * ms[k] / nl[k],
            "algorithmic_flops_per_launch": fl[k] / nl[k], "algorithmic_bytes_per_launch": by[k] / nl[k],
            "launches_per_step": nl[k] / len(info_list), "hbm_gbs_algorithmic": by[k] / t / 1e9}
    if top is not None and top != k:
        roof["dominant_overall"] = names[top]
    return roof


# timer slots that cover several kernels launched back to back (summed per launch)
SLOT_KERNELS = {"k_apply_off": ("k_apply_p2m", "k_apply_m2m", "k_apply_far", "k_apply_near")}


def summarize_pmc(fetch_csv, write_csv, kname, workload_tag):
    """HBM bytes per launch of `kname` from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE,
    KiB per dispatch), each scaled by what the same counter reads for the 256 MiB device
    copy that --copy-calibration runs first (expected 256 MiB fetched and 256 MiB written).
    `kname` may carry template arguments ("k_ts_update<double>") to pick one instantiation;
    a timer slot of several kernels (k_apply_off: expansions, translations, far and near
    parts) sums each part's dispatches per launch of the slot (the first part's dispatch
    count).  The summary is stored under the plain name."""
    import csv
    base = kname.split("<")[0]
    parts = SLOT_KERNELS.get(kname, (kname,))

    def matches(name, part):
        if "<" in part:
            return name.startswith("void " + part)
        return name.startswith(part + "(") or name.startswith("void " + part + "<")

    def load(path, counter):
        per, copy = {p: [] for p in parts}, []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            name = r["Kernel_Name"]
            hit = [p for p in parts if matches(name, p)]
            if hit:
                per[hit[0]].append(v)
            elif name.startswith("__amd_rocclr_copyBuffer") and not copy:
                copy.append(v)   # the first runtime copy of the run: the 256 MiB calibration copy
        return per, copy

    fetch, cf = load(fetch_csv, "FETCH_SIZE")
    write, cw = load(write_csv, "WRITE_SIZE")
    ref = float(256 << 20)
    ff = cf[0] / ref if cf else 1.0
    fw = cw[0] / ref if cw else 1.0
    nl = len(fetch[parts[0]])
    fb = sum(np.sum(fetch[p]) for p in parts) / nl / ff
    wb = sum(np.sum(write[p]) for p in parts) / nl / fw
    out = {"kernel": base, "instantiation": kname, "parts": list(parts), "workload": workload_tag,
           "source_hash": kernel_source_hash(base), "bytes_per_launch": fb + wb,
           "launches": len(fetch[parts[0]]), "fetch_scale": ff, "write_scale": fw,
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb}
    json.dump(out, open(traffic_file(base, workload_tag), "w"), indent=1)
    print(json.dumps(out))


def run_form(pmx, w, kw, steps, warmup, timing):
    """Warm-up steps time every kernel (time shares, dominant kernel); the timed steps time
    only the dominant counted kernel, so that events around the other launches do not
    slow the step (and solve sequences without it replay their graphs)."""
    import torch
    names = pmx.KERNEL_NAMES
    winfos = []
    opts = pmx.options(w, timing=timing, **kw)
    for _ in range(warmup):
        fac = pmx.Factor(w, opts)
        fac.solve_plane_waves(w.angles)
        winfos.append(fac.info())
        fac.close()
    torch.cuda.synchronize()
    k, top, share = dominant_kernel(winfos, names) if timing else (None, None, {})
    if k is not None:
        opts = pmx.options(w, timing=timing, timing_kernels=1 << k, **kw)
    times, infos = [], []
    dens = None
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = pmx.Factor(w, opts)
        dens = fac.solve_plane_waves(w.angles)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(fac.info())
        fac.close()
    if timing and k is None:     # no warm-up: every kernel was timed in the timed steps
        k, top, share = dominant_kernel(infos, names)
    return times, infos, dens, (k, top, share)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        summarize_pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
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
    tag = f"stars{a.grid}"   # traffic summaries are per form: <tag>_tuned, <tag>_plain
    timing = 0 if a.no_timing else 1
    forms = {k: dict(v) for k, v in FORMS.items()}
    tune_s = {}
    if not a.no_autotune:
        # launch-parameter tables for this GPU and workload, built before (outside) the timed steps
        import tempfile
        tdir = a.tune_dir or tempfile.mkdtemp(prefix="pmx_tune_")
        os.makedirs(tdir, exist_ok=True)
        for name in ("tuned", "plain") if not a.no_plain else ("tuned",):
            path = os.path.join(tdir, f"{tag}_{name}.txt")
            if os.path.exists(path):
                tune_s[name] = None
            else:
                t0 = time.perf_counter()
                pmx.autotune(w, path, reps=2, **forms[name])
                tune_s[name] = time.perf_counter() - t0
            forms[name]["tune_path"] = path
    times, infos, dens, dom = run_form(pmx, w, forms["tuned"], a.steps, a.warmup, timing)
    total = sum(times)
    info = infos[-1]
    res = {"metric": METRIC, "value": N * a.steps / total, "unit": "unknowns/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * total / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64 factor, f64 residual (mixed)", "data": "synthetic",
           "config": {"workload": f"{a.grid}x{a.grid} rotated stars, 128 nodes, k+=10, k-=15, 4 plane waves",
                      "n_unknowns": N, "nrhs": len(w.angles), "tuned": FORMS["tuned"], "plain": FORMS["plain"],
                      "root_size": info.root_size, "levels": info.levels,
                      "refinement_steps": info.ir_iterations, "final_relative_residual": info.ir_residual,
                      "launch_table": ("autotuned before the timed steps, s: " +
                                       ", ".join(f"{k} {v:.1f}" if v is not None else f"{k} loaded"
                                                 for k, v in tune_s.items())) if tune_s
                                      else "built-in rules"}}
    if timing:
        res["roofline"] = roofline(infos, dom[0], dom[1], pmx.KERNEL_NAMES, 4, tag + "_tuned")
        res["kernel_time_share"] = dom[2]
    else:
        res["roofline"] = None
    if not a.no_check:
        rel, ed = accuracy(w, pmx.dens_to_numpy(dens, w))
        res["accuracy"] = {"sampled_row_rel_residual": rel, "max_energy_defect": ed}
    if not a.no_plain:
        ptimes, pinfos, pdens, pdom = run_form(pmx, w, forms["plain"], a.steps, a.warmup, timing)
        ptotal = sum(ptimes)
        plain = {"value": N * a.steps / ptotal, "ms_per_step": 1e3 * ptotal / a.steps,
                 "root_size": pinfos[-1].root_size}
        if not a.no_check:
            prel, ped = accuracy(w, pmx.dens_to_numpy(pdens, w))
            plain["accuracy"] = {"sampled_row_rel_residual": prel, "max_energy_defect": ped}
        if timing:
            plain["roofline"] = roofline(pinfos, pdom[0], pdom[1], pmx.KERNEL_NAMES, 8, tag + "_plain")
            plain["kernel_time_share"] = pdom[2]
        res["plain"] = plain
        res["speedup_vs_plain"] = res["value"] / plain["value"]
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
