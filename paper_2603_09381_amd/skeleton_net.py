"""Training recipe of the learned-skeleton network and the measurement of what it gains.

The network proposes each leaf cell's skeleton columns and ranks (the adaptive-rank ID of
the paper's Sec. 3 at the leaves); a short CPQR on the proposals, a judge and a full-CPQR
fallback keep the factorisation exact to the ID tolerance.  Everything here goes through
the library's C-ABI: pmx_id_dataset labels leaf nodes with the full IDs of training
geometries, pmx_mlp_train fits the network on the GPU, and factorisations with and
without the model are timed from pmx_info.

Recipe (20k cells): training geometries `workloads.config5_train(i)` (32 x 32 random smooth
shapes, k+ a in [1, 8]) for i < ceil(cells / 1024); 3 hidden layers of 256.  Evaluation:
`workloads.config5(k)`, the 32 x 32 grid of random shapes with seed 6, at k+ in {5, 10, 20}.

    python -m paper_2603_09381_amd.skeleton_net train  MODEL [--cells 20480] [--epochs 30]
    python -m paper_2603_09381_amd.skeleton_net gain   MODEL [--grid 32] [--k 5 10 20]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import tempfile
import time

from . import pmx, workloads as W


def train(model_path, cells=20480, grid=32, epochs=30, batch=4096, hidden=256, layers=3, seed=1, data_path=None):
    """Label the leaf nodes of ceil(cells / grid^2) training geometries with the full IDs and
    train the network; returns (final loss, seconds for the labels, seconds for training)."""
    ngeo = max(1, math.ceil(cells / (grid * grid)))
    own = data_path is None
    if own:
        fd, data_path = tempfile.mkstemp(prefix="pmx_ids_", suffix=".bin")
        os.close(fd)
    try:
        t0 = time.perf_counter()
        for i in range(ngeo):
            pmx.id_dataset(W.config5_train(i, g=grid), data_path, append=i > 0)
        t1 = time.perf_counter()
        loss = pmx.mlp_train(data_path, model_path, epochs=epochs, batch=batch, hidden=hidden, layers=layers,
                             seed=seed)
        t2 = time.perf_counter()
    finally:
        if own and os.path.exists(data_path):
            os.remove(data_path)
    return loss, t1 - t0, t2 - t1


def _factor(w, reps, **kw):
    """Best of `reps` factorisations: (info of the fastest, densities of the last)."""
    import torch
    best, dens = None, None
    for _ in range(reps):
        fac = pmx.Factor(w, pmx.options(w, timing=1, **kw))
        info = fac.info()
        dens = fac.solve_plane_waves(w.angles)
        torch.cuda.synchronize()
        fac.close()
        if best is None or info.t_factor_ms < best.t_factor_ms:
            best = info
    return best, dens


def gain(model_path, grid=32, ks=(5.0, 10.0, 20.0), reps=3, precision=0, id_tol=1e-10):
    """Per k+: factor time, leaf-ID stage time and their kernels with and without the
    network, cells the proposals settled and those that fell back, and the relative
    difference of the two solutions."""
    import torch
    names = pmx.KERNEL_NAMES
    leaf_kernels = ("k_ts_leaf", "k_ts_update", "k_cpqr_update", "k_cpqr")
    out = []
    for k in ks:
        w = W.config5(k_ext=float(k), g=grid)
        full, xf = _factor(w, reps, precision=precision, id_tol=id_tol)
        lrn, xl = _factor(w, reps, precision=precision, id_tol=id_tol, learned=1, model_path=str(model_path))
        row = {"k_ext": k, "n_unknowns": w.n_unknowns, "cells": w.m,
               "factor_ms": {"full": full.t_factor_ms, "learned": lrn.t_factor_ms},
               "leaf_id_ms": {"full": full.t_phase_ms[7], "learned": lrn.t_phase_ms[7]},
               "proposal_ms": lrn.t_phase_ms[8],
               "qr_cpqr_kernel_ms": {"full": sum(full.t_kernel_ms[names.index(n)] for n in leaf_kernels),
                                     "learned": sum(lrn.t_kernel_ms[names.index(n)] for n in leaf_kernels)},
               "learned_cells": lrn.id_learned, "fallback_cells": lrn.id_fallback,
               "fallback_rate": lrn.id_fallback / max(1, lrn.id_learned + lrn.id_fallback),
               "root_size": {"full": full.root_size, "learned": lrn.root_size},
               "rel_diff": float(torch.linalg.norm(xl - xf) / torch.linalg.norm(xf))}
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=("train", "gain"))
    ap.add_argument("model")
    ap.add_argument("--cells", type=int, default=20480)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--grid", type=int, default=32)
    ap.add_argument("--k", type=float, nargs="+", default=[5.0, 10.0, 20.0])
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if a.what == "train":
        loss, tl, tt = train(a.model, cells=a.cells, epochs=a.epochs)
        print(json.dumps({"model": a.model, "cells": a.cells, "final_loss": loss, "label_s": tl, "train_s": tt}))
    else:
        for row in gain(a.model, grid=a.grid, ks=a.k):
            print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
