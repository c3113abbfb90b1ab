"""GPU tests of the autotuner and the launch-parameter table.

The table built for a workload holds one valid choice per recorded launch shape.  Factors
that use it, and factors forced onto the alternative kernels of every knob (global-memory,
tall-panel or wider register LU panels, multi- or single-workgroup column-pivoted QR, blocked or
fused level solves, other apply groupings and source splits), solve the same system: their
solutions match the oracle's dense FP64 solve to the bound of their form (plain FP64 at ID
tolerance 1e-10: 5e-9; refined forms, stopped at a relative residual of 1e-10: 1e-8).
"""
import numpy as np
import pytest

from oracle import dense
from paper_2603_09381_amd import workloads as W

pytestmark = pytest.mark.gpu

VALID = {"lu_panel": {0, 1, 2, 3, 4, 6, 8, 10}, "cpqr": {0, 1, 2}, "getrs": {0, 1, 2}, "apply_nr": {1, 2, 4, 8},
         "apply_wg": {512, 1024, 2048, 4096, 8192}, "ts_leaf": {256, 512, 1024}}
FORMS = {0: dict(precision=0, id_tol=1e-10), 1: dict(precision=1, id_tol=1e-5, ir_tol=1e-10),
         2: dict(precision=2, id_tol=1e-6, ir_tol=1e-10)}
BOUND = {0: 5e-9, 1: 1e-8, 2: 1e-8}


def _solve(pmx, w, **kw):
    import torch
    fac = pmx.Factor(w, pmx.options(w, **kw))
    dens = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    x = pmx.dens_to_numpy(dens, w)
    info = fac.info()
    fac.close()
    return x, info


def _forced_table(path, lu, cpqr, getrs, nr=8, wg=2048):
    """Every key of every knob set to one choice (launchers fall back to their built-in
    rule where the choice does not hold the shape)."""
    lines = []
    for rb in (4, 8):
        for a in range(16):
            for b in range(9):
                lines.append(f"lu_panel {rb} {a} {b} 0 {lu}")
                lines.append(f"cpqr {rb} {a} {b} 0 {cpqr}")
                lines.extend(f"getrs {rb} {a} {b} {c} {getrs}" for c in range(10))
    for a in range(28):
        for b in range(10):
            lines.append(f"apply_nr 8 {a} {b} 0 {nr}")
            lines.append(f"apply_wg 8 {a} {b} 0 {wg}")
    path.write_text("\n".join(lines) + "\n")


@pytest.mark.parametrize("form", [1, 0])
def test_autotune_table_and_solve(pmx, tmp_path, form):
    w = W.sub_grid(W.config2(), 4)
    path = tmp_path / "tune.txt"
    print("autotune", w.name, FORMS[form], flush=True)
    pmx.autotune(w, path, reps=2, **FORMS[form])
    text = open(path).read()
    print(text)
    t = pmx.read_tune_table(path)
    knobs = {k[0] for k in t}
    assert {"lu_panel", "cpqr", "getrs"} <= knobs
    if form:
        assert {"apply_nr", "apply_wg"} <= knobs
    for k, v in t.items():
        assert v in VALID[k[0]], (k, v)
        assert k[1] == (8 if form != 1 or k[0].startswith("apply") else 4)
    x, info = _solve(pmx, w, tune_path=str(path), **FORMS[form])
    err = dense.rel_error(x, dense.solve(w))
    print("tuned table: err", err, "root", info.root_size)
    assert err < BOUND[form]


@pytest.mark.parametrize("form,table", [
    (0, dict(lu=3, cpqr=1, getrs=1)),
    (0, dict(lu=1, cpqr=0, getrs=0)),
    (1, dict(lu=3, cpqr=1, getrs=1, nr=1, wg=512)),
    (1, dict(lu=2, cpqr=0, getrs=0, nr=4, wg=8192)),
    (2, dict(lu=3, cpqr=1, getrs=1, nr=2, wg=1024)),
    (0, dict(lu=6, cpqr=0, getrs=0)),
    (1, dict(lu=8, cpqr=0, getrs=0)),
    (1, dict(lu=4, cpqr=1, getrs=0)),
    (0, dict(lu=4, cpqr=1, getrs=2)),
    (2, dict(lu=6, cpqr=0, getrs=2)),
    (0, dict(lu=10, cpqr=1, getrs=1)),
    (1, dict(lu=10, cpqr=0, getrs=2)),
    (0, dict(lu=4, cpqr=2, getrs=1)),
    (1, dict(lu=8, cpqr=2, getrs=2)),
], ids=["plain-global", "plain-wide", "fp32-global", "fp32-wide", "fp64ir-global", "plain-unrolled512",
        "fp32-unrolled1024", "fp32-unrolled256", "plain-ldssolve", "fp64ir-ldssolve", "plain-tall", "fp32-tall",
        "plain-cpqr-persistent", "fp32-cpqr-persistent"])
def test_forced_alternatives_match_dense(pmx, tmp_path, form, table):
    w = W.sub_grid(W.config2(), 4)
    path = tmp_path / "forced.txt"
    _forced_table(path, **table)
    print("forced", table, "form", FORMS[form], flush=True)
    x, info = _solve(pmx, w, tune_path=str(path), **FORMS[form])
    ref = dense.solve(w)
    err = dense.rel_error(x, ref)
    print("forced: err", err, "iters", info.ir_iterations)
    assert err < BOUND[form]
    x0, _ = _solve(pmx, w, **FORMS[form])
    assert dense.rel_error(x, x0) < 2 * BOUND[form]


def test_forced_apply_groupings_agree(pmx, tmp_path):
    """Eight right-hand sides in groups of 1, 2, 4 and 8 per thread and several source
    splits: the refined solutions agree to the refinement tolerance."""
    w = W.sub_grid(W.config2(), 2)
    w.angles = 2 * np.pi * np.arange(8) / 8
    ref = dense.solve(w)
    for nr, wg in ((1, 512), (2, 8192), (4, 1024), (8, 4096)):
        path = tmp_path / f"a{nr}.txt"
        _forced_table(path, lu=3, cpqr=1, getrs=1, nr=nr, wg=wg)
        print("apply grouping", nr, wg, flush=True)
        x, info = _solve(pmx, w, tune_path=str(path), **FORMS[1])
        assert info.ir_residual <= 1e-10
        assert dense.rel_error(x, ref) < 1e-8
