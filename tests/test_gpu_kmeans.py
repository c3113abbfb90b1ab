"""General arrangements on the GPU (Sec. 4.4, Discussions): the k-means tree, the
eta-admissibility near rule and leaves of several inclusions, end to end against the
oracle's dense solve of the same Nystrom system.

A leaf of several inclusions is compressed as one cell: its block holds the inclusions'
self blocks and the exterior-kernel blocks between them, and its interpolative
decompositions see its near cells and its proxy circle.  The leaves' vectors are no longer
one inclusion after another, so the right-hand sides and the densities pass through the
library's row maps; these tests cover the plane-wave, the general right-hand-side, the
far-field, the refined and the refactorisation paths on such leaves."""
import dataclasses
import functools

import numpy as np
import pytest

from oracle import dense
from paper_2603_09381_amd import workloads as W

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _close():
    """20 random inclusions in a 3.5 x 3.5 box, bounding circles 0.02 apart (N = 3,908)."""
    return W.random_close(m=20, box=3.5, k_ext=6.0)


@functools.lru_cache(maxsize=None)
def _close_ref():
    return dense.solve(_close())


def _solve(pmx, w, **kw):
    import torch
    fac = pmx.Factor(w, pmx.options(w, **kw))
    dens = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    return fac, dens


@pytest.mark.parametrize("near_rule", [1, 2])
@pytest.mark.parametrize("leaf_size", [1, 2, 4])
def test_close_inclusions_against_dense(pmx, leaf_size, near_rule):
    w = dataclasses.replace(_close(), leaf_size=leaf_size, near_rule=near_rule)
    fac, dens = _solve(pmx, w)
    x = pmx.dens_to_numpy(dens, w)
    err = dense.rel_error(x, _close_ref())
    info = fac.info()
    plan = pmx.plan_query(w)
    first = plan[1] if leaf_size > 1 else plan[0]
    print(w.name, "leaf", leaf_size, "rule", near_rule, "vs dense", err, "levels", info.levels,
          "leaves", len(first), "root", info.root_size, flush=True)
    assert err < 5e-9
    # the first compressed level is the plan's leaf level
    assert info.cells[0] == len(first) and info.levels == len(plan) - 1 - (leaf_size > 1)
    assert np.max(np.abs(dense.energy_defect(dense.Geometry(w), x))) < 1e-8


def test_close_inclusions_refined_forms(pmx):
    """FP32 factor at id_tol 1e-3 and the FP64 factor at 1e-6, both refined against the FP64
    operator (whose fast multipole tree is the k-means tree)."""
    w = _close()
    for kw in (dict(precision=1, id_tol=1e-3, ir_tol=1e-10, ir_max_iter=30),
               dict(precision=2, id_tol=1e-6, ir_tol=1e-12)):
        fac, dens = _solve(pmx, w, **kw)
        err = dense.rel_error(pmx.dens_to_numpy(dens, w), _close_ref())
        info = fac.info()
        print("refined", kw, "steps", info.ir_iterations, "residual", info.ir_residual, "vs dense", err, flush=True)
        assert info.ir_residual <= kw["ir_tol"]
        assert err < 1e-8


def test_general_rhs_and_far_field(pmx):
    """A general right-hand side gives the plane-wave solution; the far field of the
    GPU's densities equals the oracle's sum over every inclusion and right-hand side."""
    import torch
    w = _close()
    fac, dens = _solve(pmx, w)
    x = pmx.dens_to_numpy(dens, w)
    f = dense.rhs(dense.Geometry(w), w.angles)
    y = fac.solve(torch.as_tensor(f.T.copy(), device="cuda")).cpu().numpy().T
    assert dense.rel_error(y, x) < 1e-11
    dirs = np.linspace(0, 2 * np.pi, 73)
    ff = fac.far_field(dens, dirs).cpu().numpy().T
    ref = dense.far_field(dense.Geometry(w), x, dirs)
    assert np.abs(ff - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("m,box", [(3, 2.0), (1, 2.0), (5, 2.2)])
def test_few_inclusions(pmx, m, box):
    """All inclusions in one leaf (the top system is that leaf's block), a single
    inclusion, and a root over two leaves."""
    w = W.random_close(m=m, box=box, k_ext=4.0)
    fac, dens = _solve(pmx, w)
    err = dense.rel_error(pmx.dens_to_numpy(dens, w), dense.solve(w))
    print(w.name, "vs dense", err, "levels", fac.info().levels, flush=True)
    assert err < 5e-9


def test_star_grid_with_kmeans_tree(pmx):
    """The grid arrangement of Sec. 4 under the k-means tree and the eta rule."""
    w = dataclasses.replace(W.sub_grid(W.config2(), 4), tree="kmeans", leaf_size=4, near_rule=2, eta=1.0)
    fac, dens = _solve(pmx, w)
    err = dense.rel_error(pmx.dens_to_numpy(dens, w), dense.solve(w))
    print(w.name, "kmeans vs dense", err, "root", fac.info().root_size, flush=True)
    assert err < 5e-9


def test_refactor_with_leaves_of_several_inclusions(pmx):
    """New interior media by replay: the uncompressed inclusion level and the merge into
    the leaves are part of the kept numeric phase."""
    import torch
    w = _close()
    new_k = w.k_int * np.linspace(0.9, 1.25, w.m)
    w2 = dataclasses.replace(w, k_int=new_k)
    fac = pmx.Factor(w, pmx.options(w, refactor=1))
    fac.refactor(new_k)
    x2 = fac.solve_plane_waves(w2.angles)
    torch.cuda.synchronize()
    fresh = pmx.Factor(w2, pmx.options(w2))
    y2 = fresh.solve_plane_waves(w2.angles)
    torch.cuda.synchronize()
    assert torch.equal(x2, y2), float((x2 - y2).abs().max())
    err = dense.rel_error(pmx.dens_to_numpy(x2, w2), dense.solve(w2))
    print("kmeans refactor vs dense", err, flush=True)
    assert err < 5e-9
    fac.close()
    fresh.close()
