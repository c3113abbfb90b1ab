"""GPU parity of the mixed-precision form: complex FP32 primitives (MFMA GEMM, LU, ID), the
dense FP64 operator apply of the refinement residual, and the refined solutions against
the oracle's dense FP64 solve.

Tolerances.  FP32 primitives are compared with FP64 results on the same (rounded) inputs:
sums of k products carry a relative error of about k u32 (u32 = 6e-8), so the GEMM bound
is 4e-7 sqrt(k) relative to the largest |A||B| entry.  The operator apply is FP64 (sums of
N terms of rounding 1e-16): 1e-12 relative.  Refined solutions stop at a relative residual
of 1e-10; with the condition numbers of these systems (~1e3) the error against the dense
solve stays below 1e-8 (the accuracy target), and is typically 1e-10.
"""
import numpy as np
import pytest

from oracle import analytic, dense
from paper_2603_09381_amd import workloads as W

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(4321)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def c64(a):
    return a.astype(np.complex64).astype(np.complex128)


@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1), (0, 2), (1, 0), (2, 0), (2, 2)])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (37, 5, 70), (130, 129, 17), (64, 64, 0), (16, 16, 4), (256, 4, 256),
                                   (300, 7, 600)])
def test_cgemm_fp32(pmx, opa, opb, m, n, k):
    batch = 3
    A = c64(crandn(batch, m, k) if opa == 0 else crandn(batch, k, m))
    B = c64(crandn(batch, k, n) if opb == 0 else crandn(batch, n, k))
    op = {0: lambda X: X, 1: lambda X: np.swapaxes(X, 1, 2), 2: lambda X: np.conj(np.swapaxes(X, 1, 2))}
    ref = op[opa](A) @ op[opb](B)
    got = pmx.probe_zgemm(A, B, opa, opb, fp32=True)
    assert got.dtype == np.complex64
    scale = max(1.0, np.abs(op[opa](np.abs(A)) @ op[opb](np.abs(B))).max())
    assert np.abs(got - ref).max() < 4e-7 * np.sqrt(max(k, 1)) * scale


@pytest.mark.parametrize("variant", [-1, 0, 1, 2])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (31, 3), (100, 40), (257, 7), (120, 70), (1000, 4), (600, 6)])
def test_lu_solve_fp32(pmx, n, nrhs, variant):
    batch = 3
    A = c64(crandn(batch, n, n) + 2 * np.sqrt(n) * np.eye(n))
    B = c64(crandn(batch, n, nrhs))
    _, _, X, info = pmx.probe_lu_solve(A, B, fp32=True, variant=variant)
    assert (info == 0).all()
    ref = np.linalg.solve(A, B)
    # backward stable: residual of the FP32 solution ~ n u32 |A| |x|
    res = np.abs(A @ X.astype(np.complex128) - B).max()
    assert res < 1e-6 * n * np.abs(A).max() * np.abs(ref).max()


def test_lu_tall_panels_fp32(pmx):
    """FP32 panels above 1024 rows (the tall-panel kernel) on unshifted random matrices,
    which pivot at almost every column: backward error of the solution."""
    n, batch = 2100, 2
    A = c64(crandn(batch, n, n))
    B = c64(crandn(batch, n, 2))
    _, piv, X, info = pmx.probe_lu_solve(A, B, fp32=True)
    assert (info == 0).all()
    for b in range(batch):
        assert piv[b].min() >= 0 and piv[b].max() < n and (piv[b] >= np.arange(n)).all()
        res = np.abs(A[b].astype(np.complex128) @ X[b].astype(np.complex128) - B[b]).max()
        assert res < 1e-6 * n * np.abs(A[b]).max() * np.abs(X[b]).max()


def _lowrank(m, c, r, decay):
    U = crandn(m, r)
    V = crandn(r, c)
    return (U * decay ** np.arange(r)) @ V


@pytest.mark.parametrize("m,c", [(300, 60), (60, 60), (1000, 128), (700, 300)])
def test_id_fp32(pmx, m, c):
    batch = 2
    tol = 1e-5
    M = c64(np.stack([_lowrank(m, c, min(m, c), 0.6) for _ in range(batch)]))
    piv, rank, T = pmx.probe_id(M.copy(), tol, fp32=True)
    for b in range(batch):
        k = int(rank[b])
        p = piv[b]
        assert sorted(p) == list(range(c))
        Z = np.zeros((k, c), complex)
        Z[:, p[:k]] = np.eye(k)
        Z[:, p[k:]] = T[b][:k, :c - k]
        res = np.linalg.norm(M[b] - M[b][:, p[:k]] @ Z, 2) / np.linalg.norm(M[b], 2)
        assert res < 1e2 * tol, res
        assert 0.6 ** k < 1e2 * tol and 0.6 ** max(k - 8, 0) > tol * 1e-2, k


@pytest.mark.parametrize("g,n,k,nrhs", [(2, 64, 10.0, 3), (3, 48, 10.0, 3), (4, 48, 45.0, 3), (2, 64, 1.0, 1),
                                        (3, 48, 30.0, 5), (4, 64, 60.0, 16), (3, 48, 10.0, 12)])
def test_dense_apply_against_oracle(pmx, g, n, k, nrhs):
    """k = 45 on a 4x4 grid puts k r between about 20 and 190: every branch of the apply's
    Hankel evaluation (near pairs: series, Chebyshev, 20-term expansion; far pairs: 20-,
    16- and 12-term expansions).  k = 1 makes every inclusion near every wave; 432 nodes
    (3 x 48) leave a partial last wave; 5 and 16 right-hand sides take groups of 4 + 1 and
    8 + 8."""
    w = W.star_grid(g, n=n, k_ext=k, k_int=1.5 * k, seed=5)
    A = dense.assemble(dense.Geometry(w))
    x = crandn(w.n_unknowns, nrhs)
    ref = A @ x
    got = pmx.probe_apply(w, x)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("dense apply rel err", err)
    assert err < 1e-12


def test_dense_apply_scattered_uneven(pmx):
    """Scattered inclusions with uneven node counts: waves straddle inclusions of different
    sizes and the near lists come from bounding circles of mixed radii."""
    w = W.config3(m=14, box=7.0, seed=3)
    A = dense.assemble(dense.Geometry(w))
    x = crandn(w.n_unknowns, 4)
    ref = A @ x
    got = pmx.probe_apply(w, x)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("scattered dense apply rel err", err, "nodes", w.n_unknowns // 2)
    assert err < 1e-12


@pytest.mark.parametrize("g,n,nrhs,nrow", [(12, 16, 2, 96), (16, 128, 4, 48)])
def test_dense_apply_clusters_sampled_rows(pmx, g, n, nrhs, nrow):
    """Grids large enough that the apply takes clusters of 2x2 and 4x4 inclusions through
    translated expansions (the 16x16 grid of 128-node stars is the benchmark's): sampled rows
    of A x against the oracle's on-the-fly row evaluation."""
    w = W.star_grid(g, n=n, k_ext=10.0, k_int=15.0, seed=5)
    w.angles = 2 * np.pi * np.arange(nrhs) / nrhs
    x = crandn(w.n_unknowns, nrhs)
    got = pmx.probe_apply(w, x)
    rows = np.sort(np.random.default_rng(11).choice(w.n_unknowns, size=nrow, replace=False))
    f = dense.rhs(dense.Geometry(w), w.angles)[rows]
    ref = f - dense.residual_rows(w, x, rows)
    err = np.abs(got[rows] - ref).max() / np.abs(ref).max()
    print("cluster apply rel err", err, "N", w.n_unknowns)
    assert err < 1e-12


def _mixed(pmx, w, **kw):
    import torch
    o = pmx.options(w, precision=1, id_tol=kw.pop("id_tol", 1e-6), **kw)
    fac = pmx.Factor(w, o)
    dens = fac.solve_plane_waves(w.angles)
    torch.cuda.synchronize()
    return fac, pmx.dens_to_numpy(dens, w)


def test_mixed_cfg1_against_dense_and_multipole(pmx):
    w = W.config1()
    fac, x = _mixed(pmx, w)
    ref = dense.solve(w)
    info = fac.info()
    print("cfg1 mixed: iters", info.ir_iterations, "res", info.ir_residual, "err", dense.rel_error(x, ref))
    assert info.ir_residual <= 1e-10
    assert dense.rel_error(x, ref) < 1e-9
    g = dense.Geometry(w)
    bnd, _, _ = analytic.multi_disk(w.centers, 0.4, w.k_ext, w.k_int[0], g.eps_p, g.eps_m[0])
    th = 2 * np.pi * np.arange(64) / 64
    mref = np.concatenate([np.concatenate(bnd(j, th)) for j in range(4)])
    assert dense.rel_error(x[:, 0], mref) < 5e-9


@pytest.mark.parametrize("g", [2, 4])
def test_mixed_star_grid_against_dense(pmx, g):
    w = W.sub_grid(W.config2(), g)
    fac, x = _mixed(pmx, w)
    ref = dense.solve(w)
    err = dense.rel_error(x, ref)
    info = fac.info()
    print(w.name, "mixed: iters", info.ir_iterations, "res", info.ir_residual, "err", err, "root", info.root_size)
    assert info.ir_residual <= 1e-10 and info.ir_iterations >= 2
    assert err < 1e-8
    assert np.max(np.abs(dense.energy_defect(dense.Geometry(w), x))) < 1e-8


def test_mixed_general_rhs(pmx):
    import torch
    w = W.sub_grid(W.config2(), 2)
    fac, x = _mixed(pmx, w)
    f = dense.rhs(dense.Geometry(w), w.angles)
    y = fac.solve(torch.as_tensor(f.T.copy(), device="cuda")).cpu().numpy().T
    assert dense.rel_error(y, dense.solve(w)) < 1e-8


def test_mixed_reports_nonconvergence(pmx):
    w = W.sub_grid(W.config2(), 2)
    o = pmx.options(w, precision=1, id_tol=1e-4, ir_max_iter=1, ir_tol=1e-14)
    fac = pmx.Factor(w, o)
    with pytest.raises(pmx.PmxError) as e:
        fac.solve_plane_waves(w.angles)
    assert e.value.status == 6
    assert fac.info().ir_iterations == 1 and fac.info().ir_residual > 1e-14


def test_mixed_scattered_uneven_against_dense(pmx):
    w = W.config3(m=14, box=7.0, seed=3)
    fac, x = _mixed(pmx, w)
    info = fac.info()
    err = dense.rel_error(x, dense.solve(w))
    print(w.name, "mixed: iters", info.ir_iterations, "res", info.ir_residual, "err", err)
    assert info.ir_residual <= 1e-10 and err < 1e-8


def test_stars16_tuned_and_plain_against_tight_reference(pmx):
    """The 16x16 grid of stars (N = 65,536, four plane waves): the tuned form (FP32 factor
    at ID tolerance 1e-3 refined to 1e-10) and the plain FP64 form (1e-10) against the plain
    FP64 solve at ID tolerance 1e-12, by the relative 2-norm error over every entry (Sec.
    4.2); the oracle's FP64 rows f - A x on sampled rows back the reference itself."""
    import torch
    w = W.config2()
    out = {}
    for name, kw in (("ref", dict(precision=0, id_tol=1e-12)), ("plain", dict(precision=0, id_tol=1e-10)),
                     ("tuned", dict(precision=1, id_tol=1e-3, ir_tol=1e-10))):
        print("stars16 form", name, flush=True)
        fac = pmx.Factor(w, pmx.options(w, **kw))
        out[name] = fac.solve_plane_waves(w.angles)
        torch.cuda.synchronize()
        fac.close()
    ref = out["ref"]
    errs = {k: float(torch.linalg.norm(out[k] - ref) / torch.linalg.norm(ref)) for k in ("plain", "tuned")}
    rows = np.sort(np.random.default_rng(3).choice(w.n_unknowns, size=12, replace=False))
    f = dense.rhs(dense.Geometry(w), w.angles)[rows]
    res = {k: float(np.linalg.norm(dense.residual_rows(w, pmx.dens_to_numpy(out[k], w), rows)) / np.linalg.norm(f))
           for k in ("ref", "tuned")}
    print("stars16 rel error vs reference", errs, "oracle sampled residual", res)
    assert errs["plain"] <= 1e-8 and errs["tuned"] <= 1e-8
    assert res["ref"] <= 1e-10 and res["tuned"] <= 1e-9


def test_dense_apply_fast_multipole_sixteen_rhs(pmx):
    """The benchmark's shape of the apply: 32x32 stars at k+ = 8 with sixteen right-hand
    sides (translations on three tree levels, near groups of eight, expansion groups), on
    sampled rows against the oracle's FP64 row evaluation."""
    w = W.star_grid(32, n=128, k_ext=8.0, k_int=12.0, seed=4)
    w.angles = 2 * np.pi * np.arange(16) / 16
    st = pmx.apply_structure(w)
    assert st["m2l_pairs"] > 1000 and st["l2l_pairs"] > 100
    x = crandn(w.n_unknowns, 16)
    got = pmx.probe_apply(w, x)
    rows = np.sort(np.random.default_rng(12).choice(w.n_unknowns, size=10, replace=False))
    f = dense.rhs(dense.Geometry(w), w.angles)[rows]
    ref = f - dense.residual_rows(w, x, rows)
    err = np.abs(got[rows] - ref).max() / np.abs(ref).max()
    print("fast multipole apply rel err", err, "N", w.n_unknowns, st)
    assert err < 1e-12
