"""General arrangements (Sec. 4.4, Discussions): the k-means tree, the eta-admissibility near
rule and leaves of several inclusions.  Host only (no GPU).

The oracle's k-means is pinned to scikit-learn's Lloyd iteration started from the same
seeds, to the textbook case of well-separated groups and to the fixed-point property of
Lloyd's method; the library's plan is then compared with the oracle's bit for bit, and the
plan's invariants (a partition at every level, nested cells, leaf sizes, the near rule
and the proxy circles' separation) are checked by brute force."""
import ctypes as C
import dataclasses
import math

import numpy as np
import pytest

from oracle import fast
from paper_2603_09381_amd import pmx
from paper_2603_09381_amd import workloads as W


def _kmeans_workload(w, leaf_size=4, near_rule=2, eta=1.0):
    return dataclasses.replace(w, tree="kmeans", leaf_size=leaf_size, near_rule=near_rule, eta=eta)


CASES = [
    ("close20_l4_eta1", lambda: W.random_close(m=20, box=3.5, k_ext=6.0)),
    ("close60_l2_eta0.5", lambda: _kmeans_workload(W.random_close(m=60, box=7.0, k_ext=6.0), 2, 2, 0.5)),
    ("close60_l1_geom", lambda: _kmeans_workload(W.random_close(m=60, box=7.0, k_ext=6.0), 1, 1)),
    ("scattered40_l3_eta2", lambda: _kmeans_workload(W.config3(m=40, box=12.0, seed=5), 3, 2, 2.0)),
    ("stars6x6_l4", lambda: _kmeans_workload(W.star_grid(6, n=64))),
    ("three_in_one_leaf", lambda: W.random_close(m=3, box=2.0, k_ext=4.0)),
    ("single", lambda: W.random_close(m=1, box=2.0, k_ext=4.0)),
]


@pytest.mark.parametrize("make", [c[1] for c in CASES], ids=[c[0] for c in CASES])
def test_kmeans_plan_matches_oracle_exactly(make):
    """Membership, children, centres, radii, proxy radius and count and near lists of every
    cell of every level: the library's plan equals the oracle's bit for bit."""
    w = make()
    got = pmx.plan_query(w)
    ref = fast.plan(w)
    assert [len(l) for l in got] == [len(l) for l in ref]
    for lg, lr in zip(got, ref):
        for cg, cr in zip(lg, lr):
            assert cg["incl"] == cr.incl and cg["children"] == cr.children
            assert cg["center"] == cr.center and cg["rc"] == cr.rc
            assert cg["Rp"] == cr.Rp and cg["P"] == cr.P
            assert cg["near"] == list(cr.near)


def _points(w):
    px, py, wt = fast.node_means(w)
    return np.array(px), np.array(py), np.array(wt)


def test_node_means_are_the_node_centroids():
    w = W.random_close(m=12, box=3.0, k_ext=4.0)
    px, py, wt = _points(w)
    for j in range(w.m):
        a, b = w.node_off[j], w.node_off[j + 1]
        assert wt[j] == b - a
        assert abs(px[j] - np.mean(w.x[a:b])) < 1e-14 and abs(py[j] - np.mean(w.y[a:b])) < 1e-14


def _seeds(S, px, py, wt, k):
    """The seeds of the split, recomputed independently (numpy, vectorised)."""
    P = np.stack([px[S], py[S]], 1)
    mean = (wt[S, None] * P).sum(0) / wt[S].sum()
    idx = [int(np.argmax(((P - mean) ** 2).sum(1)))]
    while len(idx) < k:
        d = np.min(((P[:, None, :] - P[idx][None, :, :]) ** 2).sum(2), axis=1)
        idx.append(int(np.argmax(d)))
    return P[idx]


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_kmeans_split_equals_sklearn_lloyd(seed):
    """One split equals scikit-learn's weighted Lloyd k-means started from the same seeds
    (same partition)."""
    from sklearn.cluster import KMeans
    w = W.random_close(m=120, box=12.0, k_ext=6.0, seed=seed)
    px, py, wt = _points(w)
    S = list(range(w.m))
    parts = fast.kmeans_split(S, list(px), list(py), list(wt))
    init = _seeds(np.array(S), px, py, wt, 4)
    km = KMeans(n_clusters=4, init=init, n_init=1, algorithm="lloyd", tol=0.0, max_iter=300)
    lab = km.fit(np.stack([px, py], 1), sample_weight=wt).labels_
    mine = {frozenset(p) for p in parts}
    theirs = {frozenset(np.flatnonzero(lab == c).tolist()) for c in range(4)}
    assert mine == theirs


def test_kmeans_split_finds_separated_groups():
    """Four tight groups far apart: the split returns exactly the groups."""
    w = W.random_close(m=16, box=2.2, k_ext=4.0, seed=3)
    shifts = [(0, 0), (40, 0), (0, 40), (40, 40)]
    groups = [list(range(4 * q, 4 * q + 4)) for q in range(4)]
    px, py, wt = _points(w)
    px, py = px.copy(), py.copy()
    for q, (sx, sy) in enumerate(shifts):
        px[groups[q]] += sx
        py[groups[q]] += sy
    parts = fast.kmeans_split(list(range(16)), list(px), list(py), list(wt))
    assert sorted(map(sorted, parts)) == sorted(groups)


def test_kmeans_split_is_a_lloyd_fixed_point():
    """Every member is nearest to the weighted mean of its own cluster."""
    w = W.random_close(m=200, box=16.0, k_ext=6.0, seed=11)
    px, py, wt = _points(w)
    S = list(range(w.m))
    parts = fast.kmeans_split(S, list(px), list(py), list(wt))
    cen = np.array([[np.sum(wt[p] * px[p]) / np.sum(wt[p]), np.sum(wt[p] * py[p]) / np.sum(wt[p])] for p in parts])
    for c, p in enumerate(parts):
        for j in p:
            d = (cen[:, 0] - px[j]) ** 2 + (cen[:, 1] - py[j]) ** 2
            assert d[c] <= d.min() * (1 + 1e-12)


@pytest.mark.parametrize("make", [c[1] for c in CASES[:5]], ids=[c[0] for c in CASES[:5]])
def test_kmeans_plan_invariants(make):
    """Partition at every level, nested cells, leaves within leaf_size, every pair the
    eta rule calls near in the near lists, own nodes inside and far nodes outside every
    proxy circle."""
    w = make()
    lv = fast.plan(w)
    g = fast.dense.Geometry(w)
    L = w.leaf_size
    passthrough = L > 1
    for l, cells in enumerate(lv):
        allin = sorted(j for c in cells for j in c.incl)
        assert allin == list(range(w.m)), l
        if l > 0:
            for c in cells:
                assert sorted(j for ch in c.children for j in lv[l - 1][ch].incl) == c.incl
                assert 1 <= len(c.children) <= 4
    leaves = lv[1] if passthrough else lv[0]
    assert all(1 <= len(c.incl) <= L for c in leaves)
    assert all(len(c.incl) == 1 for c in lv[0])
    for l, cells in enumerate(lv):
        if len(cells) == 1 or (l == 0 and passthrough):
            continue
        pts = [fast._cell_nodes(g, c) for c in cells]
        for t, c in enumerate(cells):
            if w.near_rule == 2:
                for s, o in enumerate(cells):
                    if s != t and w.eta * math.dist(c.center, o.center) < 2 * max(c.rc, o.rc):
                        assert s in c.near, (l, t, s)
            if c.P == 0:
                assert len(c.near) == len(cells) - 1
                continue
            own = np.hypot(pts[t][0] - c.center[0], pts[t][1] - c.center[1])
            assert own.max() < c.Rp
            for s in range(len(cells)):
                if s != t and s not in c.near:
                    far = np.hypot(pts[s][0] - c.center[0], pts[s][1] - c.center[1])
                    assert far.min() > c.Rp, (l, t, s)


def test_eta_rule_grows_near_lists_as_eta_falls():
    """A smaller eta calls more pairs near: each near list at eta = 0.5 contains the one at
    eta = 2 (same tree)."""
    base = W.random_close(m=60, box=7.0, k_ext=6.0)
    a = fast.plan(dataclasses.replace(base, eta=2.0))
    b = fast.plan(dataclasses.replace(base, eta=0.5))
    more = 0
    for la, lb in zip(a, b):
        for ca, cb in zip(la, lb):
            assert set(ca.near) <= set(cb.near)
            more += len(cb.near) - len(ca.near)
    assert more > 0


def _create_opts(w, **okw):
    lib = pmx.load()
    keep = pmx._GeomKeep(w)
    o = pmx.options(w, **okw)
    h = C.c_void_p()
    st = lib.pmx_factor_create(C.byref(keep.g), C.byref(o), None, C.byref(h))
    if st == 0:
        lib.pmx_factor_destroy(h)
    return st, lib.pmx_last_error().decode()


@pytest.mark.parametrize("kw,want", [
    (dict(near_rule=0), "near_rule 1 or 2"),
    (dict(leaf_size=5), "leaf_size"),
    (dict(leaf_size=0), "leaf_size"),
    (dict(eta=0.0), "eta"),
    (dict(eta=float("nan")), "eta"),
    (dict(learned=1), "tree 0"),
    (dict(tree=2), "tree must be"),
    (dict(near_rule=3), "near_rule must be"),
])
def test_kmeans_options_are_validated(kw, want):
    """Bad tree options are argument errors, found before any device work."""
    st, msg = _create_opts(W.random_close(m=8, box=2.5, k_ext=4.0), **kw)
    assert st == 1 and want in msg, msg


def test_apply_structure_with_kmeans_tree():
    """The refinement's operator apply over the k-means tree's clusters takes every (wave,
    source inclusion) pair exactly once."""
    w = W.random_close(m=60, box=7.0, k_ext=6.0)
    st = pmx.apply_structure(w, check=True)
    assert st["pairs_checked"] == st["waves"] * w.m
    assert st["coverage_violations"] == 0


def test_large_plans_of_several_inclusions_per_leaf_are_refused():
    """Leaves of several inclusions are accepted up to 512 leaves; a larger plan is an
    argument error reported before any device work, while one inclusion per leaf has no
    such limit."""
    base = W.random_close(m=1600, box=32.0)
    w = dataclasses.replace(base, leaf_size=2)
    assert len(pmx.plan_query(w)[1]) > 512
    st, msg = _create_opts(w)
    assert st == 1 and "up to 512 leaves" in msg, msg
    st, msg = _create_opts(dataclasses.replace(base, leaf_size=1))
    assert st != 1, msg
