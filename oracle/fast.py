"""Proxy + interpolative-decomposition recursive direct solver, plain CPU (oracle).

TEST INFRASTRUCTURE ONLY.  Written step by step in the order of Sec. 3, for step
level comparison and rank statistics; the pass/fail reference for solutions is
the dense solve in ``dense``.

Sec. 3 in brief.  Every off-diagonal block is low rank (weak admissibility):
A_ij ~ L_i S_ij R_j with S_ij = A(rskel_i, cskel_j) a sub-matrix of A and L, R
block diagonal with one block per density type (eq. low_rank_block_linear and the
sub-matrix structure after it).  The skeletons and interpolation matrices come
from the proxy method and an interpolative decomposition by column-pivoted QR with
adaptive rank (diagonal of R above a threshold).  With At_i = (R_i A_ii^-1 L_i)^-1
the system becomes the compressed system of eq. compressed in the unknowns
psi_i = R_i phi_i, and phi is recovered from psi by the recovery formula; applied
recursively up a tree of cells (children skeletons merge into parents) this gives
the multi-level solver, with the top compressed system solved by partial pivoted
LU (Sec. 4).

Readings where the paper is silent (listed in the design notes):
  * four IDs per cell, one per density type: q-columns, u-columns, value rows,
    derivative rows; q pairs with value rows and u with derivative rows and both
    members of a pair keep k = max of their two threshold ranks, so At is square;
  * threshold rank: |R_jj| > tol * |R_11|;
  * quadtree over grid coordinates, four Morton children per parent;
  * near cells: the four edge-adjacent cells of the same level (Sec. 4), plus any
    same-level cell with a node inside the proxy circle; the circle is centred at
    the mean of the cell's inclusion centres, radius max(ratio r_c, 0.9 rho_far)
    with r_c the farthest own node and rho_far the nearest node of a far cell;
  * proxy rows (column ID): value and normal derivative of each source's field at
    the proxy points; proxy columns (row ID): single and double layer sources at
    the proxy points with the trapezoid weight 2 pi R_p / P; exterior kernel only
    (the Omit property, Sec. 2.1);
  * number of proxy points P = max(P_min, 2 ceil(k+ R_p) + 2 ceil(ln tol / ln(r_c/rho_far)) + 16),
    or a fixed P when the workload fixes it; no proxy when no cell is far.

General arrangements (Sec. 4.4, Discussions): cells from a k-means clustering, near pairs
by eta-admissibility, several inclusions per leaf.  Readings (``kmeans_plan``):
  * the clustered points are the inclusions, each at the mean of its nodes with its node
    count as weight (k-means of the integration points with no inclusion split); four
    clusters per split, depth by depth, while some cell of the depth holds more than
    leaf_size inclusions (cells within the limit continue as single children);
  * seeds: the member farthest from the weighted mean, then repeatedly the member
    farthest from all seeds so far; Lloyd steps (nearest seed, then weighted means) until
    no member changes cluster, at most 100;
  * near when eta times the distance of the centres is below the larger of the two
    diameters 2 r_c, then the same proxy-circle closure as above;
  * with leaf_size > 1 the inclusions form level 0 and the leaves level 1; level 0 is not
    compressed (the leaves' blocks hold their inclusions' self blocks and the exterior
    blocks between them) and has no near lists.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as la

from . import dense, layer


def morton(i, j):
    code = 0
    for b in range(32):
        code |= ((i >> b) & 1) << (2 * b)
        code |= ((j >> b) & 1) << (2 * b + 1)
    return code


@dataclass
class Cell:
    level: int
    coord: tuple
    incl: list                      # inclusion indices (ascending)
    children: list = field(default_factory=list)   # indices into the level below
    center: tuple = (0.0, 0.0)
    rc: float = 0.0
    near: list = field(default_factory=list)
    rho_far: float = math.inf
    Rp: float = 0.0
    P: int = 0


def grid_assignment(centers):
    """Integer cells for scattered inclusions (reading of Sec. 4's general arrangements as
    an adaptive quadtree with at most one inclusion per leaf): a uniform grid of spacing
    h = 0.99 d_min / sqrt(2), d_min the smallest distance between two centres, so that no
    cell holds two centres (a cell's diagonal is shorter than d_min); the quadtree over
    the occupied cells then prunes the empty ones."""
    c = np.asarray(centers, dtype=float)
    m = len(c)
    if m == 1:
        return np.zeros((1, 2), dtype=np.int64)
    d2 = math.inf
    for i in range(m):
        for j in range(i + 1, m):
            dx = float(c[i, 0]) - float(c[j, 0])
            dy = float(c[i, 1]) - float(c[j, 1])
            d2 = min(d2, dx * dx + dy * dy)
    h = 0.99 * math.sqrt(d2 / 2.0)
    x0 = float(np.min(c[:, 0]))
    y0 = float(np.min(c[:, 1]))
    out = np.zeros((m, 2), dtype=np.int64)
    for i in range(m):
        out[i, 0] = math.floor((float(c[i, 0]) - x0) / h)
        out[i, 1] = math.floor((float(c[i, 1]) - y0) / h)
    return out


def node_means(w):
    """Per inclusion: the mean of its nodes (plain left-to-right sums) and its node count."""
    px, py, wt = [], [], []
    for j in range(w.m):
        a, b = int(w.node_off[j]), int(w.node_off[j + 1])
        sx = sy = 0.0
        for i in range(a, b):
            sx += float(w.x[i])
            sy += float(w.y[i])
        n = float(b - a)
        px.append(sx / n)
        py.append(sy / n)
        wt.append(n)
    return px, py, wt


def kmeans_split(S, px, py, wt):
    """Weighted k-means of the inclusions S into at most four clusters (readings in the
    module header): clusters in seed order, members in the order of S, empty ones dropped."""
    n = len(S)
    k = min(4, n)
    sx = sy = sw = 0.0
    for j in S:
        sx += wt[j] * px[j]
        sy += wt[j] * py[j]
        sw += wt[j]
    mx, my = sx / sw, sy / sw
    best, bd = 0, -1.0
    for i, j in enumerate(S):
        dx, dy = px[j] - mx, py[j] - my
        d = dx * dx + dy * dy
        if d > bd:
            best, bd = i, d
    cx, cy = [px[S[best]]], [py[S[best]]]
    dmin = [math.inf] * n
    while len(cx) < k:
        best, bd = -1, 0.0
        for i, j in enumerate(S):
            dx, dy = px[j] - cx[-1], py[j] - cy[-1]
            dmin[i] = min(dmin[i], dx * dx + dy * dy)
            if dmin[i] > bd:
                best, bd = i, dmin[i]
        if best < 0:
            break
        cx.append(px[S[best]])
        cy.append(py[S[best]])
    kk = len(cx)
    a = [-1] * n
    for _ in range(100):
        moved = False
        for i, j in enumerate(S):
            b, bd = 0, math.inf
            for c in range(kk):
                dx, dy = px[j] - cx[c], py[j] - cy[c]
                d = dx * dx + dy * dy
                if d < bd:
                    b, bd = c, d
            if b != a[i]:
                a[i] = b
                moved = True
        if not moved:
            break
        for c in range(kk):
            sx = sy = sw = 0.0
            for i, j in enumerate(S):
                if a[i] == c:
                    sx += wt[j] * px[j]
                    sy += wt[j] * py[j]
                    sw += wt[j]
            if sw > 0:
                cx[c], cy[c] = sx / sw, sy / sw
    out = [[j for i, j in enumerate(S) if a[i] == c] for c in range(kk)]
    return [q for q in out if q]


def kmeans_plan(w):
    """Tree of Sec. 4.4's general arrangements (readings in the module header)."""
    g = dense.Geometry(w)
    L = int(w.leaf_size)
    if not 1 <= L <= 4:
        raise ValueError("leaf_size must be in 1..4")
    px, py, wt = node_means(w)
    depth, parent = [[list(range(w.m))]], [[-1]]
    while any(len(c) > L for c in depth[-1]):
        nxt, par = [], []
        for t, c in enumerate(depth[-1]):
            parts = kmeans_split(c, px, py, wt) if len(c) > L else [c]
            if len(c) > L and len(parts) < 2:
                raise ValueError("inclusions whose node means coincide")
            for q in parts:
                nxt.append(q)
                par.append(t)
        depth.append(nxt)
        parent.append(par)
    D = len(depth) - 1
    passthrough = L > 1
    l0, first = [], []
    for c in depth[D]:
        first.append(len(l0))
        l0.extend(Cell(0, (0, 0), [j]) for j in c)
    first.append(len(l0))
    levels = [l0]
    for d in range(D if passthrough else D - 1, -1, -1):
        cells = [Cell(len(levels), (0, 0), sorted(c)) for c in depth[d]]
        if d == D:
            for t, cell in enumerate(cells):
                cell.children = list(range(first[t], first[t + 1]))
        else:
            for q, p in enumerate(parent[d + 1]):
                cells[p].children.append(q)
        levels.append(cells)
    for lev, cells in enumerate(levels):
        _near_and_proxy(w, g, cells, lists=not (lev == 0 and passthrough))
    return levels


def plan(w):
    """Tree, near lists and proxy circles for every level (grid workloads; scattered ones
    through grid_assignment; the k-means tree when the workload asks for it)."""
    if getattr(w, "tree", "quad") == "kmeans":
        return kmeans_plan(w)
    g = dense.Geometry(w)
    gi = np.asarray(w.grid_index) if w.grid_index is not None else grid_assignment(w.centers)
    levels = []
    cur = {}
    for j in range(w.m):
        cur.setdefault((int(gi[j, 0]), int(gi[j, 1])), []).append(j)
    lev = 0
    prev = None
    while True:
        keys = sorted(cur.keys(), key=lambda c: morton(c[0], c[1]))
        cells = [Cell(lev, c, sorted(cur[c])) for c in keys]
        if prev is not None:
            index = {c.coord: t for t, c in enumerate(prev)}
            for cell in cells:
                I, J = cell.coord
                for b in range(2):
                    for a in range(2):
                        cc = (2 * I + a, 2 * J + b)
                        if cc in index:
                            cell.children.append(index[cc])
        levels.append(cells)
        if len(cells) == 1:
            break
        nxt = {}
        for c in cells:
            nxt.setdefault((c.coord[0] >> 1, c.coord[1] >> 1), []).extend(c.incl)
        cur = nxt
        prev = cells
        lev += 1
    for cells in levels:
        _near_and_proxy(w, g, cells)
    return levels


def _cell_nodes(g, cell):
    idx = np.concatenate([np.arange(g.off[j], g.off[j + 1]) for j in cell.incl])
    return g.x[idx], g.y[idx]


def _near_and_proxy(w, g, cells, lists=True):
    pts = [_cell_nodes(g, c) for c in cells]
    for c in cells:
        sx = sy = 0.0
        for j in c.incl:                      # plain left-to-right sums
            sx += float(w.centers[j, 0])
            sy += float(w.centers[j, 1])
        c.center = (sx / len(c.incl), sy / len(c.incl))
    for t, c in enumerate(cells):
        px, py = pts[t]
        c.rc = float(np.max(np.hypot(px - c.center[0], py - c.center[1])))
    if len(cells) == 1 or not lists:
        return
    for t, c in enumerate(cells):
        dmin = np.array([np.min(np.hypot(pts[s][0] - c.center[0], pts[s][1] - c.center[1]))
                         if s != t else math.inf for s in range(len(cells))])
        near = set()
        if w.near_rule == 0:
            for s, o in enumerate(cells):
                if s != t and abs(o.coord[0] - c.coord[0]) + abs(o.coord[1] - c.coord[1]) == 1:
                    near.add(s)
        if w.near_rule == 2:   # eta-admissibility (Sec. 4.4): diameters 2 r_c
            for s, o in enumerate(cells):
                ex, ey = o.center[0] - c.center[0], o.center[1] - c.center[1]
                if s != t and w.eta * math.sqrt(ex * ex + ey * ey) < 2.0 * max(c.rc, o.rc):
                    near.add(s)
        while True:
            far = [s for s in range(len(cells)) if s != t and s not in near]
            rho = float(min(dmin[s] for s in far)) if far else math.inf
            if w.proxy_paper_rule and far:
                Rp = max(w.proxy_ratio * c.rc, 0.9 * rho)
            else:
                Rp = w.proxy_ratio * c.rc
            add = [s for s in far if dmin[s] <= Rp]
            if not add:
                break
            near.update(add)
        c.near = sorted(near)
        c.rho_far = rho
        if far:
            c.Rp = Rp
            if w.proxy_paper_rule:
                q = min(c.rc / rho, 0.95)
                P = 2 * math.ceil(w.k_ext * Rp) + 2 * math.ceil(math.log(w.id_tol) / math.log(q)) + 16
                c.P = max(int(w.proxy_min), P)
            else:
                c.P = int(w.proxy_min)
        else:
            c.Rp, c.P = 0.0, 0


def proxy_points(c: Cell):
    th = 2.0 * np.pi * np.arange(c.P) / c.P
    return (c.center[0] + c.Rp * np.cos(th), c.center[1] + c.Rp * np.sin(th),
            np.cos(th), np.sin(th), np.full(c.P, 2.0 * np.pi * c.Rp / c.P))


class Points:
    """A list of (position, normal, weight, type) used as matrix rows or columns."""

    def __init__(self, x, y, nx, ny, wt, typ):
        self.x, self.y, self.nx, self.ny = map(np.asarray, (x, y, nx, ny))
        self.wt = np.asarray(wt)
        self.typ = np.asarray(typ, dtype=int)

    def __len__(self):
        return len(self.x)

    @staticmethod
    def cat(items):
        return Points(*[np.concatenate([getattr(p, a) for p in items])
                        for a in ("x", "y", "nx", "ny", "wt", "typ")])


def entries(w, g, rows: Points, cols: Points):
    """Off-diagonal matrix entries of the Omit form between disjoint point sets:
    row type 0 = value equation, 1 = normal-derivative equation; column type 0 = q,
    1 = u; the column's quadrature weight multiplies the kernel."""
    with np.errstate(invalid="ignore", divide="ignore"):
        S, D, Ds, N = layer.kernel_blocks(rows.x, rows.y, rows.nx, rows.ny,
                                          cols.x, cols.y, cols.nx, cols.ny, w.k_ext)
    ep = g.eps_p
    rt = rows.typ[:, None]
    ct = cols.typ[None, :]
    out = np.where(rt == 0, np.where(ct == 0, -ep * S, D), np.where(ct == 0, -Ds, N / ep))
    return out * cols.wt[None, :]


def node_points(g, nodes, typ):
    nodes = np.asarray(nodes, dtype=int)
    return Points(g.x[nodes], g.y[nodes], g.nx[nodes], g.ny[nodes], g.wt[nodes], typ)


def cpqr_id(M, tol):
    """Column-pivoted QR (LAPACK geqp3); threshold rank |R_jj| > tol |R_11| (Sec. 3)."""
    R, piv = la.qr(M, mode="r", pivoting=True)
    d = np.abs(np.diag(R))
    if d.size == 0 or d[0] == 0.0:
        return R, piv, 0
    rank = int(np.sum(d > tol * d[0]))
    return R, piv, rank


def interp_matrix(R, piv, k, c):
    """Z (k x c) with M[:, piv[:k]] Z ~ M: Z[:, piv[:k]] = I, Z[:, piv[k:]] = R11^-1 R12."""
    Z = np.zeros((k, c), dtype=complex)
    Z[:, piv[:k]] = np.eye(k)
    if k < c:
        T = la.solve_triangular(R[:k, :k], R[:k, k:c])
        Z[:, piv[k:]] = T
    return Z


@dataclass
class Active:
    rows: np.ndarray     # node index per active row
    rtyp: np.ndarray     # 0 value row, 1 derivative row
    cols: np.ndarray
    ctyp: np.ndarray


class FastSolver:
    """Multi-level proxy + ID solver of the Omit system, all in FP64 numpy."""

    def __init__(self, w, tol=None):
        self.w = w
        self.g = dense.Geometry(w)
        self.tol = w.id_tol if tol is None else tol
        if getattr(w, "tree", "quad") == "kmeans" and int(w.leaf_size) > 1:
            raise NotImplementedError("the oracle's step-level solver takes one inclusion per leaf; "
                                      "leaves of several inclusions are checked against the dense solve")
        self.levels = plan(w)
        self.data = []          # per level: list of dicts per cell
        self._factor()

    # -- level 0 active sets: every node of the inclusion, value rows then derivative rows
    def _leaf_active(self, cell):
        g = self.g
        nodes = np.concatenate([np.arange(g.off[j], g.off[j + 1]) for j in cell.incl])
        n = len(nodes)
        both = np.concatenate([nodes, nodes])
        typ = np.concatenate([np.zeros(n, int), np.ones(n, int)])
        return Active(both, typ, both.copy(), typ.copy())

    def _row_points(self, act, sel=None):
        sel = slice(None) if sel is None else sel
        return node_points(self.g, act.rows[sel], act.rtyp[sel])

    def _col_points(self, act, sel=None):
        sel = slice(None) if sel is None else sel
        return node_points(self.g, act.cols[sel], act.ctyp[sel])

    def _id_matrices(self, cell, act, acts_level, cells):
        """The two column-ID and two (transposed) row-ID matrices of one cell."""
        w, g = self.w, self.g
        near_rows = [self._row_points(acts_level[s]) for s in cell.near]
        near_cols = [self._col_points(acts_level[s]) for s in cell.near]
        if cell.P > 0:
            px, py, pnx, pny, pw = proxy_points(cell)
            P = cell.P
            prow = Points(np.tile(px, 2), np.tile(py, 2), np.tile(pnx, 2), np.tile(pny, 2),
                          np.ones(2 * P), np.repeat([0, 1], P))
            pcol = Points(np.tile(px, 2), np.tile(py, 2), np.tile(pnx, 2), np.tile(pny, 2),
                          np.tile(pw, 2), np.repeat([0, 1], P))
            near_rows.append(prow)
            near_cols.append(pcol)
        out = {}
        tgt = Points.cat(near_rows) if near_rows else None
        src = Points.cat(near_cols) if near_cols else None
        for b in (0, 1):
            csel = act.ctyp == b
            rsel = act.rtyp == b
            out[("col", b)] = entries(w, g, tgt, self._col_points(act, csel))
            out[("row", b)] = entries(w, g, self._row_points(act, rsel), src).T
        return out

    def _factor(self):
        w, g = self.w, self.g
        acts = [self._leaf_active(c) for c in self.levels[0]]
        Dmats = [dense.diagonal_block(g, c.incl[0]) if len(c.incl) == 1 else None
                 for c in self.levels[0]]
        for lev, cells in enumerate(self.levels):
            if lev > 0:
                acts, Dmats = self._merge(lev, cells)
            if len(cells) == 1:
                self.root = dict(act=acts[0], D=Dmats[0], lu=la.lu_factor(Dmats[0]))
                break
            info = []
            for t, cell in enumerate(cells):
                act = acts[t]
                mats = self._id_matrices(cell, act, acts, cells)
                ids = {key: cpqr_id(M, self.tol) for key, M in mats.items()}
                sb = [int(np.sum(act.ctyp == b)) for b in (0, 1)]
                ks = []
                for b in (0, 1):
                    cap = min(sb[b], mats[("col", b)].shape[0])
                    kb = max(ids[("col", b)][2], ids[("row", b)][2])
                    ks.append(max(1, min(kb, cap)))
                Zc = [interp_matrix(ids[("col", b)][0], ids[("col", b)][1], ks[b], sb[b]) for b in (0, 1)]
                Zr = [interp_matrix(ids[("row", b)][0], ids[("row", b)][1], ks[b], sb[b]) for b in (0, 1)]
                Rm = la.block_diag(*Zc)              # K x s  (columns ordered type 0 then 1)
                Lm = la.block_diag(*Zr).T            # s x K  (rows ordered type 0 then 1)
                D = Dmats[t]
                lu = la.lu_factor(D)
                Y = la.lu_solve(lu, Lm)
                Mk = Rm @ Y
                At = np.linalg.inv(Mk)
                ccols = [np.flatnonzero(act.ctyp == b)[ids[("col", b)][1][:ks[b]]] for b in (0, 1)]
                crows = [np.flatnonzero(act.rtyp == b)[ids[("row", b)][1][:ks[b]]] for b in (0, 1)]
                info.append(dict(act=act, lu=lu, Y=Y, R=Rm, L=Lm, At=At, k=ks,
                                 ranks={key: v[2] for key, v in ids.items()},
                                 cskel=ccols, rskel=crows, D=D))
            self.data.append(info)

    def _merge(self, lev, cells):
        """Parent active sets (children skeletons, type 0 first) and parent blocks."""
        w, g = self.w, self.g
        below = self.data[lev - 1]
        acts, Dmats = [], []
        for cell in cells:
            rows, rtyp, cols, ctyp, owner_r, loc_r, owner_c, loc_c = [], [], [], [], [], [], [], []
            for b in (0, 1):
                for ch in cell.children:
                    d = below[ch]
                    kb = d["k"][b]
                    base = 0 if b == 0 else d["k"][0]
                    rows.append(d["act"].rows[d["rskel"][b]]); rtyp.append(np.full(kb, b))
                    cols.append(d["act"].cols[d["cskel"][b]]); ctyp.append(np.full(kb, b))
                    owner_r.append(np.full(kb, ch)); loc_r.append(base + np.arange(kb))
                    owner_c.append(np.full(kb, ch)); loc_c.append(base + np.arange(kb))
            act = Active(*(np.concatenate(v) for v in (rows, rtyp, cols, ctyp)))
            orr, lr = np.concatenate(owner_r), np.concatenate(loc_r)
            oc, lc = np.concatenate(owner_c), np.concatenate(loc_c)
            D = entries(w, g, self._row_points(act), self._col_points(act))
            for ch in cell.children:
                ri = np.flatnonzero(orr == ch)
                ci = np.flatnonzero(oc == ch)
                D[np.ix_(ri, ci)] = below[ch]["At"][np.ix_(lr[ri], lc[ci])]
            acts.append(act)
            Dmats.append(D)
        return acts, Dmats

    def ranks(self):
        return [[d["k"] for d in lev] for lev in self.data]

    def root_size(self):
        return self.root["D"].shape[0]

    def solve(self, angles=None):
        """Upward pass, root solve, downward pass (eq. compressed and the recovery formula)."""
        w, g = self.w, self.g
        ang = w.angles if angles is None else angles
        f_all = dense.rhs(g, ang)
        bo = dense.block_offsets(g)
        fs = [f_all[bo[c.incl[0]]:bo[c.incl[0] + 1]] for c in self.levels[0]]
        ys, gs = [], []
        for lev, info in enumerate(self.data):
            y_l, g_l = [], []
            for t, d in enumerate(info):
                y = la.lu_solve(d["lu"], fs[t])
                gv = d["At"] @ (d["R"] @ y)
                y_l.append(y)
                g_l.append(gv)
            ys.append(y_l)
            gs.append(g_l)
            cells_up = self.levels[lev + 1]
            fs = [self._gather_up(cells_up[p], info, g_l) for p in range(len(cells_up))]
        x_up = [la.lu_solve(self.root["lu"], fs[0])]
        for lev in range(len(self.data) - 1, -1, -1):
            info = self.data[lev]
            cells_up = self.levels[lev + 1]
            xs = [None] * len(info)
            for p, cell in enumerate(cells_up):
                parts = self._scatter_down(cell, info, x_up[p])
                for ch, psi in parts.items():
                    d = info[ch]
                    xs[ch] = ys[lev][ch] - d["Y"] @ (gs[lev][ch] - d["At"] @ psi)
            x_up = xs
        out = np.zeros_like(f_all)
        for t, c in enumerate(self.levels[0]):
            j = c.incl[0]
            out[bo[j]:bo[j + 1]] = x_up[t]
        return out

    @staticmethod
    def _gather_up(cell, info, g_l):
        parts = []
        for b in (0, 1):
            for ch in cell.children:
                k0 = info[ch]["k"][0]
                sl = slice(0, k0) if b == 0 else slice(k0, None)
                parts.append(g_l[ch][sl])
        return np.concatenate(parts)

    @staticmethod
    def _scatter_down(cell, info, x):
        out = {ch: [None, None] for ch in cell.children}
        pos = 0
        for b in (0, 1):
            for ch in cell.children:
                kb = info[ch]["k"][b]
                out[ch][b] = x[pos:pos + kb]
                pos += kb
        return {ch: np.concatenate(v) for ch, v in out.items()}
