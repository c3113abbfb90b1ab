"""Seeded synthetic workloads: inclusion layouts and sampled boundary curves.

This module only *draws* inputs.  It holds none of the solver's arithmetic:
for every inclusion it produces the centre, the radial shape parameters and the
boundary curve x(t) with its first and second t-derivatives, sampled at the
equispaced parameter nodes t_j = 2*pi*j/n, counterclockwise.  Normals, weights,
curvature, kernels and everything after them are computed independently by the
library and by the oracle.

The paper's own workload (Sec. 4: star-shaped inclusions on a regular grid,
counts that are powers of four) is given only as a figure, so the shapes below
are seeded stand-ins of the same kind: rotated five-pointed stars on unit-spaced
grids, circles, and random smooth Fourier boundaries.

Shape model: rho(t) = a * (1 + sum_m c_m cos(m t + phi_m)),
x(t) = centre + rho(t) * (cos(t + theta), sin(t + theta)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    centers: np.ndarray          # (m, 2)
    node_off: np.ndarray         # int64 (m+1,)
    x: np.ndarray                # float64 (sum n,) boundary samples
    y: np.ndarray
    dx: np.ndarray               # first t-derivative
    dy: np.ndarray
    ddx: np.ndarray              # second t-derivative
    ddy: np.ndarray
    k_ext: float
    k_int: np.ndarray            # (m,)
    eps_ext: float = 1.0
    angles: np.ndarray = field(default_factory=lambda: np.zeros(1))
    id_tol: float = 1e-10
    grid: tuple | None = None    # (gx, gy) grid shape, inclusion j*gx+i at (i, j)
    grid_index: np.ndarray | None = None  # (m, 2) integer grid coordinates
    proxy_ratio: float = 1.5
    proxy_min: int = 0
    near_rule: int = 0           # 0: 4-adjacent + geometric, 1: geometric only
    proxy_paper_rule: bool = True  # radius max(ratio*r_c, 0.9*rho_far)
    shapes: list = field(default_factory=list)  # per inclusion (a, theta, [(m, c_m, phi_m)])
    quadrature: str = "kress"    # self blocks: "kress" or "zeta" (the 41-point corrected trapezoid)
    tree: str = "quad"           # "quad": grid quadtree; "kmeans": k-means clusters (Sec. 4.4)
    leaf_size: int = 4           # kmeans: at most this many inclusions per leaf
    eta: float = 1.0             # near_rule 2: eta-admissibility constant

    @property
    def m(self) -> int:
        return len(self.node_off) - 1

    @property
    def n_nodes(self) -> int:
        return int(self.node_off[-1])

    @property
    def n_unknowns(self) -> int:
        return 2 * self.n_nodes

    def sizes(self) -> np.ndarray:
        return np.diff(self.node_off)


def sample_curve(center, a, theta, modes, n):
    """Sample x(t), x'(t), x''(t) at t_j = 2*pi*j/n for one radial shape."""
    t = 2.0 * np.pi * np.arange(n) / n
    rho = np.ones(n)
    drho = np.zeros(n)
    ddrho = np.zeros(n)
    for (mm, cm, ph) in modes:
        arg = mm * t + ph
        rho = rho + cm * np.cos(arg)
        drho = drho - mm * cm * np.sin(arg)
        ddrho = ddrho - mm * mm * cm * np.cos(arg)
    rho, drho, ddrho = a * rho, a * drho, a * ddrho
    ex, ey = np.cos(t + theta), np.sin(t + theta)
    px, py = -ey, ex
    x = center[0] + rho * ex
    y = center[1] + rho * ey
    dx = drho * ex + rho * px
    dy = drho * ey + rho * py
    ddx = ddrho * ex + 2.0 * drho * px - rho * ex
    ddy = ddrho * ey + 2.0 * drho * py - rho * ey
    return x, y, dx, dy, ddx, ddy


def _assemble(name, centers, shapes, ns, k_ext, k_int, **kw) -> Workload:
    m = len(centers)
    off = np.zeros(m + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)
    arrs = [np.empty(off[-1]) for _ in range(6)]
    for j in range(m):
        a, th, modes = shapes[j]
        parts = sample_curve(centers[j], a, th, modes, int(ns[j]))
        for arr, p in zip(arrs, parts):
            arr[off[j]:off[j + 1]] = p
    return Workload(name=name, centers=np.asarray(centers, float), node_off=off,
                    x=arrs[0], y=arrs[1], dx=arrs[2], dy=arrs[3], ddx=arrs[4], ddy=arrs[5],
                    k_ext=float(k_ext), k_int=np.asarray(k_int, float), shapes=list(shapes), **kw)


def _grid(gx, gy, spacing=1.0):
    ij = np.array([(i, j) for j in range(gy) for i in range(gx)], dtype=np.int64)
    return ij, ij.astype(float) * spacing


STAR_MODES = [(5, 0.2, 0.0)]


def star_grid(g, n=128, k_ext=10.0, k_int=15.0, seed=2, angles=None, id_tol=1e-10,
              gy=None, a=0.3, name=None) -> Workload:
    """g x gy grid of rotated stars r(t) = a(1 + 0.2 cos 5t), unit spacing.

    Rotations are U(0, 2*pi) from default_rng(seed), drawn in row-major order
    (i fastest along x1)."""
    gy = g if gy is None else gy
    ij, c = _grid(g, gy)
    rng = np.random.default_rng(seed)
    rot = rng.uniform(0.0, 2.0 * np.pi, size=len(c))
    shapes = [(a, float(rot[j]), STAR_MODES) for j in range(len(c))]
    ns = np.full(len(c), n)
    ang = np.zeros(1) if angles is None else np.asarray(angles, float)
    return _assemble(name or f"stars{g}x{gy}_n{n}", c, shapes, ns, k_ext,
                     np.full(len(c), k_int), angles=ang, id_tol=id_tol,
                     grid=(g, gy), grid_index=ij)


def disk_grid(g, n=64, radius=0.4, k_ext=2 * np.pi, k_int=4 * np.pi, gy=None,
              angles=None, id_tol=1e-10, proxy_min=64, name=None) -> Workload:
    gy = g if gy is None else gy
    ij, c = _grid(g, gy)
    shapes = [(radius, 0.0, []) for _ in range(len(c))]
    ns = np.full(len(c), n)
    ang = np.zeros(1) if angles is None else np.asarray(angles, float)
    return _assemble(name or f"disks{g}x{gy}_n{n}", c, shapes, ns, k_ext,
                     np.full(len(c), k_int), angles=ang, id_tol=id_tol, grid=(g, gy),
                     grid_index=ij, proxy_min=proxy_min, proxy_paper_rule=False)


def single_disk(n=64, radius=0.4, k_ext=2 * np.pi, k_int=4 * np.pi, angles=None) -> Workload:
    w = disk_grid(1, n=n, radius=radius, k_ext=k_ext, k_int=k_int, angles=angles)
    w.name = f"disk_n{n}"
    return w


def config1() -> Workload:
    """2x2 disks, R=0.4, spacing 1, k+=2pi, k-=2k+, 64 nodes, proxy 64 pts at 1.5 r_c,
    tol 1e-10, one plane wave at angle 0 (N=512)."""
    w = disk_grid(2, n=64, radius=0.4, k_ext=2 * np.pi, k_int=4 * np.pi, angles=[0.0],
                  id_tol=1e-10, proxy_min=64)
    w.name = "cfg1_disks2x2_n64"
    return w


def config2(g=16) -> Workload:
    """16x16 rotated stars, 128 nodes, k+=10, k-=15, tol 1e-10, 4 angles 2*pi*j/4 (N=65536)."""
    w = star_grid(g, n=128, k_ext=10.0, k_int=15.0, seed=2,
                  angles=2 * np.pi * np.arange(4) / 4, id_tol=1e-10)
    w.name = f"cfg2_stars{g}x{g}_n128_k10"
    return w


def config4(g=64) -> Workload:
    """64x64 rotated stars (N ~ 1.05M), k+=8, k-=12, 16 angles 2*pi*j/16."""
    w = star_grid(g, n=128, k_ext=8.0, k_int=12.0, seed=4,
                  angles=2 * np.pi * np.arange(16) / 16, id_tol=1e-10)
    w.name = f"cfg4_stars{g}x{g}_n128_k8"
    return w


def sub_grid(w: Workload, g: int, name=None) -> Workload:
    """The g x g corner block of a grid workload (same shapes, same parameters)."""
    gx, gy = w.grid
    sel = [j * gx + i for j in range(g) for i in range(g)]
    shapes = [w.shapes[s] for s in sel]
    ns = w.sizes()[sel]
    out = _assemble(name or f"{w.name}_sub{g}", w.centers[sel], shapes, ns, w.k_ext,
                    w.k_int[sel], angles=w.angles.copy(), id_tol=w.id_tol, grid=(g, g),
                    grid_index=w.grid_index[sel].copy(), proxy_ratio=w.proxy_ratio,
                    proxy_min=w.proxy_min, near_rule=w.near_rule,
                    proxy_paper_rule=w.proxy_paper_rule)
    return out


def random_shapes(m, seed, a_lo=0.1, a_hi=0.4, cmax=0.05, rng=None):
    rng = np.random.default_rng(seed) if rng is None else rng
    out = []
    for _ in range(m):
        a = rng.uniform(a_lo, a_hi)
        modes = [(mm, rng.uniform(-cmax, cmax), rng.uniform(0, 2 * np.pi)) for mm in range(2, 7)]
        out.append((a, 0.0, modes))
    return out


def perimeter(a, modes, nfine=2048):
    x, y, dx, dy, _, _ = sample_curve((0.0, 0.0), a, 0.0, modes, nfine)
    return float(np.sum(np.hypot(dx, dy)) * 2 * np.pi / nfine)


def config3(m=400, box=24.0, seed=3, k_ext=12.0) -> Workload:
    """400 random smooth inclusions, dart-throwing placement in a 24x24 box, per-inclusion
    contrast k-/k+ ~ U(1.2, 2.0), nodes = even(clamp(ceil(8 k- perimeter), 64, 256))."""
    rng = np.random.default_rng(seed)
    shapes, centers, kin, ns = [], [], [], []
    tries = 0
    while len(centers) < m:
        tries += 1
        if tries > 2_000_000:
            raise RuntimeError("dart throwing did not place all inclusions")
        a = rng.uniform(0.1, 0.4)
        modes = [(mm, rng.uniform(-0.05, 0.05), rng.uniform(0, 2 * np.pi)) for mm in range(2, 7)]
        rad = a * (1 + sum(abs(c) for _, c, _ in modes))
        cx, cy = rng.uniform(rad, box - rad, size=2)
        ok = True
        for (c2, r2) in centers:
            if math.hypot(cx - c2[0], cy - c2[1]) < rad + r2 + 0.1:
                ok = False
                break
        if not ok:
            continue
        ratio = rng.uniform(1.2, 2.0)
        centers.append(((cx, cy), rad))
        shapes.append((a, 0.0, modes))
        kin.append(ratio * k_ext)
        nn = int(math.ceil(8 * ratio * k_ext * perimeter(a, modes)))
        nn = min(max(nn, 64), 256)
        nn += nn % 2
        ns.append(nn)
    c = np.array([cc for cc, _ in centers])
    return _assemble("cfg3_random400", c, shapes, np.array(ns), k_ext, np.array(kin),
                     angles=2 * np.pi * np.arange(4) / 4, id_tol=1e-10, near_rule=1)


def random_close(m=400, box=16.0, gap=0.02, seed=7, k_ext=12.0, a_lo=0.1, a_hi=0.3, nrhs=4,
                 name=None) -> Workload:
    """Randomly placed smooth inclusions, some of them nearly touching (Sec. 4.4's random
    arrangements with close scatterers): dart throwing in a box x box square with bounding
    circles at least `gap` apart, shapes a(1 + sum_{m=2..6} c_m cos(m t + phi_m)) with
    a ~ U(a_lo, a_hi), |c_m| <= 0.05, per-inclusion contrast k-/k+ ~ U(1.2, 2.0), nodes
    even(clamp(ceil(8 k- perimeter), 64, 256)), nrhs plane waves at 2 pi j / nrhs; the
    k-means tree with up to four inclusions per leaf and the eta-admissibility rule."""
    rng = np.random.default_rng(seed)
    shapes, placed, kin, ns = [], [], [], []
    tries = 0
    while len(placed) < m:
        tries += 1
        if tries > 2_000_000:
            raise RuntimeError("dart throwing did not place all inclusions")
        a = rng.uniform(a_lo, a_hi)
        modes = [(mm, rng.uniform(-0.05, 0.05), rng.uniform(0, 2 * np.pi)) for mm in range(2, 7)]
        rad = a * (1 + sum(abs(c) for _, c, _ in modes))
        cx, cy = rng.uniform(rad, box - rad, size=2)
        if any(math.hypot(cx - c2[0], cy - c2[1]) < rad + r2 + gap for (c2, r2) in placed):
            continue
        ratio = rng.uniform(1.2, 2.0)
        placed.append(((cx, cy), rad))
        shapes.append((a, 0.0, modes))
        kin.append(ratio * k_ext)
        nn = int(math.ceil(8 * ratio * k_ext * perimeter(a, modes)))
        nn = min(max(nn, 64), 256)
        nn += nn % 2
        ns.append(nn)
    c = np.array([cc for cc, _ in placed])
    return _assemble(name or f"close{m}_box{box:g}_gap{gap:g}_s{seed}", c, shapes, np.array(ns), k_ext,
                     np.array(kin), angles=2 * np.pi * np.arange(nrhs) / nrhs, id_tol=1e-10, near_rule=2,
                     tree="kmeans", leaf_size=4)


def random_shape_grid(g, seed, k_ext, n=128, a_lo=0.25, a_hi=0.35, cmax=0.05, contrast=1.5, angles=None,
                      id_tol=1e-10, name=None) -> Workload:
    """g x g grid (spacing 1) of random smooth shapes r(t) = a(1 + sum_{m=2..6} c_m cos(m t + phi_m)),
    a ~ U(a_lo, a_hi), c_m ~ U(-cmax, cmax), phi_m ~ U(0, 2 pi), rotation ~ U(0, 2 pi), drawn in
    row-major cell order from default_rng(seed); k- = contrast k+, n nodes each."""
    ij, c = _grid(g, g)
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(len(c)):
        a = rng.uniform(a_lo, a_hi)
        modes = [(mm, rng.uniform(-cmax, cmax), rng.uniform(0, 2 * np.pi)) for mm in range(2, 7)]
        rot = rng.uniform(0.0, 2.0 * np.pi)
        shapes.append((a, rot, modes))
    ang = np.zeros(1) if angles is None else np.asarray(angles, float)
    return _assemble(name or f"shapes{g}x{g}_k{k_ext:g}_s{seed}", c, shapes, np.full(len(c), n), k_ext,
                     np.full(len(c), contrast * k_ext), angles=ang, id_tol=id_tol, grid=(g, g), grid_index=ij)


def config5_train(i, g=32):
    """Training geometry i of the learned-skeleton form: seed 5 + i, k+ a in [1, 8] through
    k+ ~ U(1, 8) / 0.3 drawn from default_rng(1000 + i)."""
    k = float(np.random.default_rng(1000 + i).uniform(1.0, 8.0)) / 0.3
    return random_shape_grid(g, 5 + i, k)


def config5(k_ext=10.0, g=32, seed=6):
    """Evaluation grid of the learned-skeleton form: 32 x 32 random shapes, seed 6."""
    return random_shape_grid(g, seed, k_ext)


def plane_wave_angles(nrhs):
    return 2 * np.pi * np.arange(nrhs) / nrhs
