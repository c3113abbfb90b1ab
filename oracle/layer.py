"""Layer-potential kernels and their Nystrom matrices (oracle; test infrastructure only).

Conventions (readings of the paper, each listed in the design notes):
  * fundamental solution G(x, y) = (i/4) H0^(1)(k|x-y|)  (Sec. 2.1 prints H0 without
    the 1/4 i factor; the jump terms 1/2 of the Burton-Miller form only hold with it);
  * the normal n points into the exterior Omega+ (Sec. 2.1), t runs counterclockwise
    and n = (x2', -x1') / |x'|;
  * S, D, D*, N are the single layer, double layer, adjoint double layer and the
    hypersingular operator of Sec. 2.1 (eqs. slp, dlp, d_slp, d_dlp);
  * off-diagonal blocks use the trapezoid rule on the equispaced parameter nodes;
    the self-interaction blocks use Kress' logarithmic product quadrature
    (Colton & Kress, Inverse Acoustic and EM Scattering Theory, Sec. 3.5) and the
    hypersingular operator is written through Maue's identity
    N = d/ds S d/ds + k^2 n.S n with trigonometric differentiation.
The Bessel and Hankel functions come from scipy.special (a library primitive).
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp

EULER_GAMMA = 0.57721566490153286060651209008240243


def boundary_quantities(dx, dy, ddx, ddy, node_off):
    """Speed |x'|, unit normal, trapezoid weight and curvature per node (Sec. 2.2)."""
    speed = np.hypot(dx, dy)
    nx = dy / speed
    ny = -dx / speed
    sizes = np.diff(node_off)
    h = np.repeat(2.0 * np.pi / sizes, sizes)
    w = h * speed
    kappa = (dx * ddy - dy * ddx) / speed ** 3
    return speed, nx, ny, w, kappa


def h01(z):
    return sp.hankel1(0, z), sp.hankel1(1, z)


def kernel_blocks(tx, ty, tnx, tny, sx, sy, snx, sny, k):
    """Pointwise kernels between disjoint target and source sets (no weights).

    Returns G, dG/dn_y, dG/dn_x and d^2G/dn_x dn_y for G = (i/4) H0(k r), d = x - y.
    """
    d1 = tx[:, None] - sx[None, :]
    d2 = ty[:, None] - sy[None, :]
    r = np.hypot(d1, d2)
    H0, H1 = h01(k * r)
    ndy = (snx[None, :] * d1 + sny[None, :] * d2) / r   # n_y . d / r
    ndx = (tnx[:, None] * d1 + tny[:, None] * d2) / r   # n_x . d / r
    nn = tnx[:, None] * snx[None, :] + tny[:, None] * sny[None, :]
    S = 0.25j * H0
    D = 0.25j * k * H1 * ndy
    Ds = -0.25j * k * H1 * ndx
    N = 0.25j * k * (k * H0 * ndx * ndy - 2.0 * H1 * ndx * ndy / r + H1 * nn / r)
    return S, D, Ds, N


def kress_log_weights(n):
    """R_d for d = 0..n-1: weights of the product rule for ln(4 sin^2((t-tau)/2)) f(tau)
    on n = 2h equispaced nodes (Kress 1991)."""
    h = n // 2
    t = 2.0 * np.pi * np.arange(n) / n
    R = np.zeros(n)
    for m in range(1, h):
        R -= (2.0 * np.pi / h) * np.cos(m * t) / m
    R -= (np.pi / h ** 2) * np.cos(h * t)
    return R


def trig_diff_matrix(n):
    """Derivative of the trigonometric interpolant at the nodes, n even."""
    t = 2.0 * np.pi * np.arange(n) / n
    a = np.arange(n)
    diff = t[:, None] - t[None, :]
    with np.errstate(divide="ignore"):
        Dt = 0.5 * (-1.0) ** (a[:, None] - a[None, :]) / np.tan(diff / 2.0)
    np.fill_diagonal(Dt, 0.0)
    return Dt


def self_blocks(x, y, dx, dy, ddx, ddy, k):
    """Kress-quadrature matrices S, D, D*, N of one closed curve onto itself.

    Each kernel times |x'(tau)| is split as K1 ln(4 sin^2((t-tau)/2)) + K2; the
    entry is R_{a-b} K1(t_a, t_b) + (2 pi / n) K2(t_a, t_b).
    """
    n = len(x)
    off = np.array([0, n])
    speed, nx, ny, _, kappa = boundary_quantities(dx, dy, ddx, ddy, off)
    t = 2.0 * np.pi * np.arange(n) / n
    a = np.arange(n)
    R = kress_log_weights(n)[(a[:, None] - a[None, :]) % n]
    eye = np.eye(n, dtype=bool)
    d1 = x[:, None] - x[None, :]
    d2 = y[:, None] - y[None, :]
    r = np.hypot(d1, d2)
    r[eye] = 1.0
    with np.errstate(divide="ignore"):
        L = np.log(4.0 * np.sin((t[:, None] - t[None, :]) / 2.0) ** 2)
    L[eye] = 0.0
    kr = k * r
    J0, J1 = sp.j0(kr), sp.j1(kr)
    H0, H1 = h01(kr)
    sb = speed[None, :]
    ndy = (nx[None, :] * d1 + ny[None, :] * d2) / r
    ndx = (nx[:, None] * d1 + ny[:, None] * d2) / r
    nn = nx[:, None] * nx[None, :] + ny[:, None] * ny[None, :]
    q = 2.0 * np.pi / n
    diag_s = (0.25j - EULER_GAMMA / (2 * np.pi) - np.log(k * speed / 2.0) / (2 * np.pi)) * speed

    def assemble(K, K1, K2diag):
        K2 = K - K1 * L
        K2[eye] = K2diag
        return R * K1 + q * K2

    # single layer
    K = 0.25j * H0 * sb
    K1 = -J0 * sb / (4 * np.pi)
    K1[eye] = -speed / (4 * np.pi)
    S = assemble(K, K1, diag_s)
    # double layer
    K = 0.25j * k * H1 * ndy * sb
    K1 = -(k / (4 * np.pi)) * J1 * ndy * sb
    K1[eye] = 0.0
    D = assemble(K, K1, -kappa * speed / (4 * np.pi))
    # adjoint double layer
    K = -0.25j * k * H1 * ndx * sb
    K1 = (k / (4 * np.pi)) * J1 * ndx * sb
    K1[eye] = 0.0
    Ds = assemble(K, K1, -kappa * speed / (4 * np.pi))
    # single layer with n(t).n(tau), for Maue's identity
    K = 0.25j * H0 * nn * sb
    K1 = -J0 * nn * sb / (4 * np.pi)
    K1[eye] = -speed / (4 * np.pi)
    Snn = assemble(K, K1, diag_s)
    Dt = trig_diff_matrix(n)
    Linv = np.diag(1.0 / speed)
    N = Linv @ Dt @ S @ Linv @ Dt + k * k * Snn
    return S, D, Ds, N
