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
    (Colton & Kress, Inverse Acoustic and EM Scattering Theory, Sec. 3.5) or, as the paper
    does (Sec. 2.2), the zeta-corrected trapezoid rule with 41 local correction points, and
    the hypersingular operator is written through Maue's identity
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


ZETA_P = 20   # correction half-width: 2 p + 1 = 41 local correction points (Sec. 2.2)


def zeta_weights(p=ZETA_P):
    """omega_0 .. omega_p of the zeta-corrected trapezoid rule for a logarithmic point
    singularity (Wu and Martinsson, the correction the paper uses in Sec. 2.2).

    For a 2 pi-periodic f(u) = A(u) ln|2 sin(u/2)| + B(u) with A, B smooth and h = 2 pi / n,
    the punctured trapezoid sum h sum_{j != 0} f(jh) misses, beyond h B(0), the terms
    h A(0) ln(h / 2 pi) + 2 sum_{k >= 1} zeta'(-2k) A^(2k)(0) h^(2k+1) / (2k)!
    (the Navot expansion; ln|2 sin(u/2)| - ln|u| is smooth and vanishes at 0).  The
    symmetric weights omega_l (l = -p..p, omega_-l = omega_l) reproduce the derivative sum
    on polynomials of degree 2p: sum_l omega_l = 0 and sum_l omega_l l^(2k) = 2 zeta'(-2k),
    k = 1..p.  The moment system is solved in 60-digit arithmetic (mpmath, a library
    primitive for zeta').
    """
    import mpmath as mp
    with mp.workdps(60):
        M = mp.matrix(p + 1, p + 1)
        rhs = mp.matrix(p + 1, 1)
        for kk in range(p + 1):
            for l in range(p + 1):
                mult = 1 if l == 0 else 2
                M[kk, l] = mult * (mp.mpf(1) if kk == 0 else mp.mpf(l) ** (2 * kk))
            rhs[kk] = 0 if kk == 0 else 2 * mp.zeta(-2 * kk, derivative=1)
        w = mp.lu_solve(M, rhs)
        return np.array([float(w[l]) for l in range(p + 1)])


def zeta_corrected(K, A, Bdiag, p=ZETA_P):
    """Nystrom matrix of a kernel K(t_a, t_b) = A ln|2 sin((t_a - t_b)/2)| + B on n
    equispaced nodes by the zeta-corrected trapezoid rule: off the diagonal h K; on row a,
    h (B(t_a, t_a) + A(t_a, t_a) ln(h / 2 pi)) on the diagonal and h omega_|l| A(t_a, t_a+l)
    added for |l| <= p (indices mod n).  K's diagonal is ignored."""
    n = K.shape[0]
    if n < 2 * p + 2:
        raise ValueError("the zeta-corrected rule needs n >= 2p + 2 nodes")
    h = 2.0 * np.pi / n
    om = zeta_weights(p)
    M = h * K.astype(complex)
    a = np.arange(n)
    M[a, a] = h * (Bdiag + A[a, a] * np.log(h / (2.0 * np.pi)))
    for l in range(-p, p + 1):
        b = (a + l) % n
        M[a, b] += h * om[abs(l)] * A[a, b]
    return M


def self_blocks_zeta(x, y, dx, dy, ddx, ddy, k, p=ZETA_P):
    """S, D, D*, N of one closed curve onto itself with the zeta-corrected trapezoid rule
    (41 local correction points for p = 20, Sec. 2.2); N by Maue's identity as in
    self_blocks.  Each kernel times |x'(tau)| is K1 ln(4 sin^2((t - tau)/2)) + K2, so A = 2 K1
    multiplies ln|2 sin| and B = K2."""
    n = len(x)
    off = np.array([0, n])
    speed, nx, ny, _, kappa = boundary_quantities(dx, dy, ddx, ddy, off)
    eye = np.eye(n, dtype=bool)
    d1 = x[:, None] - x[None, :]
    d2 = y[:, None] - y[None, :]
    r = np.hypot(d1, d2)
    r[eye] = 1.0
    kr = k * r
    J0, J1 = sp.j0(kr), sp.j1(kr)
    H0, H1 = h01(kr)
    sb = speed[None, :]
    ndy = (nx[None, :] * d1 + ny[None, :] * d2) / r
    ndx = (nx[:, None] * d1 + ny[:, None] * d2) / r
    nn = nx[:, None] * nx[None, :] + ny[:, None] * ny[None, :]
    diag_s = (0.25j - EULER_GAMMA / (2 * np.pi) - np.log(k * speed / 2.0) / (2 * np.pi)) * speed
    diag_d = -kappa * speed / (4 * np.pi)
    # single layer: K1 = -J0 |x'| / 4 pi (its diagonal value -|x'| / 4 pi)
    K1 = -J0 * sb / (4 * np.pi)
    K1[eye] = -speed / (4 * np.pi)
    S = zeta_corrected(0.25j * H0 * sb, 2 * K1, diag_s, p)
    Snn = zeta_corrected(0.25j * H0 * nn * sb, 2 * K1 * nn, diag_s, p)
    # double layer and its adjoint: K1 vanishes on the diagonal
    K1 = -(k / (4 * np.pi)) * J1 * ndy * sb
    K1[eye] = 0.0
    D = zeta_corrected(0.25j * k * H1 * ndy * sb, 2 * K1, diag_d, p)
    K1 = (k / (4 * np.pi)) * J1 * ndx * sb
    K1[eye] = 0.0
    Ds = zeta_corrected(-0.25j * k * H1 * ndx * sb, 2 * K1, diag_d, p)
    Dt = trig_diff_matrix(n)
    Linv = np.diag(1.0 / speed)
    N = Linv @ Dt @ S @ Linv @ Dt + k * k * Snn
    return S, D, Ds, N


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
