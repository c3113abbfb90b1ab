"""Dense PMCHWT (Omit) Nystrom system and its direct solve (oracle; test infrastructure only).

Unknowns per inclusion i: phi_i = (q_i; u_i), q = (1/eps) du/dn (Sec. 2.1, eqs.
pressure and flux); right-hand side f_i = (-u^I_i; -q^I_i).  Blocks (Sec. 2.2, the
discrete Omit form):
  A_ii = [[-(e+ S+ + e- S-), D+ + D-], [-(D*+ + D*-), N+/e+ + N-/e-]]
  A_ij = [[-e+ S+, D+], [-D*+, N+/e+]]                   (i != j, exterior k+ only)
The system is solved by LU with partial pivoting, as the paper does for the
conventional method and for the compressed top-level system (Sec. 4).
Material reading: e+ = 1 and e-_j = e+ (k-_j / k+)^2, from k = omega sqrt(eps).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la

from . import layer


def materials(w):
    eps_p = float(w.eps_ext)
    eps_m = eps_p * (np.asarray(w.k_int) / w.k_ext) ** 2
    return eps_p, eps_m


class Geometry:
    def __init__(self, w):
        self.w = w
        self.off = np.asarray(w.node_off)
        self.x, self.y = w.x, w.y
        (self.speed, self.nx, self.ny, self.wt, self.kappa) = layer.boundary_quantities(
            w.dx, w.dy, w.ddx, w.ddy, self.off)
        self.eps_p, self.eps_m = materials(w)

    def nodes(self, j):
        return slice(self.off[j], self.off[j + 1])


def diagonal_block(g: Geometry, j):
    """A_jj of the Omit form: both wavenumbers; Kress self-interaction quadrature, or the
    zeta-corrected trapezoid rule (41 points, Sec. 2.2) when the workload asks for it."""
    w = g.w
    s = g.nodes(j)
    args = (w.x[s], w.y[s], w.dx[s], w.dy[s], w.ddx[s], w.ddy[s])
    blocks = layer.self_blocks_zeta if getattr(w, "quadrature", "kress") == "zeta" else layer.self_blocks
    Sp, Dp, Dsp, Np = blocks(*args, w.k_ext)
    Sm, Dm, Dsm, Nm = blocks(*args, w.k_int[j])
    ep, em = g.eps_p, g.eps_m[j]
    return np.block([[-(ep * Sp + em * Sm), Dp + Dm],
                     [-(Dsp + Dsm), Np / ep + Nm / em]])


def offdiag_block(g: Geometry, i, j):
    """A_ij (i != j): exterior kernels times the trapezoid weights of Gamma_j."""
    si, sj = g.nodes(i), g.nodes(j)
    S, D, Ds, N = layer.kernel_blocks(g.x[si], g.y[si], g.nx[si], g.ny[si],
                                      g.x[sj], g.y[sj], g.nx[sj], g.ny[sj], g.w.k_ext)
    wj = g.wt[sj][None, :]
    ep = g.eps_p
    return np.block([[-ep * S * wj, D * wj], [-Ds * wj, N * wj / ep]])


def block_offsets(g: Geometry):
    return 2 * g.off


def assemble(g: Geometry):
    """Full 2N x 2N matrix, block (i, j) at rows 2*off[i].., columns 2*off[j]..."""
    m = g.w.m
    bo = block_offsets(g)
    A = np.zeros((bo[-1], bo[-1]), dtype=complex)
    for i in range(m):
        for j in range(m):
            blk = diagonal_block(g, i) if i == j else offdiag_block(g, i, j)
            A[bo[i]:bo[i + 1], bo[j]:bo[j + 1]] = blk
    return A


def incident(g: Geometry, angles):
    """u^I = exp(i k+ d.x), q^I = (1/e+) du^I/dn with d = (cos a, sin a) (Sec. 4)."""
    k = g.w.k_ext
    ang = np.atleast_1d(angles)
    dxv, dyv = np.cos(ang), np.sin(ang)
    uI = np.exp(1j * k * (np.outer(g.x, dxv) + np.outer(g.y, dyv)))
    qI = 1j * k * (np.outer(g.nx, dxv) + np.outer(g.ny, dyv)) * uI / g.eps_p
    return uI, qI


def rhs(g: Geometry, angles):
    """f_i = (-u^I_i; -q^I_i) stacked per inclusion, one column per angle."""
    uI, qI = incident(g, angles)
    m = g.w.m
    bo = block_offsets(g)
    f = np.zeros((bo[-1], uI.shape[1]), dtype=complex)
    for j in range(m):
        s = g.nodes(j)
        n = s.stop - s.start
        f[bo[j]:bo[j] + n] = -uI[s]
        f[bo[j] + n:bo[j + 1]] = -qI[s]
    return f


def split_density(g: Geometry, phi):
    """(q, u) per node from the stacked solution vector(s)."""
    phi = phi.reshape(phi.shape[0], -1)
    q = np.zeros((g.off[-1], phi.shape[1]), dtype=complex)
    u = np.zeros_like(q)
    bo = block_offsets(g)
    for j in range(g.w.m):
        s = g.nodes(j)
        n = s.stop - s.start
        q[s] = phi[bo[j]:bo[j] + n]
        u[s] = phi[bo[j] + n:bo[j + 1]]
    return q, u


def solve(w, angles=None):
    """Conventional method: assemble, LU with partial pivoting, solve."""
    g = Geometry(w)
    ang = w.angles if angles is None else angles
    A = assemble(g)
    f = rhs(g, ang)
    lu = la.lu_factor(A, overwrite_a=True, check_finite=False)
    return la.lu_solve(lu, f, check_finite=False)


def far_field(g: Geometry, phi, dirs):
    """u_inf(xh) = e^{i pi/4}/sqrt(8 pi k) sum_b w_b [-i k (xh.n_b) u_b - e+ q_b] e^{-i k xh.y_b}
    for the scattered field u^S ~ e^{ikr}/sqrt(r) u_inf (exterior representation
    u^S = D u - e+ S q outside the inclusions)."""
    k = g.w.k_ext
    q, u = split_density(g, phi)
    dirs = np.atleast_1d(dirs)
    cx, cy = np.cos(dirs), np.sin(dirs)
    ph = np.exp(-1j * k * (np.outer(cx, g.x) + np.outer(cy, g.y)))      # (ndir, nodes)
    xn = np.outer(cx, g.nx) + np.outer(cy, g.ny)
    out = np.zeros((len(dirs), q.shape[1]), dtype=complex)
    for r in range(q.shape[1]):
        integrand = g.wt[None, :] * (-1j * k * xn * u[None, :, r] - g.eps_p * q[None, :, r])
        out[:, r] = np.sum(integrand * ph, axis=1)
    return np.exp(1j * np.pi / 4) / np.sqrt(8 * np.pi * k) * out


def energy_defect(g: Geometry, phi):
    """Per inclusion Im sum_b w_b conj(u_b) q_b: zero for lossless media (Green's
    identity in each inclusion); returned relative to sum_b w_b |u_b||q_b|."""
    q, u = split_density(g, phi)
    res = []
    for j in range(g.w.m):
        s = g.nodes(j)
        num = np.imag(np.sum(g.wt[s, None] * np.conj(u[s]) * q[s], axis=0))
        den = np.sum(g.wt[s, None] * np.abs(u[s]) * np.abs(q[s]), axis=0)
        res.append(num / den)
    return np.array(res)


def rel_error(phi, ref):
    """Relative 2-norm error over all 2N entries (Sec. 4.2, eq. relative_norm)."""
    return np.linalg.norm(phi - ref) / np.linalg.norm(ref)


def residual_rows(w, phi, rows, angles=None):
    """r = f - A phi on a subset of global rows, each row of A evaluated on the fly
    (diagonal blocks by Kress quadrature, all other inclusions by the trapezoid rule)."""
    g = Geometry(w)
    ang = w.angles if angles is None else angles
    f = rhs(g, ang)
    bo = block_offsets(g)
    phi = phi.reshape(phi.shape[0], -1)
    q, u = split_density(g, phi)
    out = np.zeros((len(rows), phi.shape[1]), dtype=complex)
    incl = np.searchsorted(bo, rows, side="right") - 1
    cache = {}
    owner = np.repeat(np.arange(w.m), np.diff(g.off))
    for idx, (row, i) in enumerate(zip(rows, incl)):
        if i not in cache:
            cache[i] = diagonal_block(g, i)
        loc = row - bo[i]
        n_i = g.off[i + 1] - g.off[i]
        a = g.off[i] + (loc % n_i)
        acc = cache[i][loc] @ phi[bo[i]:bo[i + 1]]
        far = owner != i
        S, D, Ds, N = layer.kernel_blocks(g.x[a:a + 1], g.y[a:a + 1], g.nx[a:a + 1],
                                          g.ny[a:a + 1], g.x[far], g.y[far], g.nx[far],
                                          g.ny[far], w.k_ext)
        wf = g.wt[far]
        if loc < n_i:
            cq, cu = -g.eps_p * S[0] * wf, D[0] * wf
        else:
            cq, cu = -Ds[0] * wf, N[0] * wf / g.eps_p
        acc = acc + cq @ q[far] + cu @ u[far]
        out[idx] = f[row] - acc
    return out
