"""Closed-form references for circular inclusions (oracle; test infrastructure only).

Single disk (Mie series) and several equal disks (multipole / T-matrix method with
Graf's addition theorem), both for the transmission conditions of Sec. 2.1:
u continuous and (1/eps) du/dn continuous across the boundary, plane-wave incidence
u^I = exp(i k+ (cos a, sin a).x).  They produce the boundary data (q, u) at the
quadrature nodes and the far-field pattern, independent of any boundary integral.
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp


def _jh(l, z):
    J = sp.jv(l, z)
    H = sp.hankel1(l, z)
    Jp = sp.jvp(l, z)
    Hp = sp.h1vp(l, z)
    return J, H, Jp, Hp


def mie_alpha(l, kp, km, R, eps_p, eps_m):
    """Scattering coefficient of mode l: incident J_l e^{il theta} -> scattered alpha_l H_l e^{il theta}."""
    rho = (km * eps_p) / (kp * eps_m)
    J, H, Jp, Hp = _jh(l, kp * R)
    Jm, Jmp = sp.jv(l, km * R), sp.jvp(l, km * R)
    return (rho * J * Jmp - Jp * Jm) / (Hp * Jm - rho * H * Jmp)


def mie_boundary(theta, kp, km, R, eps_p, eps_m, angle=0.0, L=60):
    """(q, u) on a disk of radius R centred at the origin, plane wave at `angle`."""
    ls = np.arange(-L, L + 1)
    u = np.zeros(len(theta), dtype=complex)
    q = np.zeros(len(theta), dtype=complex)
    for l in ls:
        a_inc = (1j) ** l * np.exp(-1j * l * angle)
        al = mie_alpha(l, kp, km, R, eps_p, eps_m)
        J, H, Jp, Hp = _jh(l, kp * R)
        e = np.exp(1j * l * theta)
        u += a_inc * (J + al * H) * e
        q += a_inc * (kp / eps_p) * (Jp + al * Hp) * e
    return q, u


def mie_far_field(dirs, kp, km, R, eps_p, eps_m, angle=0.0, L=60):
    """u_inf(theta) = sqrt(2/(pi k)) e^{-i pi/4} sum_l i^l e^{-il a} alpha_l (-i)^l e^{il theta}."""
    out = np.zeros(len(dirs), dtype=complex)
    for l in range(-L, L + 1):
        al = mie_alpha(l, kp, km, R, eps_p, eps_m)
        out += (1j) ** l * np.exp(-1j * l * angle) * al * (-1j) ** l * np.exp(1j * l * dirs)
    return np.sqrt(2.0 / (np.pi * kp)) * np.exp(-1j * np.pi / 4) * out


def multi_disk(centers, R, kp, km, eps_p, eps_m, angle=0.0, L=40):
    """Multipole solution for equal disks.

    Outgoing field of disk l: sum_m a_{l,m} H_m(k+|x-c_l|) e^{i m theta_l}.  Field
    incident on disk j (regular part): sum_n beta_{j,n} J_n(k+|x-c_j|) e^{i n theta_j},
    with beta = plane wave + the translated outgoing fields of the other disks:
      H_m(k|x-c_l|) e^{i m theta_l} = sum_n H_{m-n}(k b) e^{i (m-n) phi} J_n(k|x-c_j|) e^{i n theta_j},
    (b, phi) = polar coordinates of c_j - c_l (Graf).  Each disk maps beta_{j,n} to
    a_{j,n} = alpha_n beta_{j,n}.  The system is solved in balanced variables
    bt = beta J_n(k+R), at = a H_n(k+R), i.e. the regular and outgoing boundary
    amplitudes of each mode, which keeps every coefficient of order one.
    Returns a function (j, theta) -> (q, u) on disk j's boundary and the coefficients.
    """
    centers = np.asarray(centers, float)
    nd = len(centers)
    ls = np.arange(-L, L + 1)
    nm = len(ls)
    kR = kp * R
    Jn = sp.jv(ls, kR)
    Hn = sp.hankel1(ls, kR)
    al = np.array([mie_alpha(l, kp, km, R, eps_p, eps_m) for l in ls])
    gain = al * Hn / Jn                                  # at = gain * bt
    # translation blocks in balanced variables: bt_j += C_jl at_l
    M = np.zeros((nd * nm, nd * nm), dtype=complex)
    for j in range(nd):
        for l in range(nd):
            if j == l:
                continue
            dvec = centers[j] - centers[l]
            b = np.hypot(*dvec)
            phi = np.arctan2(dvec[1], dvec[0])
            diff = ls[None, :] - ls[:, None]             # m - n, row n, column m
            T = sp.hankel1(diff, kp * b) * np.exp(1j * diff * phi)
            M[j * nm:(j + 1) * nm, l * nm:(l + 1) * nm] = (Jn[:, None] * T / Hn[None, :]) * gain[None, :]
    d = np.array([np.cos(angle), np.sin(angle)])
    p = np.zeros(nd * nm, dtype=complex)
    for j in range(nd):
        p[j * nm:(j + 1) * nm] = np.exp(1j * kp * d @ centers[j]) * (1j) ** ls * np.exp(-1j * ls * angle) * Jn
    bt = np.linalg.solve(np.eye(nd * nm) - M, p)
    bt = bt.reshape(nd, nm)
    at = gain[None, :] * bt
    Jp = sp.jvp(ls, kR)
    Hp = sp.h1vp(ls, kR)

    def boundary(j, theta):
        e = np.exp(1j * np.outer(theta, ls))
        u = e @ (bt[j] + at[j])
        q = (kp / eps_p) * (e @ (bt[j] * Jp / Jn + at[j] * Hp / Hn))
        return q, u

    return boundary, bt, at
