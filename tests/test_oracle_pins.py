"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here touches the HIP path.  Each test pins one part of the oracle to
something other than itself: closed forms (circle eigenvalues, Mie series),
identities (Calderon), an independent method (multipole), invariants (energy,
optical theorem, reciprocity), high-precision arithmetic (mpmath), brute force
(fast vs dense) and the paper's printed degree-of-freedom table.
"""
import os

import mpmath
import numpy as np
import pytest
from scipy import special as sp

from oracle import analytic, dense, fast, layer
from paper_2603_09381_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_scipy_hankel_matches_mpmath():
    """The oracle's library primitive (scipy Hankel functions) against 30-digit mpmath."""
    mpmath.mp.dps = 30
    for z in [1e-6, 0.01, 0.3, 1.0, 2.5, 7.9, 12.3, 19.0, 33.3, 150.0, 999.0]:
        for nu in (0, 1):
            ref = complex(mpmath.hankel1(nu, z))
            got = sp.hankel1(nu, z)
            assert abs(got - ref) <= 2e-15 * max(1.0, abs(ref)), (nu, z, got, ref)


@pytest.mark.parametrize("n", [16, 64])
def test_kress_weights_exact_on_trig_polynomials(n):
    """int_0^2pi ln(4 sin^2((t-tau)/2)) e^{i m tau} dtau = -2pi/|m| e^{i m t} (0 for m = 0),
    reproduced exactly for |m| < n/2."""
    h = n // 2
    R = layer.kress_log_weights(n)
    t = 2 * np.pi * np.arange(n) / n
    a = np.arange(n)
    Rm = R[(a[:, None] - a[None, :]) % n]
    for m in range(-h + 1, h):
        got = Rm @ np.exp(1j * m * t)
        ref = np.zeros(n, complex) if m == 0 else -2 * np.pi / abs(m) * np.exp(1j * m * t)
        assert np.max(np.abs(got - ref)) < 1e-12


def test_trig_diff_matrix_exact():
    n = 32
    t = 2 * np.pi * np.arange(n) / n
    Dt = layer.trig_diff_matrix(n)
    for m in range(-n // 2 + 1, n // 2):
        assert np.max(np.abs(Dt @ np.exp(1j * m * t) - 1j * m * np.exp(1j * m * t))) < 1e-11


def _circle(n, R=0.4):
    w = W.single_disk(n=n, radius=R)
    return w


@pytest.mark.parametrize("k", [2 * np.pi, 4 * np.pi])
def test_circle_eigenvalues(k):
    """Kress S, D, D* and Maue N on a circle against the Graf closed forms:
    S -> (i pi R/2) J H, D = D* -> (i pi k R/4)(J'H + JH'), N -> (i pi k^2 R/2) J'H'."""
    n, R = 64, 0.4
    w = _circle(n, R)
    S, D, Ds, N = layer.self_blocks(w.x, w.y, w.dx, w.dy, w.ddx, w.ddy, k)
    t = 2 * np.pi * np.arange(n) / n
    z = k * R
    for l in range(-n // 4 + 1, n // 4):
        e = np.exp(1j * l * t)
        J, H, Jp, Hp = sp.jv(l, z), sp.hankel1(l, z), sp.jvp(l, z), sp.h1vp(l, z)
        lamS = 1j * np.pi * R / 2 * J * H
        lamD = 1j * np.pi * k * R / 4 * (Jp * H + J * Hp)
        lamN = 1j * np.pi * k * k * R / 2 * Jp * Hp
        for M, lam, tol in ((S, lamS, 1e-12), (D, lamD, 1e-12), (Ds, lamD, 1e-12), (N, lamN, 1e-10)):
            err = np.max(np.abs(M @ e - lam * e))
            assert err <= tol * max(1.0, abs(lam)), (l, err, lam)


def _point_source(x, y, nx, ny, z, k):
    d1, d2 = x - z[0], y - z[1]
    r = np.hypot(d1, d2)
    v = 0.25j * sp.hankel1(0, k * r)
    dv = -0.25j * k * sp.hankel1(1, k * r) * (nx * d1 + ny * d2) / r
    return v, dv


@pytest.mark.parametrize("k", [10.0, 15.0])
def test_calderon_identities_on_star(k):
    """(D - 1/2) v - S dv = 0 and -(D* + 1/2) dv + N v = 0 for v radiating from a point
    inside; (D + 1/2) w - S dw = 0 and -(D* - 1/2) dw + N w = 0 for a source outside."""
    w = W.star_grid(1, n=128, k_ext=k, k_int=k)
    S, D, Ds, N = layer.self_blocks(w.x, w.y, w.dx, w.dy, w.ddx, w.ddy, k)
    speed, nx, ny, _, _ = layer.boundary_quantities(w.dx, w.dy, w.ddx, w.ddy, w.node_off)
    I = np.eye(128)
    v, dv = _point_source(w.x, w.y, nx, ny, (0.05, -0.03), k)
    r1 = (D - I / 2) @ v - S @ dv
    r2 = -(Ds + I / 2) @ dv + N @ v
    assert np.max(np.abs(r1)) < 1e-11 * np.max(np.abs(v))
    assert np.max(np.abs(r2)) < 1e-9 * np.max(np.abs(dv))
    v, dv = _point_source(w.x, w.y, nx, ny, (0.9, 0.7), k)
    r1 = (D + I / 2) @ v - S @ dv
    r2 = -(Ds - I / 2) @ dv + N @ v
    assert np.max(np.abs(r1)) < 1e-11 * np.max(np.abs(v))
    assert np.max(np.abs(r2)) < 1e-9 * np.max(np.abs(dv))


def test_single_disk_against_mie():
    w = W.single_disk(n=64, angles=[0.0, 0.7])
    g = dense.Geometry(w)
    phi = dense.solve(w)
    q, u = dense.split_density(g, phi)
    th = 2 * np.pi * np.arange(64) / 64
    ep, em = dense.materials(w)
    for c, a in enumerate(w.angles):
        qm, um = analytic.mie_boundary(th, w.k_ext, w.k_int[0], 0.4, ep, em[0], angle=a)
        ref = np.concatenate([qm, um])
        assert np.linalg.norm(np.concatenate([q[:, c], u[:, c]]) - ref) / np.linalg.norm(ref) < 1e-13
        ff = dense.far_field(g, phi[:, c:c + 1], th)[:, 0]
        ffm = analytic.mie_far_field(th, w.k_ext, w.k_int[0], 0.4, ep, em[0], angle=a)
        assert np.max(np.abs(ff - ffm)) < 1e-13 * np.max(np.abs(ffm))


def test_graf_translation_formula():
    """The multipole translation used by the multi-disk reference, against direct evaluation."""
    k = 2 * np.pi
    cj, cl = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    x = cj + np.array([0.21, -0.13])
    dvec = cj - cl
    b, phi = np.hypot(*dvec), np.arctan2(dvec[1], dvec[0])
    rj, tj = np.hypot(*(x - cj)), np.arctan2(*(x - cj)[::-1])
    rl, tl = np.hypot(*(x - cl)), np.arctan2(*(x - cl)[::-1])
    for m in (-3, 0, 2, 5):
        lhs = sp.hankel1(m, k * rl) * np.exp(1j * m * tl)
        ns = np.arange(-60, 61)
        rhs = np.sum(sp.hankel1(m - ns, k * b) * np.exp(1j * (m - ns) * phi) * sp.jv(ns, k * rj)
                     * np.exp(1j * ns * tj))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("n,tol", [(64, 5e-9), (128, 1e-11)])
def test_two_by_two_disks_against_multipole(n, tol):
    """Dense Nystrom solve of the 2x2 disk grid against the multipole solution."""
    w = W.disk_grid(2, n=n)
    g = dense.Geometry(w)
    phi = dense.solve(w)
    ep, em = dense.materials(w)
    bnd, _, _ = analytic.multi_disk(w.centers, 0.4, w.k_ext, w.k_int[0], ep, em[0])
    th = 2 * np.pi * np.arange(n) / n
    ref = np.concatenate([np.concatenate(bnd(j, th)) for j in range(4)])
    assert dense.rel_error(phi[:, 0], ref) < tol
    assert np.max(np.abs(dense.energy_defect(g, phi))) < 1e-11


def test_optical_theorem_and_reciprocity():
    """int |u_inf|^2 = -sqrt(8 pi/k) Re(e^{i pi/4} u_inf(a)); u_inf(t; a) = u_inf(a+pi; t+pi)."""
    w = W.star_grid(2, n=128, k_ext=10.0, k_int=15.0, seed=2,
                    angles=2 * np.pi * np.arange(4) / 4)
    g = dense.Geometry(w)
    phi = dense.solve(w)
    nd = 720
    th = 2 * np.pi * np.arange(nd) / nd
    ff = dense.far_field(g, phi, th)
    k = w.k_ext
    for c, a in enumerate(w.angles):
        lhs = np.sum(np.abs(ff[:, c]) ** 2) * 2 * np.pi / nd
        f0 = dense.far_field(g, phi[:, c:c + 1], np.array([a]))[0, 0]
        rhs = -np.sqrt(8 * np.pi / k) * np.real(np.exp(1j * np.pi / 4) * f0)
        assert abs(lhs - rhs) < 1e-9 * lhs
    A = dense.far_field(g, phi, w.angles)        # A[i, j] = u_inf(angle_i; incidence angle_j)
    for i in range(4):
        for j in range(4):
            assert abs(A[i, j] - A[(j + 2) % 4, (i + 2) % 4]) < 1e-9 * np.max(np.abs(A))
    assert np.max(np.abs(dense.energy_defect(g, phi))) < 1e-10


def test_paper_dof_table():
    """N = 2 n m unknowns (Sec. 4, Table tb:dof), for the star grids at n = 200."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "table_dof.txt"))
            if l.strip() and not l.startswith("#")]
    for m, dof in rows:
        g = int(round(np.sqrt(int(m))))
        w = W.star_grid(1, n=200)
        assert g * g * w.n_unknowns == int(dof)


def test_fast_method_against_dense_2x2_disks():
    """Every leaf ID is full rank at this geometry: the fast method reproduces LU."""
    w = W.config1()
    ref = dense.solve(w)
    fs = fast.FastSolver(w)
    assert dense.rel_error(fs.solve(), ref) < 1e-12
    assert fs.root_size() == 512


@pytest.mark.parametrize("tol,bound", [(1e-10, 5e-9), (1e-6, 5e-5)])
def test_fast_method_tracks_tolerance(tol, bound):
    w = W.sub_grid(W.config2(), 4)
    w.id_tol = tol
    ref = dense.solve(w)
    fs = fast.FastSolver(w)
    err = dense.rel_error(fs.solve(), ref)
    assert err < bound
    assert err > 1e-3 * tol        # it does compress: not an exact solve
    assert fs.root_size() < w.n_unknowns // 4


def test_id_residual_and_rank_on_proxy_matrices():
    """ID of a leaf's proxy/near matrix: residual ~ tol, rank >= SVD tol-rank."""
    w = W.sub_grid(W.config2(), 4)
    fs = fast.FastSolver.__new__(fast.FastSolver)
    fs.w, fs.g, fs.tol = w, dense.Geometry(w), w.id_tol
    fs.levels = fast.plan(w)
    cells = fs.levels[0]
    acts = [fs._leaf_active(c) for c in cells]
    mats = fs._id_matrices(cells[5], acts[5], acts, cells)
    for key, M in mats.items():
        R, piv, k = fast.cpqr_id(M, w.id_tol)
        Z = fast.interp_matrix(R, piv, k, M.shape[1])
        res = np.linalg.norm(M - M[:, piv[:k]] @ Z, 2) / np.linalg.norm(M, 2)
        s = np.linalg.svd(M, compute_uv=False)
        svd_rank = int(np.sum(s > w.id_tol * s[0]))
        assert res < 50 * w.id_tol, key
        assert k >= svd_rank - 2, key


def test_planted_sign_error_is_caught():
    """A plausible mistake in the oracle (the sign of D*) breaks the Calderon pin."""
    w = W.star_grid(1, n=128, k_ext=10.0, k_int=10.0)
    S, D, Ds, N = layer.self_blocks(w.x, w.y, w.dx, w.dy, w.ddx, w.ddy, 10.0)
    _, nx, ny, _, _ = layer.boundary_quantities(w.dx, w.dy, w.ddx, w.ddy, w.node_off)
    v, dv = _point_source(w.x, w.y, nx, ny, (0.05, -0.03), 10.0)
    I = np.eye(128)
    good = np.max(np.abs(-(Ds + I / 2) @ dv + N @ v))
    bad = np.max(np.abs(-(-Ds + I / 2) @ dv + N @ v))
    assert good < 1e-9 * np.max(np.abs(dv)) < bad


def test_planted_missing_interior_term_is_caught():
    """Dropping the interior wavenumber from the diagonal block breaks the Mie pin."""
    w = W.single_disk(n=64)
    g = dense.Geometry(w)
    A = dense.diagonal_block(g, 0)
    s = (w.x, w.y, w.dx, w.dy, w.ddx, w.ddy)
    Sm, Dm, Dsm, Nm = layer.self_blocks(*s, w.k_int[0])
    em = g.eps_m[0]
    A_bad = A - np.block([[-em * Sm, Dm], [-Dsm, Nm / em]])
    f = dense.rhs(g, [0.0])[:, 0]
    th = 2 * np.pi * np.arange(64) / 64
    qm, um = analytic.mie_boundary(th, w.k_ext, w.k_int[0], 0.4, g.eps_p, em)
    ref = np.concatenate([qm, um])
    good = np.linalg.norm(np.linalg.solve(A, f) - ref) / np.linalg.norm(ref)
    bad = np.linalg.norm(np.linalg.solve(A_bad, f) - ref) / np.linalg.norm(ref)
    assert good < 1e-13 and bad > 1e-2


# ---- skeleton-proposal network oracle --------------------------------------------------
def _mlp_case(shape, B, seed):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    _, npar = mlp.offsets(shape)
    p = rng.standard_normal(npar) * 0.5
    X = rng.standard_normal((B, shape[0]))
    ns = shape[3] // 2
    Y = np.concatenate([(rng.random((B, ns)) < 0.4).astype(float), rng.random((B, shape[3] - ns))], axis=1)
    return p, X, Y


def test_mlp_gradient_matches_finite_differences():
    """The hand-written backward pass against central differences of the loss."""
    from oracle import mlp
    shape = (5, 7, 2, 4)
    p, X, Y = _mlp_case(shape, 6, 3)
    _, L, g = mlp.value_and_grad(p, shape, X, Y, 3.0)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.value_and_grad(p + e, shape, X, Y, 3.0)[1] - mlp.value_and_grad(p - e, shape, X, Y, 3.0)[1]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-7 * max(1.0, np.abs(g).max())


def test_mlp_without_hidden_layers_is_logistic_regression():
    """No hidden layer and no regression weight: the gradient of the mean binary cross
    entropy of a linear model is X^T (sigmoid(z) - y) / B (closed form)."""
    from oracle import mlp
    shape = (3, 1, 0, 2)
    p, X, Y = _mlp_case(shape, 9, 4)
    out, L, g = mlp.value_and_grad(p, shape, X, Y, 0.0)
    (W, b), = mlp.unpack(p, shape)
    z = X @ W.T + b
    assert np.allclose(out, z)
    s = 1.0 / (1.0 + np.exp(-z[:, :1]))
    gW = np.zeros_like(W)
    gW[0] = ((s[:, 0] - Y[:, 0])[:, None] * X).mean(axis=0)
    gb = np.array([(s[:, 0] - Y[:, 0]).mean(), 0.0])
    gref = mlp.pack([(gW, gb)])
    assert np.allclose(g, gref, rtol=0, atol=1e-14)
    Lref = np.mean(-Y[:, 0] * np.log(s[:, 0]) - (1 - Y[:, 0]) * np.log(1 - s[:, 0]))
    assert abs(L - Lref) < 1e-12


def test_residual_rows_equal_rows_of_the_assembled_system():
    """residual_rows builds each row of f - A phi on its own (Kress self block of the row's
    inclusion, trapezoid sums over every other inclusion).  The assembled system is pinned
    by the Mie, multipole and Calderon tests; the row evaluation must reproduce its rows for
    any phi, on q-rows and u-rows of the first, an inner and the last inclusion (Sec. 2.2,
    block system)."""
    w = W.star_grid(3, n=32, k_ext=10.0, k_int=15.0, seed=2, angles=[0.0, 1.1])
    g = dense.Geometry(w)
    A = dense.assemble(g)
    f = dense.rhs(g, w.angles)
    rng = np.random.default_rng(11)
    phi = rng.standard_normal((A.shape[0], 2)) + 1j * rng.standard_normal((A.shape[0], 2))
    last = A.shape[0] - 1
    rows = np.array([0, 31, 32, 63, 64 * 4 + 7, 64 * 4 + 40, last - 32, last])
    got = dense.residual_rows(w, phi, rows)
    ref = (f - A @ phi)[rows]
    scale = (np.abs(A) @ np.abs(phi) + np.abs(f))[rows]
    assert np.all(np.abs(got - ref) <= 1e-14 * scale * 10), np.max(np.abs(got - ref) / scale)
    # a row of the wrong block type or inclusion is far off: the check has teeth
    wrong = (f - A @ phi)[(rows + 1) % A.shape[0]]
    assert np.min(np.abs(wrong - got) / scale) > 1e-6
    # at the dense solution the sampled residual vanishes to rounding
    x = dense.solve(w)
    r = dense.residual_rows(w, x, rows)
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(f[rows])


def test_residual_rows_vanish_at_the_multipole_solution():
    """The closed-form (multipole) boundary data of the 2x2 disks leaves a residual at
    discretisation level in every sampled row (Sec. 4.2 measures errors against such a
    reference); a density off by 1e-6 does not."""
    w = W.disk_grid(2, n=128, angles=[0.0])
    g = dense.Geometry(w)
    ep, em = dense.materials(w)
    bnd, _, _ = analytic.multi_disk(w.centers, 0.4, w.k_ext, w.k_int[0], ep, em[0])
    th = 2 * np.pi * np.arange(128) / 128
    phi = np.concatenate([np.concatenate(bnd(j, th)) for j in range(4)])[:, None]
    rows = np.arange(0, 1024, 37)
    f = dense.rhs(g, w.angles)[rows]
    r = dense.residual_rows(w, phi, rows)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(f)
    bad = phi * (1 + 1e-6)
    assert np.linalg.norm(dense.residual_rows(w, bad, rows)) > 1e-8 * np.linalg.norm(f)


def test_energy_defect_closed_form_for_a_centred_point_source():
    """u = (i/4) H0(k|x - z|) and q = du/dn on a circle of radius R about z: the radiated
    flux gives Im int conj(u) du/dn ds = 1/4 (Green's identity out to infinity), and
    |u|, |du/dn| are constant, so the defect is exactly 2 / (pi k R |H0(kR)| |H1(kR)|)."""
    k, R = 7.0, 0.4
    w = W.disk_grid(1, n=64, radius=R, k_ext=k, k_int=k)
    g = dense.Geometry(w)
    v, dv = _point_source(w.x, w.y, g.nx, g.ny, (0.0, 0.0), k)
    ed = dense.energy_defect(g, np.concatenate([dv, v])[:, None])
    ref = 2.0 / (np.pi * k * R * abs(sp.hankel1(0, k * R)) * abs(sp.hankel1(1, k * R)))
    assert abs(ed[0, 0] - ref) <= 1e-13 * ref
    assert ref > 1e-3


def test_energy_defect_sees_a_source_inside_a_star():
    """For a point source inside a star the weighted sum Im sum_b w_b conj(u_b) q_b is the
    radiated flux 1/4 (trapezoid rule, spectrally accurate); for one outside it is 0."""
    k = 10.0
    w = W.star_grid(1, n=128, k_ext=k, k_int=k)
    g = dense.Geometry(w)
    for z, flux in (((0.05, -0.03), 0.25), ((0.9, 0.7), 0.0)):
        v, dv = _point_source(w.x, w.y, g.nx, g.ny, z, k)
        ed = dense.energy_defect(g, np.concatenate([dv, v])[:, None])[0, 0]
        norm = np.sum(g.wt * np.abs(v) * np.abs(dv))
        assert abs(ed * norm - flux) <= 1e-12 * norm, (z, ed * norm)
    # a lossless transmission solution has none (Sec. 2.1 with real k+, k-)
    x = dense.solve(W.star_grid(1, n=128, k_ext=k, k_int=15.0, angles=[0.3]))
    assert np.max(np.abs(dense.energy_defect(g, x))) < 1e-11


# ---------------------------------------------------------------------------------
# zeta-corrected trapezoid rule (the paper's self-interaction quadrature, Sec. 2.2)

@pytest.mark.parametrize("n", [64, 100])
def test_zeta_rule_on_log_times_trig(n):
    """int_0^2pi cos(m u) ln|2 sin(u/2)| du = -pi/m and int ln|2 sin(u/2)| du = 0 (closed
    forms): the 41-point corrected rule reproduces them for resolved m."""
    h = 2 * np.pi / n
    u = h * np.arange(n)
    with np.errstate(divide="ignore"):
        L = np.log(np.abs(2 * np.sin(u / 2)))
    L[0] = 0.0
    for m in range(0, 9):
        K = np.zeros((n, n))
        A = np.zeros((n, n))
        K[0] = np.cos(m * u) * L
        A[0] = np.cos(m * u)
        got = layer.zeta_corrected(K, A, np.zeros(n))[0].sum().real
        exact = 0.0 if m == 0 else -np.pi / m
        assert abs(got - exact) < 1e-13, (m, got, exact)


def test_zeta_rule_order():
    """The plain punctured trapezoid with only the ln(h/2pi) term is O(h^3); the corrected
    rule removes that error: on an integrand whose log coefficient has a tenth-order
    Taylor expansion the two differ by the leading Navot term 2 zeta'(-2) A''(0) h^3 / 2."""
    import mpmath as mp
    n = 64
    h = 2 * np.pi / n
    u = h * np.arange(n)
    with np.errstate(divide="ignore"):
        L = np.log(np.abs(2 * np.sin(u / 2)))
    L[0] = 0.0
    A0 = np.cos(u)          # A''(0) = -1
    K = np.zeros((n, n))
    A = np.zeros((n, n))
    K[0] = A0 * L
    A[0] = A0
    corrected = layer.zeta_corrected(K, A, np.zeros(n), p=1)[0].sum().real
    plain = h * (K[0, 1:].sum() + np.log(h / (2 * np.pi)))
    lead = 2 * float(mp.zeta(-2, derivative=1)) * (-1.0) * h ** 3 / 2
    assert abs((corrected - plain) - lead) < 1e-3 * abs(lead)


@pytest.mark.parametrize("k", [2 * np.pi, 4 * np.pi])
def test_zeta_circle_eigenvalues(k):
    """Zeta-corrected S, D, D* and N on a circle against the Graf closed forms, on the
    modes the 41-point stencil resolves (|l| <= n/8)."""
    n, R = 128, 0.4
    w = _circle(n, R)
    S, D, Ds, N = layer.self_blocks_zeta(w.x, w.y, w.dx, w.dy, w.ddx, w.ddy, k)
    t = 2 * np.pi * np.arange(n) / n
    z = k * R
    for l in range(-n // 8, n // 8 + 1):
        e = np.exp(1j * l * t)
        J, H, Jp, Hp = sp.jv(l, z), sp.hankel1(l, z), sp.jvp(l, z), sp.h1vp(l, z)
        lamS = 1j * np.pi * R / 2 * J * H
        lamD = 1j * np.pi * k * R / 4 * (Jp * H + J * Hp)
        lamN = 1j * np.pi * k * k * R / 2 * Jp * Hp
        for M, lam, tol in ((S, lamS, 1e-13), (D, lamD, 1e-13), (Ds, lamD, 1e-13), (N, lamN, 1e-11)):
            err = np.max(np.abs(M @ e - lam * e))
            assert err <= tol * max(1.0, abs(lam)), (l, err, lam)


def test_zeta_and_kress_agree_on_a_star():
    """Two independent quadratures of the same operators on a star (k = 10), applied to a
    smooth density: their difference is the zeta rule's own error, which must fall fast
    with n (high order) and be below 1e-11 at n = 256."""
    diffs = {}
    for n in (128, 256):
        w = W.star_grid(1, n=n, k_ext=10.0, k_int=10.0)
        args = (w.x, w.y, w.dx, w.dy, w.ddx, w.ddy, 10.0)
        Z = layer.self_blocks_zeta(*args)
        Kr = layer.self_blocks(*args)
        t = 2 * np.pi * np.arange(n) / n
        phi = np.exp(np.cos(t)) * (1 + 0.3j * np.sin(2 * t))
        diffs[n] = [np.max(np.abs(a @ phi - b @ phi)) / np.max(np.abs(b @ phi)) for a, b in zip(Z, Kr)]
    assert max(diffs[256]) < 1e-11, diffs
    assert diffs[256][0] < 1e-3 * diffs[128][0], diffs   # S: convergence order above 10


def test_zeta_single_disk_against_mie():
    """The dense solve with zeta-corrected self blocks on one disk matches the Mie series."""
    import dataclasses
    w = dataclasses.replace(W.single_disk(n=128, angles=[0.0, 0.7]), quadrature="zeta")
    g = dense.Geometry(w)
    x = dense.solve(w)
    q, u = dense.split_density(g, x)
    th = 2 * np.pi * np.arange(128) / 128
    for c, a in enumerate(w.angles):
        qm, um = analytic.mie_boundary(th, w.k_ext, w.k_int[0], 0.4, g.eps_p, g.eps_m[0], angle=a)
        assert np.max(np.abs(u[:, c] - um)) < 1e-10 * np.max(np.abs(um))
        assert np.max(np.abs(q[:, c] - qm)) < 1e-10 * np.max(np.abs(qm))


def test_device_zeta_table_matches_the_oracle_weights():
    """The library's generated weight table (its own derivation: exact Lagrange derivative
    weights times zeta') against the oracle's moment-system solution."""
    import os
    import re
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2603_09381_amd", "csrc", "zeta_table.h")
    vals = [float(v) for v in re.findall(r"^\s+([-0-9.e+]+),", open(path).read(), re.M)]
    w = layer.zeta_weights()
    assert len(vals) == len(w)
    assert np.max(np.abs(np.array(vals) - w)) < 1e-15
