"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: exact
steady states, one-step closed forms, a manufactured solution with its
continuous residual derived symbolically, exact mirror symmetry, published
generator outputs, and the index formulas of the paper's listings.  They are
chosen so that a dropped term, a wrong sign, index or scale, or a transposed
operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle as O

NG = O.NG


def cell_centres(n):
    return (np.arange(n) + 0.5) / n


def interior(P, q):
    return P.interior(q)


def set_interior(P, q, f, values):
    q[f, NG:NG + P.nk, NG:NG + P.nj, NG:NG + P.ni] = values


def grids(P):
    z, y, x = np.meshgrid(cell_centres(P.nk), cell_centres(P.nj), cell_centres(P.ni), indexing="ij")
    return x, y, z


# --------------------------------------------------------------------------
# Generator (input recipe): SplitMix64 outputs of the published reference
# implementation for seed 0 (Vigna's splitmix64.c; Steele, Lea & Flood 2014).
def test_splitmix64_published_vectors(orc):
    assert O.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert O.splitmix64(0, 2) == 0x06C45D188009454F


def test_init_recipe(orc):
    """Noise within +-amp and centred, p = 0, T linear in x up to the noise,
    different seeds give different fields, same seed the same bits."""
    P = O.Problem(12, 10, 8)
    q = O.init(P, 7, 1e-3)
    I = interior(P, q)
    assert np.all(I[0] == 0.0)
    for f in (1, 2, 3):
        assert np.abs(I[f]).max() <= 1e-3 and abs(I[f].mean()) < 2e-4
        assert np.abs(I[f]).max() > 0.9e-3
    x, _, _ = grids(P)
    assert np.abs(I[4] - (1.0 - x)).max() <= 1e-3 + 1e-15
    assert np.array_equal(q, O.init(P, 7, 1e-3))
    assert not np.array_equal(q, O.init(P, 8, 1e-3))


# --------------------------------------------------------------------------
# P1: quiescent isothermal state stays exactly at rest.
def test_quiescent_rest_is_exact(orc):
    P = O.Problem(8, 10, 12, t_hot=0.5, t_cold=0.5, t_inf=0.5)
    q = O.init(P, 1, 0.0)
    q0 = q.copy()
    norms = O.step(P, q, 30, halo=((2, 1, 2), (2, 1, 1, 1, 1)))
    I, I0 = interior(P, q), interior(P, q0)
    assert np.array_equal(I, I0)
    assert np.all(I[:4] == 0.0) and np.all(I[4] == 0.5)
    assert np.all(norms == 0.0)


# --------------------------------------------------------------------------
# P2: hydrostatic balance.  Uniform T != t_inf, V = 0 and a linear pressure
# with dp/dz = T - t_inf is a steady state: buoyancy balances the pressure
# gradient (sign and scale of both), and linear extrapolation keeps p linear
# at the z walls (a mirror BC would not).
def test_hydrostatic_balance(orc):
    P = O.Problem(10, 8, 16, t_hot=0.75, t_cold=0.75, t_inf=0.5, Ra=1e4)
    q = P.zeros()
    _, _, z = grids(P)
    set_interior(P, q, 0, 0.25 * (z - 0.5))
    set_interior(P, q, 4, np.full(z.shape, 0.75))
    O.step(P, q, 40)
    I = interior(P, q)
    assert np.abs(I[1:4]).max() < 1e-14
    zc = (P.nk // 2 + 0.5) / P.nk
    assert np.abs(I[0] - 0.25 * (z - zc)).max() < 1e-14
    assert np.all(I[4] == 0.75)


def test_hydrostatic_detects_wrong_buoyancy_sign(orc):
    """The same state with the opposite density difference is not steady."""
    P = O.Problem(8, t_hot=0.25, t_cold=0.25, t_inf=0.5)
    q = P.zeros()
    _, _, z = grids(P)
    set_interior(P, q, 0, 0.25 * (z - 0.5))
    set_interior(P, q, 4, np.full(z.shape, 0.25))
    O.step(P, q, 1)
    assert np.abs(interior(P, q)[3]).max() > 1e-3


# --------------------------------------------------------------------------
# P3: one-step closed forms (cells two or more away from every wall).
def dt_closed(P, lam):
    nu, alpha = math.sqrt(P.Pr / P.Ra), 1.0 / math.sqrt(P.Ra * P.Pr)
    conv = 1.0 / (lam[0] * P.ni + lam[1] * P.nj + lam[2] * P.nk)
    visc = 1.0 / (2.0 * max(nu, alpha) * (P.ni ** 2 + P.nj ** 2 + P.nk ** 2))
    return P.cfl * min(conv, visc)


@pytest.mark.parametrize("Ra", [1e3, 1e7])   # viscous-limited, convective-limited dt
def test_closed_form_buoyancy_from_rest(orc, Ra):
    theta = 0.125
    P = O.Problem(12, 10, 14, Ra=Ra, t_hot=0.5 + theta, t_cold=0.5 + theta, t_inf=0.5)
    q = P.zeros()
    set_interior(P, q, 4, np.full((P.nk, P.nj, P.ni), 0.5 + theta))
    norms = O.step(P, q, 1)
    beta = math.sqrt(P.kappa) * P.u_ref
    dt = dt_closed(P, (beta, beta, beta))
    I = interior(P, q)
    assert np.abs(I[3] - dt * theta).max() <= 1e-15 * dt * theta * 10
    assert np.all(I[0] == 0) and np.all(I[1] == 0) and np.all(I[2] == 0)
    assert np.all(I[4] == 0.5 + theta)
    np.testing.assert_allclose(norms, [0, 0, 0, theta, 0], rtol=1e-14, atol=0)


@pytest.mark.parametrize("U0", [0.0, 0.3, 0.6])     # beta^2 from the floor / from |V|^2
def test_closed_form_pressure_wave(orc, U0):
    """p = a cos(k x), u = U0, v = w = 0, T = t_inf.  Away from the walls:
    R_p = -eps4 lam_x F_x p / h with F_x cos = 16 sin^4(k h / 2) cos,
    R_u = -dp/dx = a sin(kx) sin(kh)/h, R_T = 0; lam from beta^2."""
    P = O.Problem(32, 12, 12, Ra=1e5)
    a, kw = 0.01, 2 * math.pi * 1.5
    q = P.zeros()
    x, _, _ = grids(P)
    set_interior(P, q, 0, a * np.cos(kw * x))
    set_interior(P, q, 1, np.full(x.shape, U0))
    set_interior(P, q, 4, np.full(x.shape, P.t_inf))
    O.apply_bc(P, q)
    R, dt = O.residual(P, q)
    h = 1.0 / P.ni
    beta2 = max(U0 * U0, P.kappa * P.u_ref ** 2)
    lam_x = 0.5 * (U0 + math.sqrt(U0 * U0 + 4 * beta2))
    lam_y = lam_z = math.sqrt(beta2)
    sl = (slice(2, -2), slice(2, -2), slice(2, -2))
    Rp = -P.eps4 * lam_x * 16 * math.sin(kw * h / 2) ** 4 * a * np.cos(kw * x) / h
    Ru = a * np.sin(kw * x) * math.sin(kw * h) / h
    np.testing.assert_allclose(R[0][sl], Rp[sl], rtol=1e-9, atol=1e-12 * abs(Rp).max())
    np.testing.assert_allclose(R[1][sl], Ru[sl], rtol=1e-11, atol=1e-13)
    assert np.abs(R[2][sl]).max() == 0 and np.abs(R[3][sl]).max() == 0
    assert np.abs(R[4][sl]).max() == 0
    np.testing.assert_allclose(dt[sl], dt_closed(P, (lam_x, lam_y, lam_z)), rtol=1e-14)


def test_closed_form_temperature_advection(orc):
    """T = 1 - x (exact with the hot/cold walls), u = U0: R_T = U0 at every
    cell, so T advances by dt*U0 (sign of the advection term)."""
    U0 = 0.2
    P = O.Problem(16, 8, 8, Ra=1e4)
    q = P.zeros()
    x, _, _ = grids(P)
    set_interior(P, q, 4, 1.0 - x)
    set_interior(P, q, 1, np.full(x.shape, U0))
    O.apply_bc(P, q)
    R, dt = O.residual(P, q)
    np.testing.assert_allclose(R[4], U0, rtol=1e-12)


# --------------------------------------------------------------------------
# P4: manufactured solution.  Fields compatible with the wall BCs; the
# continuous residual S is derived symbolically (sympy) from Eq. 1-3.  The
# truncation error R_h(q) - S must fall as h^2 in L-infinity, interior and
# wall cells included.
def _mms_fields():
    sp = pytest.importorskip("sympy")
    x, y, z = sp.symbols("x y z")
    pi = sp.pi
    A = sp.Rational(1, 10)
    u = A * sp.sin(pi * x) * sp.sin(2 * pi * y) * sp.sin(pi * z)
    v = A * sp.sin(2 * pi * x) * sp.sin(pi * y) * sp.sin(pi * z)
    w = A * sp.sin(pi * x) * sp.sin(pi * y) * sp.sin(2 * pi * z)
    T = 1 - x + sp.Rational(1, 5) * sp.sin(pi * x) * sp.cos(pi * y) * sp.cos(pi * z)
    p = sp.Rational(1, 20) * sp.sin(2 * pi * x) * sp.sin(2 * pi * y) * sp.sin(2 * pi * z)
    return sp, (x, y, z), (p, u, v, w, T)


def _continuous_residual(sp, X, F, Ra, Pr, t_inf, beta2):
    x, y, z = X
    p, u, v, w, T = F
    nu, alpha = sp.sqrt(sp.Float(Pr) / Ra), 1 / sp.sqrt(sp.Float(Ra) * Pr)
    grad = lambda s: (sp.diff(s, x), sp.diff(s, y), sp.diff(s, z))
    lap = lambda s: sp.diff(s, x, 2) + sp.diff(s, y, 2) + sp.diff(s, z, 2)
    adv = lambda s: u * grad(s)[0] + v * grad(s)[1] + w * grad(s)[2]
    Sp = -beta2 * (sp.diff(u, x) + sp.diff(v, y) + sp.diff(w, z))
    Su = -adv(u) - sp.diff(p, x) + nu * lap(u)
    Sv = -adv(v) - sp.diff(p, y) + nu * lap(v)
    Sw = -adv(w) - sp.diff(p, z) + nu * lap(w) + (T - t_inf)
    ST = -adv(T) + alpha * lap(T)
    return [sp.lambdify((x, y, z), s, "numpy") for s in (Sp, Su, Sv, Sw, ST)], \
           [sp.lambdify((x, y, z), s, "numpy") for s in F]


@pytest.mark.parametrize("aniso", [(1, 1, 1), (4, 6, 5)])
def test_manufactured_solution_second_order(orc, aniso):
    sp, X, F = _mms_fields()
    Ra, Pr = 40.0, 2.0
    S, Fn = _continuous_residual(sp, X, F, Ra, Pr, 0.5, sp.Rational(1, 4))
    errs = []
    for base in (8, 16, 32):
        n = [base * a // aniso[0] for a in aniso] if aniso == (1, 1, 1) else [base, base * 3 // 2, base * 5 // 4]
        P = O.Problem(n[0], n[1], n[2], Ra=Ra, Pr=Pr)
        q = P.zeros()
        x, y, z = grids(P)
        for f in range(5):
            set_interior(P, q, f, np.broadcast_to(Fn[f](x, y, z), x.shape))
        O.apply_bc(P, q)
        R, _ = O.residual(P, q)
        errs.append([np.abs(R[f] - np.broadcast_to(S[f](x, y, z), x.shape)).max() for f in range(5)])
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order[-1] > 1.85), (errs, order)
    assert np.all(order[-1] < 2.3), (errs, order)


def test_manufactured_solution_catches_planted_mistake(orc):
    """Sanity of the pin itself: a residual with a transposed advection
    operand (v d/dx u instead of v d/dy u) does not converge."""
    sp, X, F = _mms_fields()
    x, y, z = X
    p, u, v, w, T = F
    bad = sp.lambdify((x, y, z), v * sp.diff(u, x) - v * sp.diff(u, y), "numpy")
    S, Fn = _continuous_residual(sp, X, F, 40.0, 2.0, 0.5, sp.Rational(1, 4))
    errs = []
    for n in (16, 32):
        P = O.Problem(n, Ra=40.0, Pr=2.0)
        q = P.zeros()
        xg, yg, zg = grids(P)
        for f in range(5):
            set_interior(P, q, f, np.broadcast_to(Fn[f](xg, yg, zg), xg.shape))
        O.apply_bc(P, q)
        R, _ = O.residual(P, q)
        errs.append(np.abs(R[1] - S[1](xg, yg, zg) + bad(xg, yg, zg)).max())
    assert errs[1] > 0.5 * errs[0]


# --------------------------------------------------------------------------
# P5: symmetries.  Mirror y -> 1 - y maps (p,u,v,w,T) to (p,u,-v,w,T); the
# oracle pairs neighbours commutatively, so it must hold bit for bit.
def _y_symmetric_init(P, seed):
    q = O.init(P, seed, 1e-3)
    I = P.interior(q)
    half = P.nj // 2
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        I[f][:, P.nj - half:, :] = s * I[f][:, :half, :][:, ::-1, :]
    O.apply_bc(P, q)
    return q


def test_y_mirror_symmetry_bit_exact(orc):
    P = O.Problem(16, Ra=1e3)
    q = _y_symmetric_init(P, 3)
    O.step(P, q, 100, halo=((2, 2, 2), (1, 2, 2, 2, 2)))
    I = P.interior(q)
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        assert np.array_equal(I[f], s * I[f][:, ::-1, :]), O.FIELDS[f]
    assert np.abs(I[2]).max() > 0


def test_centro_symmetry(orc):
    """(x, z) -> (1-x, 1-z), T -> 1 - T, u, w odd, v, p even: holds up to
    rounding (1 - T is not exact)."""
    P = O.Problem(12, Ra=1e3)
    q = O.init(P, 4, 1e-3)
    I = P.interior(q)
    r = lambda a: a[::-1, :, ::-1]
    I[0][:] = 0.0
    for f, s in ((1, -1.0), (2, 1.0), (3, -1.0)):
        half = P.ni // 2
        I[f][:, :, half:] = s * r(I[f])[:, :, half:]
    I[4][:, :, P.ni // 2:] = 1.0 - r(I[4])[:, :, P.ni // 2:]
    O.apply_bc(P, q)
    O.step(P, q, 60)
    I = P.interior(q)
    tol = 1e-13
    assert np.abs(I[1] + r(I[1])).max() < tol * max(1.0, np.abs(I[1]).max())
    assert np.abs(I[3] + r(I[3])).max() < tol
    assert np.abs(I[2] - r(I[2])).max() < tol
    assert np.abs(I[4] - (1.0 - r(I[4]))).max() < tol
    # p is even up to the constant fixed by the rescale cell
    d = I[0] - r(I[0])
    assert np.abs(d - d.mean()).max() < tol


# --------------------------------------------------------------------------
# P6: the rescale removes any constant added to p.
def test_pressure_shift_invariance(orc):
    P = O.Problem(10, 12, 8, Ra=1e3)
    q1 = O.init(P, 5, 1e-3)
    O.step(P, q1, 3)
    q2 = q1.copy()
    P.interior(q2)[0] += 0.375
    O.step(P, q1, 5)
    O.step(P, q2, 5)
    d = np.abs(P.interior(q1) - P.interior(q2)).max(axis=(1, 2, 3))
    assert np.all(d < 1e-13), d
    c = P.interior(q1)[0][P.nk // 2, P.nj // 2, P.ni // 2]
    assert c == 0.0


# --------------------------------------------------------------------------
# P8: determinism and restart.
def test_restart_bit_exact(orc):
    P = O.Problem(9, 11, 10, Ra=1e4)
    halo = ((1, 1, 2), (2, 1, 1, 1, 1))
    a = O.init(P, 6, 1e-3)
    b = a.copy()
    na = O.step(P, a, 21, halo=halo)
    O.step(P, b, 10, halo=halo)
    nb = O.step(P, b, 11, halo=halo)
    assert np.array_equal(P.interior(a), P.interior(b))
    assert np.array_equal(na, nb)


# --------------------------------------------------------------------------
# BCs against fields the mirror rules reproduce exactly.
def test_bc_exact_for_compatible_fields(orc):
    P = O.Problem(6, 7, 8, t_hot=1.0, t_cold=0.0)
    q = P.zeros()
    xs = [(np.arange(-NG, n + NG) + 0.5) / n for n in (P.ni, P.nj, P.nk)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    exact = [0.3 + 0.2 * X - 0.1 * Y + 0.4 * Z,                 # p linear: extrapolation exact
             np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(np.pi * Z),
             np.sin(2 * np.pi * X) * np.sin(np.pi * Y) * np.sin(3 * np.pi * Z),
             np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z),
             1.0 - X + 0.1 * np.sin(np.pi * X) * np.cos(np.pi * Y) * np.cos(np.pi * Z)]
    for f in range(5):
        set_interior(P, q, f, exact[f][NG:-NG, NG:-NG, NG:-NG])
    O.apply_bc(P, q)
    for f in range(5):
        g = q[f]
        e = exact[f]
        face_x = (slice(NG, -NG), slice(NG, -NG), np.r_[0:NG, -NG:0])
        face_y = (slice(NG, -NG), np.r_[0:NG, -NG:0], slice(NG, -NG))
        face_z = (np.r_[0:NG, -NG:0], slice(NG, -NG), slice(NG, -NG))
        for sl in (face_x, face_y, face_z):
            np.testing.assert_allclose(g[sl], e[sl], rtol=0, atol=1e-14, err_msg=O.FIELDS[f])


# --------------------------------------------------------------------------
# Hot-wall Nusselt number: the one-sided second-order wall gradient is exact
# for profiles quadratic in x, so pure conduction gives Nu = 1 and
# T = 1 - x + a x (1 - x) gives Nu = 1 - a (dT/dx at the wall is a - 1).
@pytest.mark.parametrize("a", [0.0, 0.3, -0.7])
def test_nusselt_exact_for_quadratic_profiles(orc, a):
    P = O.Problem(12, 7, 9)
    q = P.zeros()
    x, y, z = grids(P)
    set_interior(P, q, 4, 1.0 - x + a * x * (1.0 - x) + 0.0 * y * z)
    assert abs(O.nusselt_hot(P, q) - (1.0 - a)) < 1e-12


def test_nusselt_scales_with_wall_difference_and_field(orc):
    """Nu is relative to t_hot - t_cold, and a per-(j,k) hot-wall field
    enters through its mean for a conduction profile."""
    P = O.Problem(10, 6, 5, t_hot=3.0, t_cold=1.0)
    q = P.zeros()
    x, _, _ = grids(P)
    set_interior(P, q, 4, 3.0 - 2.0 * x)
    assert abs(O.nusselt_hot(P, q) - 1.0) < 1e-12
    field = np.full(P.nj * P.nk, 3.0)
    field[::2] = 3.5
    P2 = O.Problem(10, 6, 5, t_hot=3.0, t_cold=1.0, t_hot_field=field)
    expect = 1.0 + 8.0 * (field.mean() - 3.0) / (3.0 / P.ni) / 2.0
    assert abs(O.nusselt_hot(P2, q) - expect) < 1e-12
