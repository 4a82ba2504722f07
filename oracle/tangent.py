"""Tangent-linear oracle of the pseudo-time solver -- TEST INFRASTRUCTURE ONLY.

Nothing in the product imports this module; tests use it to check the
discrete adjoint of the HIP library.

It runs the explicit pseudo-time step of the buoyancy-driven cavity (Sec. 2,
Eq. 1-3; wall rules and centre rescale of Sec. 2; second-order central
differences and the fourth-difference pressure dissipation of Sec. 3.1) in
complex arithmetic and differentiates by the complex step (Squire & Trapp,
SIAM Rev. 1998; Martins, Sturdza & Alonso, ACM TOMS 2003): for inputs
x + i*h*v with h = 1e-30, the imaginary part of any output divided by h is
its directional derivative along v, exact to rounding, with no subtractive
cancellation.  Every operation here is complex-analytic except |.|, max and
min, which are taken on the real part and carry the imaginary part of the
branch they select: |u| has slope +1 at u = 0, max/min follow the first
argument only where it is strictly larger/smaller.

The discretisation is written out again in numpy (whole-array slices of a
ghost-filled array, numpy's operation order), independently of the C oracle
and of the HIP path; the readings of the paper are the same ones:
  nu = sqrt(Pr/Ra), alpha = 1/sqrt(Ra Pr), buoyancy +(T - t_inf) along z,
  beta^2 = max(|V|^2, kappa u_ref^2), lambda_i = (|V_i| + sqrt(V_i^2 + 4 beta^2))/2,
  R_p = -beta^2 div V - eps4 sum_i lambda_i F_i p / h_i,
  dt = cfl min(1 / sum_i lambda_i/h_i, 1 / (2 max(nu, alpha) sum_i 1/h_i^2)),
  q <- q + dt R, then p <- p - p(ni/2, nj/2, nk/2);
  ghosts: p linear extrapolation, u v w odd, T odd about the wall value on
  x = 0 (Theta) and x = 1 (t_cold), even on the other walls;
  Nu = mean over (j, k) of -(9 T_0 - T_1 - 8 Theta) / (3 h) / (t_hot - t_cold).

Pinned in tests/test_oracle_tangent.py: its real part against the C oracle,
its derivatives against central finite differences of the C oracle, and its
zero-step derivatives against the closed form.
"""
import numpy as np

NG = 2
H_STEP = 1e-30


def _abs(z):
    return np.where(z.real < 0, -z, z)


def _max(a, b):
    return np.where(np.real(a) > np.real(b), a, b)


def _min(a, b):
    return np.where(np.real(a) < np.real(b), a, b)


class Case:
    """Grid and parameters; Ra and theta (nj*nk hot-wall temperatures, j
    fastest) may be complex."""

    def __init__(self, ni, nj, nk, Ra, theta, Pr=0.71, cfl=0.5, eps4=1.0 / 16, kappa=0.25,
                 u_ref=1.0, t_hot=1.0, t_cold=0.0, t_inf=0.5):
        self.ni, self.nj, self.nk = ni, nj, nk
        self.Ra, self.Pr, self.cfl, self.eps4 = Ra, Pr, cfl, eps4
        self.floor = kappa * u_ref * u_ref
        self.t_hot, self.t_cold, self.t_inf = t_hot, t_cold, t_inf
        self.theta = np.asarray(theta).reshape(nk, nj)


def _sl(n, d):
    return slice(NG + d, NG + d + n)


def apply_bc(C, q):
    """Fill the face ghosts (two layers) of q, shape (5, nk+4, nj+4, ni+4)."""
    ni, nj, nk = C.ni, C.nj, C.nk
    K, J, I = _sl(nk, 0), _sl(nj, 0), _sl(ni, 0)

    def fill(f, axis, lo, wall):
        # index tuple of layer m counted from the wall into the cavity (m = 0, 1)
        # and of ghost g = 1, 2 beyond it
        def at(pos):
            idx = [f, K, J, I]
            idx[3 - axis] = pos
            return tuple(idx)
        n = (ni, nj, nk)[axis]
        m0, m1 = (NG, NG + 1) if lo else (NG + n - 1, NG + n - 2)
        g1, g2 = (NG - 1, NG - 2) if lo else (NG + n, NG + n + 1)
        a, b = q[at(m0)], q[at(m1)]
        if f == 0:
            e1 = 2 * a - b
            q[at(g1)], q[at(g2)] = e1, 2 * e1 - a
        elif f in (1, 2, 3):
            q[at(g1)], q[at(g2)] = -a, -b
        elif wall is None:
            q[at(g1)], q[at(g2)] = a, b
        else:
            q[at(g1)], q[at(g2)] = 2 * wall - a, 2 * wall - b

    for f in range(5):
        fill(f, 0, True, C.theta if f == 4 else None)
        fill(f, 0, False, C.t_cold if f == 4 else None)
        for axis in (1, 2):
            fill(f, axis, True, None)
            fill(f, axis, False, None)


def residual(C, q):
    """R (5, nk, nj, ni) and dt (nk, nj, ni) of a ghost-filled state."""
    ni, nj, nk = C.ni, C.nj, C.nk
    nx, ny, nz = float(ni), float(nj), float(nk)

    def Q(f, di=0, dj=0, dk=0):
        return q[f, _sl(nk, dk), _sl(nj, dj), _sl(ni, di)]

    nu = np.sqrt(C.Pr / C.Ra)
    alpha = 1.0 / np.sqrt(C.Ra * C.Pr)
    p, u, v, w, T = (Q(f) for f in range(5))
    Dx = [(Q(f, 1) - Q(f, -1)) * (nx / 2) for f in range(5)]
    Dy = [(Q(f, 0, 1) - Q(f, 0, -1)) * (ny / 2) for f in range(5)]
    Dz = [(Q(f, 0, 0, 1) - Q(f, 0, 0, -1)) * (nz / 2) for f in range(5)]
    lap = [(Q(f, 1) + Q(f, -1) - 2 * Q(f)) * nx ** 2 + (Q(f, 0, 1) + Q(f, 0, -1) - 2 * Q(f)) * ny ** 2
           + (Q(f, 0, 0, 1) + Q(f, 0, 0, -1) - 2 * Q(f)) * nz ** 2 for f in range(5)]
    Fx = Q(0, 2) + Q(0, -2) - 4 * (Q(0, 1) + Q(0, -1)) + 6 * p
    Fy = Q(0, 0, 2) + Q(0, 0, -2) - 4 * (Q(0, 0, 1) + Q(0, 0, -1)) + 6 * p
    Fz = Q(0, 0, 0, 2) + Q(0, 0, 0, -2) - 4 * (Q(0, 0, 0, 1) + Q(0, 0, 0, -1)) + 6 * p

    beta2 = _max(u * u + v * v + w * w, C.floor)
    lx = (_abs(u) + np.sqrt(u * u + 4 * beta2)) / 2
    ly = (_abs(v) + np.sqrt(v * v + 4 * beta2)) / 2
    lz = (_abs(w) + np.sqrt(w * w + 4 * beta2)) / 2
    dt_visc = 1.0 / (2 * _max(nu, alpha) * (nx ** 2 + ny ** 2 + nz ** 2))
    dt = C.cfl * _min(1.0 / (lx * nx + ly * ny + lz * nz), dt_visc)

    def adv(f):
        return u * Dx[f] + v * Dy[f] + w * Dz[f]

    R = np.empty((5,) + p.shape, dtype=np.result_type(q, C.Ra))
    R[0] = -beta2 * (Dx[1] + Dy[2] + Dz[3]) - C.eps4 * (lx * Fx * nx + ly * Fy * ny + lz * Fz * nz)
    R[1] = -adv(1) - Dx[0] + nu * lap[1]
    R[2] = -adv(2) - Dy[0] + nu * lap[2]
    R[3] = -adv(3) - Dz[0] + nu * lap[3] + (T - C.t_inf)
    R[4] = -adv(4) + alpha * lap[4]
    return R, dt


def step(C, q):
    """One step: a new ghost-filled-size state (ghosts not filled)."""
    qq = q.astype(np.result_type(q, C.Ra, C.theta), copy=True)
    apply_bc(C, qq)
    R, dt = residual(C, qq)
    out = np.zeros_like(qq)
    inner = (slice(None), _sl(C.nk, 0), _sl(C.nj, 0), _sl(C.ni, 0))
    out[inner] = qq[inner] + dt * R
    out[0, _sl(C.nk, 0), _sl(C.nj, 0), _sl(C.ni, 0)] -= out[0, NG + C.nk // 2, NG + C.nj // 2, NG + C.ni // 2]
    return out


def nusselt(C, q):
    T0 = q[4, _sl(C.nk, 0), _sl(C.nj, 0), NG]
    T1 = q[4, _sl(C.nk, 0), _sl(C.nj, 0), NG + 1]
    flux = -(9 * T0 - T1 - 8 * C.theta) * (C.ni / 3.0)
    return flux.mean() / (C.t_hot - C.t_cold)


def run(C, q0, nsteps):
    q = q0
    for _ in range(nsteps):
        q = step(C, q)
    return q


def nusselt_tangent(ni, nj, nk, Ra, theta, q0, nsteps, dq=None, dtheta=None, dRa=0.0, h=H_STEP, **kw):
    """(Nu after nsteps, its directional derivative along (dq, dtheta, dRa)).
    q0, dq: (5, nk+4, nj+4, ni+4) arrays (ghosts ignored); theta, dtheta:
    nj*nk hot-wall temperatures, j fastest."""
    zq = np.asarray(q0, dtype=np.complex128).copy()
    if dq is not None:
        zq += 1j * h * np.asarray(dq)
    zt = np.asarray(theta, dtype=np.complex128).copy()
    if dtheta is not None:
        zt += 1j * h * np.asarray(dtheta)
    C = Case(ni, nj, nk, complex(Ra, h * dRa), zt, **kw)
    J = nusselt(C, run(C, zq, nsteps))
    return float(J.real), float(J.imag / h)


def state_after(ni, nj, nk, Ra, theta, q0, nsteps, **kw):
    """Real state after nsteps (for pinning against the C oracle)."""
    C = Case(ni, nj, nk, Ra, np.asarray(theta, dtype=np.float64), **kw)
    return run(C, np.asarray(q0, dtype=np.float64), nsteps)
