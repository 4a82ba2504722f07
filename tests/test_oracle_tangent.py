"""Pins of the complex-step tangent oracle (oracle/tangent.py).

The tangent oracle is a second, whole-array numpy implementation of the
step; it is pinned to things other than itself:
  * its real part against the C oracle (independent code, same readings);
  * its directional derivatives against central finite differences of the
    C oracle, in the viscous- and the convective-limited time-step regimes,
    along state, hot-wall and Ra directions;
  * its zero-step derivatives against the closed form of the Nusselt
    number's one-sided wall gradient.
"""
import numpy as np
import pytest

import oracle as O
from oracle import tangent as TG

NGC = TG.NG


def start(n, seed, theta_amp=0.05):
    ni, nj, nk = n
    P = O.Problem(ni, nj, nk)
    q0 = O.init(P, seed, 1e-3)
    rng = np.random.default_rng(seed)
    theta = 1.0 + theta_amp * rng.uniform(-1, 1, nj * nk)
    return q0, theta


def c_oracle_nu(n, Ra, theta, q0, nsteps):
    P = O.Problem(*n, Ra=Ra, t_hot_field=theta)
    q = q0.copy()
    O.step(P, q, nsteps)
    return O.nusselt_hot(P, q), P, q


@pytest.mark.parametrize("n,Ra", [((12, 10, 8), 1e5), ((9, 9, 9), 1e3), ((8, 11, 7), 1e6)])
def test_real_part_matches_c_oracle(n, Ra):
    q0, theta = start(n, 11)
    _, P, ref = c_oracle_nu(n, Ra, theta, q0, 10)
    got = TG.state_after(*n, Ra, theta, q0, 10)
    a, b = P.interior(got), P.interior(ref)
    for f in range(5):
        scale = max(np.abs(b[f]).max(), 1e-300)
        assert np.abs(a[f] - b[f]).max() <= 1e-12 * scale, f


def _directions(n, seed):
    ni, nj, nk = n
    rng = np.random.default_rng(seed)
    dq = np.zeros((5, nk + 4, nj + 4, ni + 4))
    dq[:, 2:-2, 2:-2, 2:-2] = rng.uniform(-1, 1, (5, nk, nj, ni))
    dq[0] *= 1e-2                       # pressure varies on a smaller scale here
    dth = rng.uniform(-1, 1, nj * nk)
    return dq, dth


@pytest.mark.parametrize("n,Ra,steps", [((8, 8, 8), 1e3, 8), ((9, 7, 6), 1e6, 8), ((8, 8, 8), 1e5, 12)])
@pytest.mark.parametrize("which", ["q", "theta", "Ra"])
def test_derivative_matches_finite_differences(n, Ra, steps, which):
    q0, theta = start(n, 21)
    dq, dth = _directions(n, 22)
    # Steps: |u| has a kink at u = 0 and the smallest seeded |u| is ~3e-7,
    # so a state step of 1e-6 can straddle it (the difference then averages
    # both slopes) while 1e-7 stays on one side; Theta and Ra move the
    # velocities far less, and larger steps keep rounding small.
    eps = {"q": 1e-7, "theta": 1e-6, "Ra": 1e-5}[which]
    if which == "q":
        kw, plus, minus = dict(dq=dq), (q0 + eps * dq, theta, Ra), (q0 - eps * dq, theta, Ra)
    elif which == "theta":
        kw, plus, minus = dict(dtheta=dth), (q0, theta + eps * dth, Ra), (q0, theta - eps * dth, Ra)
    else:
        kw, plus, minus = dict(dRa=Ra), (q0, theta, Ra * (1 + eps)), (q0, theta, Ra * (1 - eps))
    J, dJ = TG.nusselt_tangent(*n, Ra, theta, q0, steps, **kw)
    Jp = c_oracle_nu(n, plus[2], plus[1], plus[0], steps)[0]
    Jm = c_oracle_nu(n, minus[2], minus[1], minus[0], steps)[0]
    fd = (Jp - Jm) / (2 * eps)
    J0 = c_oracle_nu(n, Ra, theta, q0, steps)[0]
    assert abs(J - J0) <= 1e-12 * abs(J0)
    # truncation O(eps^2) plus rounding of J over the step, ~1e-14 |J| / eps
    assert abs(dJ - fd) <= 1e-6 * abs(fd) + 1e-14 * abs(J0) / eps, (dJ, fd)


def test_zero_step_derivatives_closed_form():
    """Nu = mean over the wall of -(9 T_0 - T_1 - 8 Theta) ni / 3 / dT, so
    dNu/dTheta_jk = 8 ni / (3 nj nk dT), dNu/dT_0 = -9 ni / (3 nj nk dT),
    dNu/dT_1 = ni / (3 nj nk dT)."""
    n = (10, 6, 5)
    ni, nj, nk = n
    q0, theta = start(n, 3)
    base = ni / 3.0 / (nj * nk)
    e = np.zeros(nj * nk)
    e[7] = 1.0
    _, d = TG.nusselt_tangent(*n, 1e4, theta, q0, 0, dtheta=e)
    assert d == pytest.approx(8 * base, rel=1e-14)
    dq = np.zeros_like(q0)
    dq[4, NGC + 2, NGC + 3, NGC] = 1.0
    _, d = TG.nusselt_tangent(*n, 1e4, theta, q0, 0, dq=dq)
    assert d == pytest.approx(-9 * base, rel=1e-14)
    dq[4, NGC + 2, NGC + 3, NGC] = 0.0
    dq[4, NGC + 2, NGC + 3, NGC + 1] = 1.0
    _, d = TG.nusselt_tangent(*n, 1e4, theta, q0, 0, dq=dq)
    assert d == pytest.approx(base, rel=1e-14)
    _, d = TG.nusselt_tangent(*n, 1e4, theta, q0, 0, dRa=1.0)
    assert d == 0.0


def test_tangent_is_linear_in_the_direction():
    n = (8, 7, 6)
    q0, theta = start(n, 5)
    dq, dth = _directions(n, 6)
    _, a = TG.nusselt_tangent(*n, 1e5, theta, q0, 5, dq=dq)
    _, b = TG.nusselt_tangent(*n, 1e5, theta, q0, 5, dtheta=dth)
    _, c = TG.nusselt_tangent(*n, 1e5, theta, q0, 5, dRa=3e4)
    _, abc = TG.nusselt_tangent(*n, 1e5, theta, q0, 5, dq=dq, dtheta=dth, dRa=3e4)
    assert abc == pytest.approx(a + b + c, rel=1e-12, abs=1e-14)


def test_planted_mistake_in_the_tangent_is_caught(monkeypatch):
    """A complex-step derivative is exact for the function as written, so a
    wrong derivative needs a non-analytic operation done wrong: np.abs on a
    complex number returns a real magnitude and drops the imaginary part.
    Planted in the oracle's |.|, the comparison with finite differences of
    the C oracle fails while the real part still agrees."""
    n, Ra, steps = (8, 8, 8), 1e6, 8
    q0, theta = start(n, 21)
    dq, _ = _directions(n, 22)
    eps = 1e-7
    fd = (c_oracle_nu(n, Ra, theta, q0 + eps * dq, steps)[0] - c_oracle_nu(n, Ra, theta, q0 - eps * dq, steps)[0]) / (2 * eps)
    monkeypatch.setattr(TG, "_abs", lambda z: np.abs(z) + 0j)
    J, dJ = TG.nusselt_tangent(*n, Ra, theta, q0, steps, dq=dq)
    J0 = c_oracle_nu(n, Ra, theta, q0, steps)[0]
    assert abs(J - J0) <= 1e-12 * abs(J0)
    assert abs(dJ - fd) > 1e-4 * abs(fd)
