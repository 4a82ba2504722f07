"""GPU tests of the FP32 precision form and of the FP64 Nusselt integral.

The FP32 form keeps the state and the stencil arithmetic in FP32 and
accumulates the residual norms and the hot-wall Nusselt number in FP64.  Its
initial state is the FP64 seeded state rounded to FP32, and its halo
pack/unpack are copies, so those match the oracle bit for bit.  After 100
steps its fields are compared with the FP64 oracle per field (max |a-b| /
max |b| over the interior); the bound is stated below with the errors it was
set from.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

# Measured per-field relative errors after 100 steps sit well below this
# bound (see test output); 1e-5 is the stated tolerance of the FP32 form.
TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def C():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2006_02602_amd as C
    C.lib()
    return C


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def get_state(C, g, t):
    import torch
    torch.cuda.synchronize()
    return C.state_view(g, t).cpu().numpy().astype(np.float64)


def put_state(C, g, t, a):
    import torch
    C.state_view(g, t).copy_(torch.from_numpy(np.ascontiguousarray(a)).to(t.dtype))


def rel_err(a, b):
    return [float(np.abs(a[f] - b[f]).max() / max(np.abs(b[f]).max(), 1e-300)) for f in range(5)]


def norm_tolerance(P, q, nref):
    """Per-field bound on |FP32 norm - FP64 oracle norm|: 1e-3 relative,
    but never below the FP32 noise floor of the residual.

    Each FP32 state value carries a rounding of up to u = 2^-24 of its
    magnitude, and the residual R_f amplifies a perturbation of the state
    by at most the sum of its stencil coefficients' magnitudes (Eq. 1-3
    with the readings of the dissipation and of beta):
      T:      |V|*S1 + 4*alpha*S2                 on max|T|
      u,v,w:  |V|*S1 + 4*nu*S2                    on max|u,v,w|,
              plus 1/h_min on max|p| and 1 on max|T| (buoyancy)
      p:      beta2*S1 on max|u,v,w| + 16*eps*lambda*S1 on max|p|
    with S1 = sum 1/h_i, S2 = sum 1/h_i^2, beta2 <= max(3|V|^2, kappa*U^2)
    and lambda <= (|V| + sqrt(|V|^2 + 4*beta2))/2.  An RMS norm moves by at
    most the largest per-cell change, so a residual whose RMS is below
    u times that sum is FP32 noise: at 384^3, Ra 1e6 the T residual (RMS
    ~2e-4) sits there, since 4*alpha*S2 ~ 2.1e3."""
    u32 = 2.0 ** -24
    I = P.interior(q)
    h = (1.0 / P.ni, 1.0 / P.nj, 1.0 / P.nk)
    S1, S2 = sum(1.0 / x for x in h), sum(1.0 / (x * x) for x in h)
    mp, mv, mT = float(np.abs(I[0]).max()), float(np.abs(I[1:4]).max()), float(np.abs(I[4]).max())
    nu, alpha = (P.Pr / P.Ra) ** 0.5, 1.0 / (P.Ra * P.Pr) ** 0.5
    beta2 = max(3.0 * mv * mv, P.kappa * P.u_ref ** 2)
    lam = 0.5 * (mv + (mv * mv + 4.0 * beta2) ** 0.5)
    floor_p = u32 * (beta2 * S1 * mv + 16.0 * P.eps4 * lam * S1 * mp)
    floor_v = u32 * ((mv * S1 + 4.0 * nu * S2) * mv + mp / min(h) + mT)
    floor_T = u32 * (mv * S1 + 4.0 * alpha * S2) * mT
    floors = np.array([floor_p, floor_v, floor_v, floor_v, floor_T])
    return np.maximum(1e-3 * np.abs(np.asarray(nref)), floors)


def problem(C, n, Ra, dtype):
    P = O.Problem(*n, Ra=Ra)
    g = C.Grid(*n, dtype=dtype)
    prm = C.Params(Ra=Ra)
    return P, g, prm


@pytest.mark.parametrize("n", [(16, 16, 16), (67, 37, 21)])
def test_f32_init_is_rounded_f64_init(C, n):
    say("f32 init", n)
    P, g, prm = problem(C, n, 1e6, C.CAV_F32)
    ref = O.init(P, 3, 1e-3)
    cav = C.Cavity(g, prm).init(3, 1e-3)
    got = get_state(C, g, cav.q)
    assert np.array_equal(P.interior(got), P.interior(ref).astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("n,split,width", [((16, 16, 16), (2, 2, 2), (1, 2, 2, 2, 2)),
                                           ((256, 256, 256), (8, 1, 1), (1, 2, 2, 2, 2)),
                                           ((96, 64, 32), (4, 2, 1), (2, 1, 1, 1, 1))])
def test_f32_pack_unpack_bit_exact(C, n, split, width):
    import torch
    say("f32 pack", n, split, width)
    P = O.Problem(*n)
    g, h = C.Grid(*n, dtype=C.CAV_F32), C.Halo(split, width)
    q = np.random.default_rng(7).standard_normal(P.shape).astype(np.float32).astype(np.float64)
    ref = O.halo_pack(P, (split, width), q)
    assert C.halo_buffer_bytes(g, h) == 4 * ref.size
    qd = torch.zeros(C.cavity_state_elems(g), dtype=torch.float32, device="cuda")
    put_state(C, g, qd, q)
    buf = torch.full((ref.size,), float("nan"), dtype=torch.float32, device="cuda")
    C.halo_pack(g, h, qd, buf)
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy().astype(np.float64), ref)
    mark = np.zeros(P.shape)
    O.halo_unpack(P, (split, width), np.ones(ref.size), mark)
    qp = q.copy()
    qp[mark == 1] = np.nan
    put_state(C, g, qd, qp)
    C.halo_unpack(g, h, buf, qd)
    assert np.array_equal(get_state(C, g, qd), q)


@pytest.mark.parametrize("n,Ra,halo", [((32, 32, 32), 1e6, None),
                                       ((16, 16, 16), 1e3, ((2, 2, 2), (1, 2, 2, 2, 2))),
                                       ((67, 37, 21), 1e5, None)])
def test_f32_against_f64_oracle(C, n, Ra, halo):
    """100 steps of the FP32 form against the FP64 oracle from the same
    (rounded) start."""
    say("f32 vs oracle", n, Ra, halo)
    P, g, prm = problem(C, n, Ra, C.CAV_F32)
    q0 = O.init(P, 3, 1e-3)
    q0r = q0.astype(np.float32).astype(np.float64)
    ref = q0r.copy()
    nref = O.step(P, ref, 100, halo=halo)
    cav = C.Cavity(g, prm, C.Halo(*halo) if halo else None)
    put_state(C, g, cav.q, q0r)
    cav.step(100)
    got = get_state(C, g, cav.q)
    e = rel_err(P.interior(got), P.interior(ref))
    say("  per-field rel err (p u v w T):", ["%.2e" % x for x in e])
    na = np.array(cav.norms())
    tol = norm_tolerance(P, ref, nref)
    say("  norms |diff| / bound:", ["%.2e" % x for x in np.abs(na - nref) / tol])
    assert max(e) <= TOL_F32, e
    assert np.all(np.abs(na - nref) <= tol), (na, nref, tol)


def test_f32_against_f64_gpu_128(C):
    """128^3, Ra 1e6, 100 steps: the FP32 form against the FP64 form of the
    same library from the same start."""
    say("f32 vs f64 gpu 128^3")
    n = (128, 128, 128)
    P = O.Problem(*n, Ra=1e6)
    g32, g64 = C.Grid(*n, dtype=C.CAV_F32), C.Grid(*n)
    prm = C.Params(Ra=1e6)
    a = C.Cavity(g64, prm).init(3, 1e-3)
    b = C.Cavity(g32, prm)
    put_state(C, g32, b.q, get_state(C, g64, a.q))
    a.step(100)
    b.step(100)
    e = rel_err(P.interior(get_state(C, g32, b.q)), P.interior(get_state(C, g64, a.q)))
    say("  per-field rel err (p u v w T):", ["%.2e" % x for x in e])
    assert max(e) <= TOL_F32, e


@pytest.mark.parametrize("dtype", [0, 1])
def test_nusselt_against_oracle(C, dtype):
    say("nusselt", dtype)
    n = (40, 24, 18)
    P, g, prm = problem(C, n, 1e5, dtype)
    q0 = O.init(P, 9, 1e-3)
    if dtype == C.CAV_F32:
        q0 = q0.astype(np.float32).astype(np.float64)
    ref = q0.copy()
    O.step(P, ref, 30)
    cav = C.Cavity(g, prm)
    put_state(C, g, cav.q, q0)
    cav.step(30)
    nu_gpu = cav.nusselt()
    nu_ref = O.nusselt_hot(P, ref)
    say("  Nu gpu %.15f oracle %.15f" % (nu_gpu, nu_ref))
    assert abs(nu_gpu - nu_ref) <= (1e-12 if dtype == 0 else 1e-5) * abs(nu_ref)
    # conduction profile: Nu = 1 exactly up to rounding of the state
    x = (np.arange(n[0]) + 0.5) / n[0]
    cond = P.zeros()
    P.interior(cond)[4][:] = 1.0 - x
    put_state(C, g, cav.q, cond)
    assert abs(cav.nusselt() - 1.0) < (1e-13 if dtype == 0 else 1e-5)


def test_f32_full_size_against_oracle(C):
    """The timed FP32 workload in full (384^3, Ra 1e6, 100 steps, its grid
    and launch: 32 x 8 tiles, k chunks from the occupancy query) against the
    FP64 oracle from the same (rounded) start, per field."""
    say("f32 vs oracle 384^3 x100")
    n = (384, 384, 384)
    P, g, prm = problem(C, n, 1e6, C.CAV_F32)
    q0 = O.init(P, 3, 1e-3).astype(np.float32).astype(np.float64)
    cav = C.Cavity(g, prm)
    put_state(C, g, cav.q, q0)
    cav.step(100)
    ref = q0
    del q0
    nref = O.step(P, ref, 100)
    say("  oracle done")
    e = rel_err(P.interior(get_state(C, g, cav.q)), P.interior(ref))
    say("  per-field rel err (p u v w T):", ["%.2e" % x for x in e])
    na = np.array(cav.norms())
    tol = norm_tolerance(P, ref, nref)
    say("  norms |diff| / bound:", ["%.2e" % x for x in np.abs(na - nref) / tol])
    assert max(e) <= TOL_F32, e
    assert np.all(np.abs(na - nref) <= tol), (na, nref, tol)


def test_f32_mirror_symmetry_full_size(C):
    """384^3 FP32, Ra 1e6, the timed 100 steps: a start mirror-symmetric in
    y (v odd, the rest even) stays symmetric bit for bit; the stencil pairs
    its operands commutatively, so this holds in FP32 as in FP64."""
    say("f32 mirror 384^3 x100")
    n = (384, 384, 384)
    P, g, prm = problem(C, n, 1e6, C.CAV_F32)
    q = O.init(P, 2, 1e-3)
    I = P.interior(q)
    half = P.nj // 2
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        I[f][:, P.nj - half:, :] = s * I[f][:, :half, :][:, ::-1, :]
    O.apply_bc(P, q)
    cav = C.Cavity(g, prm)
    put_state(C, g, cav.q, q.astype(np.float32).astype(np.float64))
    del q, I
    cav.step(100)
    J = P.interior(get_state(C, g, cav.q))
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        assert np.array_equal(J[f], s * J[f][:, ::-1, :]), O.FIELDS[f]
