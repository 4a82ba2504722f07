"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Pack/unpack and init must match bit for bit; the FP64 sweep must match the
oracle within 1e-12 relative per field (max |gpu - oracle| / max |oracle|
over the interior) after the configured number of steps, including the
full 256^3 x 200-step timed workload; properties that hold at any length
(exact mirror symmetry, determinism) are checked as well.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12
NG = 2


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


def dev(a):
    """Flat device copy of a buffer."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).cuda()


def host(t, shape):
    """Host copy of a flat device buffer."""
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


def put_state(C, g, t, a):
    """Write a (5, nk+4, nj+4, ni+4) array into state tensor t (library layout)."""
    import torch
    C.state_view(g, t).copy_(torch.from_numpy(np.ascontiguousarray(a)))


def new_state(C, g, a):
    import torch
    t = torch.zeros(C.cavity_state_elems(g), dtype=torch.float64, device="cuda")
    put_state(C, g, t, a)
    return t


def get_state(C, g, t):
    import torch
    torch.cuda.synchronize()
    return C.state_view(g, t).cpu().numpy()


def face_ghost_mask(shape):
    """Interior plus the face ghost layers (no edge or corner ghosts)."""
    _, K, J, I = shape
    m = np.zeros((K, J, I), dtype=bool)
    m[NG:K - NG, NG:J - NG, :] = True
    m[NG:K - NG, :, NG:I - NG] = True
    m[:, NG:J - NG, NG:I - NG] = True
    return m


def rel_err(a, b):
    return [float(np.abs(a[f] - b[f]).max() / max(np.abs(b[f]).max(), 1e-300)) for f in range(5)]


def problem(C, n, Ra=1e3, **kw):
    P = O.Problem(*n, Ra=Ra, **kw)
    g = C.Grid(*n)
    prm = C.Params(Ra=Ra, Pr=P.Pr, cfl=P.cfl, eps4=P.eps4, kappa=P.kappa, u_ref=P.u_ref,
                   t_hot=P.t_hot, t_cold=P.t_cold, t_inf=P.t_inf)
    return P, g, prm


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [(16, 16, 16), (67, 37, 21), (2, 3, 2)])
def test_init_bit_exact(C, n):
    say("init", n)
    P, g, prm = problem(C, n)
    ref = O.init(P, 11, 1e-3)
    cav = C.Cavity(g, prm).init(11, 1e-3)
    got = get_state(C, g, cav.q)
    m = face_ghost_mask(P.shape)
    for f in range(5):
        assert np.array_equal(got[f][m], ref[f][m]), O.FIELDS[f]


# ---------------------------------------------------------------------------
PACK_CASES = [((16, 16, 16), (2, 2, 2), (1, 2, 2, 2, 2)),
              ((16, 16, 16), (2, 2, 2), (2, 1, 1, 1, 1)),
              ((30, 12, 21), (5, 3, 7), (2, 0, 1, 2, 1)),
              ((64, 48, 40), (8, 1, 1), (1, 2, 2, 2, 2)),
              ((256, 256, 256), (2, 2, 2), (1, 2, 2, 2, 2)),
              ((256, 256, 256), (8, 1, 1), (1, 2, 2, 2, 2)),
              ((256, 256, 256), (4, 2, 1), (1, 2, 2, 2, 2)),
              ((256, 256, 256), (8, 1, 1), (2, 1, 1, 1, 1)),
              ((256, 256, 256), (4, 2, 1), (2, 1, 1, 1, 1)),
              ((256, 256, 256), (2, 2, 2), (2, 1, 1, 1, 1))]


@pytest.mark.parametrize("n,split,width", PACK_CASES)
def test_pack_unpack_bit_exact(C, n, split, width):
    import torch
    say("pack/unpack", n, split, width)
    P = O.Problem(*n)
    g, h = C.Grid(*n), C.Halo(split, width)
    q = np.random.default_rng(hash((n, split, width)) % 2**32).standard_normal(P.shape)
    ref = O.halo_pack(P, (split, width), q)
    qd = new_state(C, g, q)
    nbytes = C.halo_buffer_bytes(g, h)
    assert nbytes == 8 * ref.size
    buf = torch.full((ref.size,), float("nan"), dtype=torch.float64, device="cuda")
    C.halo_pack(g, h, qd, buf)
    got = host(buf, ref.shape)
    assert np.array_equal(got, ref)
    # unpack into a copy whose segment cells are poisoned restores q exactly
    mark = np.zeros(P.shape)
    O.halo_unpack(P, (split, width), np.ones(ref.size), mark)
    qp = q.copy()
    qp[mark == 1] = np.nan
    qpd = new_state(C, g, qp)
    C.halo_unpack(g, h, buf, qpd)
    assert np.array_equal(get_state(C, g, qpd), q)
    # and the round trip leaves q bit-identical
    C.halo_unpack(g, h, buf, qd)
    assert np.array_equal(get_state(C, g, qd), q)


@pytest.mark.parametrize("n,split,width,dtype", [
    ((64, 48, 42), (2, 2, 2), (1, 2, 2, 2, 2), 0),    # the k cut at 21 falls inside a k chunk
    ((64, 48, 40), (4, 2, 1), (2, 1, 1, 1, 1), 0),
    ((128, 32, 24), (8, 1, 1), (1, 2, 2, 2, 2), 0),   # splits along i: the sweep packs every face
    ((64, 24, 20), (2, 1, 1), (2, 1, 1, 1, 1), 0),
    ((128, 16, 12), (8, 1, 1), (1, 2, 2, 2, 2), 1),
    ((96, 64, 32), (4, 2, 1), (1, 2, 2, 2, 2), 1),
    ((12, 10, 8), (4, 1, 1), (1, 2, 2, 2, 2), 0),     # i subdomains of 3 cells: no fused i-face pack
])
def test_step_exchange_is_the_pack_of_the_new_state(C, n, split, width, dtype):
    """Within cavity_step, for splits along i only, step m+1's exchange is
    packed by the sweep of step m as it writes the new state; other splits
    use the pack kernel.  After two steps the buffer holds step 2's
    exchange: it must equal halo_pack of the state after one step, and the
    oracle's pack of it, bit for bit."""
    import torch
    say("exchange buffer", n, split, width, dtype)
    P = O.Problem(*n, Ra=1e5)
    g, h, prm = C.Grid(*n, dtype=dtype), C.Halo(split, width), C.Params(Ra=1e5)
    a = C.Cavity(g, prm, h).init(7, 1e-3)
    q0 = a.q.clone()
    a.step(1)
    ref = torch.full_like(a.buf, float("nan"))
    C.halo_pack(g, h, a.q, ref)
    torch.cuda.synchronize()
    q1 = C.state_view(g, a.q).cpu().numpy().astype(np.float64)
    assert np.array_equal(ref.cpu().numpy().astype(np.float64), O.halo_pack(P, (split, width), q1))
    b = C.Cavity(g, prm, h)
    b.q.copy_(q0)
    b.buf.fill_(float("nan"))
    b.step(2)
    torch.cuda.synchronize()
    assert np.array_equal(b.buf.cpu().numpy(), ref.cpu().numpy())


def test_sqrt_and_reciprocal_within_an_ulp(C):
    """The residual's FP64 square root (reciprocal-square-root estimate
    refined by Goldschmidt's iteration and a residual correction) and
    reciprocal (estimate refined by two Newton steps) against the correctly
    rounded IEEE results, directly: log-uniform arguments over 1e-290 ..
    1e290, the range the residual feeds them (u^2 + 4 beta^2 >= 1, sums of
    lambda/h up to ~1e5), powers of two and their neighbours."""
    import torch
    rng = np.random.default_rng(12)
    x = np.concatenate([
        10.0 ** rng.uniform(-290, 290, 200000),
        rng.uniform(1.0, 16.0, 200000),
        10.0 ** rng.uniform(-1, 6, 200000),
        np.ldexp(1.0, np.arange(-960, 961)),
        np.nextafter(np.ldexp(1.0, np.arange(-960, 961)), 0.0),
        np.nextafter(np.ldexp(1.0, np.arange(-960, 961)), np.inf),
        [1.0, 2.0, 3.0, 4.0, 0.25, 1e-300 * 10, 1.7976931348623157e+290],
    ])
    xd = torch.from_numpy(x).cuda()
    out = torch.empty(2 * x.size, dtype=torch.float64, device="cuda")
    C.cavity_selftest_math(xd, out)
    got = out.cpu().numpy().reshape(-1, 2)

    def ulps(a, b):
        return np.abs(a.view(np.int64) - b.view(np.int64))

    ds = ulps(got[:, 0], np.sqrt(x))
    dr = ulps(got[:, 1], 1.0 / x)
    say("  sqrt: max %d ulp, exact %.4f; reciprocal: max %d ulp, exact %.4f"
        % (ds.max(), np.mean(ds == 0), dr.max(), np.mean(dr == 0)))
    assert ds.max() <= 1 and dr.max() <= 1


@pytest.mark.parametrize("n,dtype", [((67, 37, 21), 0), ((64, 64, 64), 0), ((96, 40, 33), 1)])
def test_step_from_equals_one_step(C, n, dtype):
    """cavity_step_from (one step out of place) gives cavity_step's state and
    norms bit for bit and leaves its input unchanged."""
    import torch
    say("step from", n, dtype)
    g, prm = C.Grid(*n, dtype=dtype), C.Params(Ra=1e5)
    a = C.Cavity(g, prm).init(11, 1e-3)
    q_in = a.q.clone()
    out = torch.full_like(a.q, float("nan"))
    ws = torch.zeros_like(a.ws)
    C.cavity_step_from(g, prm, q_in, out, ws)
    a.step(1)
    inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    assert torch.equal(C.state_view(g, out)[inner], C.state_view(g, a.q)[inner])
    assert C.cavity_residual_norm(g, ws) == a.norms()
    b = C.Cavity(g, prm).init(11, 1e-3)
    assert torch.equal(q_in, b.q)
    C.cavity_step_from(g, prm, q_in, out)          # no norm pass
    assert torch.equal(C.state_view(g, out)[inner], C.state_view(g, a.q)[inner])


@pytest.mark.parametrize("n,dtype", [((256, 256, 256), 0), ((67, 37, 21), 0), ((96, 40, 33), 1)])
def test_stream_copy_moves_the_interior(C, n, dtype):
    """The sweep-stream copy (measurement support) writes every interior
    cell of every field into q_tmp and nothing else."""
    import torch
    say("stream copy", n, dtype)
    g = C.Grid(*n, dtype=dtype)
    td = torch.float32 if dtype else torch.float64
    q = torch.randn(C.cavity_state_elems(g), dtype=torch.float64, device="cuda").to(td)
    t = torch.full_like(q, float("nan"))
    C.cavity_stream_copy(g, q, t)
    a, b = C.state_view(g, q), C.state_view(g, t)
    inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    assert torch.equal(b[inner], a[inner])
    ghost = torch.ones_like(b, dtype=torch.bool)
    ghost[inner] = False
    assert bool(torch.isnan(b[ghost]).all())


# ---------------------------------------------------------------------------
def run_both(C, n, Ra, steps, seed, halo=None, noise=1e-3, **kw):
    P, g, prm = problem(C, n, Ra=Ra, **kw)
    q0 = O.init(P, seed, noise)
    ref = q0.copy()
    nref = O.step(P, ref, steps, halo=halo)
    cav = C.Cavity(g, prm, C.Halo(*halo) if halo else None)
    put_state(C, g, cav.q, q0)
    cav.step(steps)
    got = get_state(C, g, cav.q)
    ngot = cav.norms()
    return P, P.interior(got), P.interior(ref), np.array(ngot), nref


def test_step_parity_small_config(C):
    """16^3, Ra 1e3, 100 steps, 2x2x2 virtual split with widths p 1, others 2."""
    say("step 16^3 x100")
    P, a, b, na, nb = run_both(C, (16, 16, 16), 1e3, 100, 1, halo=((2, 2, 2), (1, 2, 2, 2, 2)))
    e = rel_err(a, b)
    say("rel err per field", e, "norms", na, nb)
    assert max(e) <= TOL_F64, e
    np.testing.assert_allclose(na, nb, rtol=TOL_F64, atol=0)


@pytest.mark.parametrize("n,Ra,steps,halo", [
    ((67, 37, 21), 1e4, 20, None),               # ragged in every tile direction
    ((130, 9, 40), 1e5, 7, ((2, 3, 4), (2, 1, 1, 1, 1))),
    ((2, 2, 2), 1e3, 10, None),                  # smallest grid
    ((5, 64, 3), 1e6, 12, ((1, 4, 1), (1, 2, 2, 2, 2))),
])
def test_step_parity_ragged(C, n, Ra, steps, halo):
    say("step", n, Ra, steps, halo)
    P, a, b, na, nb = run_both(C, n, Ra, steps, 5, halo=halo)
    e = rel_err(a, b)
    say("rel err", e)
    assert max(e) <= TOL_F64, e
    np.testing.assert_allclose(na, nb, rtol=TOL_F64, atol=0)


def test_step_parity_full_size(C):
    """The timed workload in full: 256^3, Ra 1e5, 200 steps with the 3D
    split of the timed step, compared element by element."""
    say("step 256^3 x200")
    P, a, b, na, nb = run_both(C, (256, 256, 256), 1e5, 200, 2, halo=((2, 2, 2), (1, 2, 2, 2, 2)))
    e = rel_err(a, b)
    say("rel err", e, "norms", na, nb)
    assert max(e) <= TOL_F64, e
    np.testing.assert_allclose(na, nb, rtol=TOL_F64, atol=0)


def test_step_parity_full_size_odd(C):
    """256^3, 3 steps (odd count: the result is copied back into q)."""
    say("step 256^3 x3")
    P, a, b, na, nb = run_both(C, (256, 256, 256), 1e5, 3, 2, halo=((2, 2, 2), (1, 2, 2, 2, 2)))
    e = rel_err(a, b)
    assert max(e) <= TOL_F64, e
    np.testing.assert_allclose(na, nb, rtol=TOL_F64, atol=0)


@pytest.mark.parametrize("split,width", [((8, 1, 1), (1, 2, 2, 2, 2)), ((4, 2, 1), (2, 1, 1, 1, 1))])
def test_step_parity_full_size_other_splits(C, split, width):
    """256^3, 20 steps with the 1D and 2D splits of the timed halo rows
    (8x1x1: the sweep's epilogue packs every exchange after the first;
    4x2x1: the pack kernel), against the oracle with the same exchange."""
    say("step 256^3 x20", split, width)
    P, a, b, na, nb = run_both(C, (256, 256, 256), 1e5, 20, 2, halo=(split, width))
    e = rel_err(a, b)
    say("rel err", e)
    assert max(e) <= TOL_F64, e
    np.testing.assert_allclose(na, nb, rtol=TOL_F64, atol=0)


# ---------------------------------------------------------------------------
def test_quiescent_rest_exact(C):
    say("quiescent")
    n = (20, 12, 9)
    P, g, prm = problem(C, n, t_hot=0.5, t_cold=0.5, t_inf=0.5)
    cav = C.Cavity(g, prm, C.Halo((2, 1, 1), (2, 1, 1, 1, 1))).init(3, 0.0)
    cav.step(25)
    I = P.interior(get_state(C, g, cav.q))
    assert np.all(I[:4] == 0.0) and np.all(I[4] == 0.5)
    assert cav.norms() == [0.0] * 5


def y_symmetric_state(P, seed):
    q = O.init(P, seed, 1e-3)
    I = P.interior(q)
    half = P.nj // 2
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        I[f][:, P.nj - half:, :] = s * I[f][:, :half, :][:, ::-1, :]
    O.apply_bc(P, q)
    return q


def test_y_mirror_symmetry_full_size(C):
    """Full configuration (256^3, Ra 1e5, 200 steps, 3D split): a y-mirror-
    symmetric start stays symmetric bit for bit."""
    say("mirror 256^3 x200")
    P, g, prm = problem(C, (256, 256, 256), Ra=1e5)
    cav = C.Cavity(g, prm, C.Halo((2, 2, 2), (1, 2, 2, 2, 2)))
    put_state(C, g, cav.q, y_symmetric_state(P, 2))
    cav.step(200)
    I = P.interior(get_state(C, g, cav.q))
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        assert np.array_equal(I[f], s * I[f][:, ::-1, :]), O.FIELDS[f]
    assert all(math.isfinite(x) for x in cav.norms())


@pytest.mark.parametrize("n,dtype", [(1278, 0), (1274, 1)])
def test_largest_grid_mirror_symmetry(C, n, dtype):
    """The largest accepted cubes (one field just below 2^31 elements, so the
    kernels' 32-bit cell offsets reach their limit; an FP64 state is 85 GB):
    from a seeded start made y-mirror-symmetric on the device, 2 steps with
    the 2x2x2 exchange stay symmetric bit for bit and finite.  A wrong or
    overflowing offset anywhere in the sweep or the exchange breaks the
    symmetry where it strikes."""
    import torch
    say("largest grid", n, "dtype", dtype)
    g = C.Grid.cube(n, dtype)
    assert C.cavity_layout(g).sf > 2 ** 31 - 3 * (n + 4) ** 2 * 16
    cav = C.Cavity(g, C.Params(Ra=1e5), C.Halo((2, 2, 2), (1, 2, 2, 2, 2))).init(2)
    G, half = 2, n // 2
    V = C.state_view(g, cav.q)
    with torch.no_grad():
        for f in range(5):
            s = -1.0 if f == 2 else 1.0
            I = V[f, G:G + n, G:G + n, G:G + n]
            I[:, n - half:, :] = s * torch.flip(I[:, :half, :], dims=[1])
    torch.cuda.synchronize()
    say("  symmetric start set")
    cav.step(2)
    torch.cuda.synchronize()
    say("  stepped")
    V = C.state_view(g, cav.q)
    for f in range(5):
        s = -1.0 if f == 2 else 1.0
        I = V[f, G:G + n, G:G + n, G:G + n]
        assert bool(torch.isfinite(I).all()), f
        assert torch.equal(I, s * torch.flip(I, dims=[1])), f
    assert all(math.isfinite(x) for x in cav.norms())
    del cav, V, I
    torch.cuda.empty_cache()


def test_determinism_and_restart(C):
    say("determinism")
    P, g, prm = problem(C, (48, 40, 33), Ra=1e4)
    h = C.Halo((2, 2, 3), (1, 2, 2, 2, 2))
    a = C.Cavity(g, prm, h).init(9)
    b = C.Cavity(g, prm, h).init(9)
    a.step(40)
    b.step(17).step(23)
    assert np.array_equal(P.interior(get_state(C, g, a.q)), P.interior(get_state(C, g, b.q)))
    assert a.norms() == b.norms()
    c = C.Cavity(g, prm, h).init(9)
    c.step(40)
    assert np.array_equal(P.interior(get_state(C, g, a.q)), P.interior(get_state(C, g, c.q)))


def test_ghost_cells_never_read(C):
    """The wall ghosts are derived inside the sweep: NaN in every ghost
    cell of the state (and of the scratch state) changes nothing."""
    say("ghost poison")
    n = (70, 37, 19)
    P, g, prm = problem(C, n, Ra=1e4)
    h = C.Halo((2, 1, 1), (1, 2, 2, 2, 2))
    q0 = O.init(P, 8, 1e-3)
    poisoned = np.full(P.shape, np.nan)
    P.interior(poisoned)[:] = P.interior(q0)
    a, b = C.Cavity(g, prm, h), C.Cavity(g, prm, h)
    put_state(C, g, a.q, q0)
    b.q.fill_(float("nan"))
    put_state(C, g, b.q, poisoned)
    b.q_tmp.fill_(float("nan"))
    a.step(7)
    b.step(7)
    assert np.array_equal(P.interior(get_state(C, g, a.q)), P.interior(get_state(C, g, b.q)))
    assert a.norms() == b.norms()


def test_poisoned_scratch_is_overwritten(C):
    """Every interior cell of the new state is written by the sweep."""
    say("poison")
    P, g, prm = problem(C, (70, 20, 11), Ra=1e3)
    cav = C.Cavity(g, prm).init(4)
    cav.q_tmp.fill_(float("nan"))
    cav.step(1)
    I = P.interior(get_state(C, g, cav.q))
    assert np.all(np.isfinite(I))


def test_divergence_reports_nonfinite_norm(C):
    say("divergence")
    P, g, prm = problem(C, (8, 8, 8), Ra=1e3, cfl=50.0)
    cav = C.Cavity(g, prm).init(1)
    cav.step(80)
    with pytest.raises(C.CavError) as e:
        cav.norms()
    assert e.value.code == C.CAV_ENONFINITE
