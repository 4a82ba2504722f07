"""GPU tests of the batched form: many cavities advanced by one persistent
launch per step, optionally replayed from a HIP graph.

Every member must come out bit-identical to advancing it alone with
cavity_step (the batched kernel runs the same per-tile code), whatever the
k-chunk length of its work items; graph replays must equal eager steps.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

# the FP32 form's stated per-field tolerance against the FP64 oracle after 100 steps
TOL_F32 = 1e-5

MEMBERS = [((16, 16, 16), 1e3), ((67, 37, 21), 1e5), ((24, 24, 24), 3e4), ((40, 9, 13), 1e6),
           ((96, 96, 96), 2e5), ((5, 70, 11), 1e4)]


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


def interior(C, g, t):
    import torch
    torch.cuda.synchronize()
    v = C.state_view(g, t)
    return v[:, 2:-2, 2:-2, 2:-2].cpu().numpy()


def build(C, dtype, kc=0):
    return C.Batch([(C.Grid(*n, dtype=dtype), C.Params(Ra=Ra), kc) for n, Ra in MEMBERS])


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("nsteps", [6, 7])
def test_batch_matches_single_cavities(C, dtype, nsteps):
    say("batch vs single", dtype, nsteps)
    b = build(C, dtype).init(range(100, 100 + len(MEMBERS)))
    b.step(nsteps)
    for m, (n, Ra) in enumerate(MEMBERS):
        g = C.Grid(*n, dtype=dtype)
        cav = C.Cavity(g, C.Params(Ra=Ra)).init(100 + m)
        cav.step(nsteps)
        assert np.array_equal(interior(C, g, b.state(m)), interior(C, g, cav.q)), (m, n)
        # the norms' partial sums are grouped by work item, so they agree to rounding
        np.testing.assert_allclose(b.norms(m), cav.norms(), rtol=1e-12)


def test_batch_result_is_independent_of_k_chunks(C):
    """Per-cell arithmetic does not depend on how the k columns are cut into
    work items: states bit-identical, norms (summed in another grouping)
    equal to rounding."""
    say("batch kc invariance")
    a = build(C, 0).init(range(len(MEMBERS)))
    b = build(C, 0, kc=3).init(range(len(MEMBERS)))
    a.step(5)
    b.step(5)
    for m, (n, _) in enumerate(MEMBERS):
        g = C.Grid(*n)
        assert np.array_equal(interior(C, g, a.state(m)), interior(C, g, b.state(m)))
        np.testing.assert_allclose(b.norms(m), a.norms(m), rtol=1e-13)


@pytest.mark.parametrize("dtype", [0, 1])
def test_batch_result_is_independent_of_tile_shape(C, dtype):
    """The narrow tile (FP64 32 x 16, FP32 16 x 16) gives the same states as
    the wide one (FP64 64 x 8, FP32 32 x 8), and so does a batch mixing
    both, bit for bit; norms to rounding."""
    wide, narrow = C.BATCH_TILE_WIDTHS[dtype]
    say("batch tile shape", dtype, wide, narrow)
    a = C.Batch([(C.Grid(*n, dtype=dtype), C.Params(Ra=Ra), 0, wide) for n, Ra in MEMBERS]).init(range(len(MEMBERS)))
    b = C.Batch([(C.Grid(*n, dtype=dtype), C.Params(Ra=Ra), kc, narrow)
                 for (n, Ra), kc in zip(MEMBERS, (0, 5, 8, 3, 16, 0))])
    b.init(range(len(MEMBERS)))
    # both shapes in one batch (the kernel compiled for both; a batch of one
    # shape runs the kernel compiled for that shape alone)
    c = C.Batch([(C.Grid(*n, dtype=dtype), C.Params(Ra=Ra), 0, (wide, narrow)[m % 2])
                 for m, (n, Ra) in enumerate(MEMBERS)])
    c.init(range(len(MEMBERS)))
    assert (a.handle.shapes, b.handle.shapes, c.handle.shapes) == (1, 2, 3)
    a.step(5)
    b.step(5)
    c.step(5)
    for m, (n, _) in enumerate(MEMBERS):
        g = C.Grid(*n, dtype=dtype)
        assert np.array_equal(interior(C, g, a.state(m)), interior(C, g, b.state(m))), m
        assert np.array_equal(interior(C, g, a.state(m)), interior(C, g, c.state(m))), m
        np.testing.assert_allclose(b.norms(m), a.norms(m), rtol=1e-12 if dtype == 0 else 1e-5)
        np.testing.assert_allclose(c.norms(m), a.norms(m), rtol=1e-12 if dtype == 0 else 1e-5)


@pytest.mark.parametrize("dtype", [0, 1])
def test_graph_replays_equal_eager_steps(C, dtype):
    import torch
    say("batch graph", dtype)
    s = torch.cuda.Stream()
    eager = build(C, dtype).init(range(7, 7 + len(MEMBERS)))
    graphed = build(C, dtype).init(range(7, 7 + len(MEMBERS)))
    eager.step(6)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        gr = graphed.graph(2, stream=s)
        for r in range(3):
            gr.launch(stream=s)
            s.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()      # eager work between replays
        gr.destroy()
    torch.cuda.synchronize()
    for m, (n, _) in enumerate(MEMBERS):
        g = C.Grid(*n, dtype=dtype)
        assert np.array_equal(interior(C, g, eager.state(m)), interior(C, g, graphed.state(m))), m
        assert eager.norms(m) == graphed.norms(m)


def test_batch_member_against_oracle(C):
    """One member of a mixed batch against the FP64 oracle (1e-12)."""
    say("batch vs oracle")
    b = C.Batch([(C.Grid(*n), C.Params(Ra=Ra)) for n, Ra in MEMBERS[:4]])
    P = O.Problem(*MEMBERS[1][0], Ra=MEMBERS[1][1])
    q0 = O.init(P, 42, 1e-3)
    b.init(range(4))
    import torch
    C.state_view(b.grids[1], b.q[1]).copy_(torch.from_numpy(q0))
    b.step(10)
    ref = q0.copy()
    O.step(P, ref, 10)
    got = interior(C, b.grids[1], b.state(1))
    want = P.interior(ref)
    err = max(float(np.abs(got[f] - want[f]).max() / np.abs(want[f]).max()) for f in range(5))
    say("  rel err", err)
    assert err <= 1e-12


def test_autotuner_returns_valid_choices(C):
    from paper_2006_02602_amd import autotune
    say("autotune")
    shapes = autotune.tune_shapes([24, 32], dtype=1, steps=2, reps=1, probe_members=2)
    assert set(shapes) == {24, 32}
    for e, (ti, kc) in shapes.items():
        assert ti in autotune.ti_candidates(1) and kc in autotune.KC_CANDIDATES and kc <= e
    b = C.Batch([(C.Grid.cube(e, 1), C.Params(), shapes[e][1], shapes[e][0]) for e in (24, 32, 32)]).init([1, 2, 3])
    nb, t = autotune.tune_blocks(b, steps=2, reps=1)
    assert nb in autotune.BLOCK_CANDIDATES and len(t) == len(autotune.BLOCK_CANDIDATES)


def test_batch_member_with_hot_wall_field(C):
    """A member whose hot wall is a per-row field advances bit-identically to
    the same cavity alone (the work items carry the member's field)."""
    import torch
    say("batch wall field")
    n = (40, 24, 18)
    theta = torch.from_numpy(1.0 + 0.05 * np.random.default_rng(8).uniform(-1, 1, n[1] * n[2])).cuda()
    prm = C.Params(Ra=1e5, t_hot_field=theta)
    b = C.Batch([(C.Grid(*n), prm), (C.Grid(16, 16, 16), C.Params(Ra=1e3))]).init([5, 6])
    b.step(7)
    cav = C.Cavity(C.Grid(*n), prm).init(5)
    cav.step(7)
    g = C.Grid(*n)
    assert np.array_equal(interior(C, g, b.state(0)), interior(C, g, cav.q))
    uniform = C.Cavity(C.Grid(*n), C.Params(Ra=1e5)).init(5)
    uniform.step(7)
    assert not np.array_equal(interior(C, g, uniform.q), interior(C, g, cav.q))


def test_batch96_workload_matches_single_runs(C):
    """The timed batched workload (96 FP32 cavities, edges 24..96, Ra 1e3..1e6)
    with the tile shapes, k chunks and block count tuned on the whole batch,
    100 steps replayed from one HIP graph: sampled members (every edge, the
    lowest and highest Ra) come out bit-identical to advancing each alone
    with cavity_step, and within 1e-5 per field of the FP64 oracle run from
    the same (FP32-rounded) start."""
    import torch
    from paper_2006_02602_amd import autotune
    from paper_2006_02602_amd.configs import batch_workload
    say("batch96 workload x100 (graph)")
    wl = batch_workload()
    b = C.Batch([(C.Grid.cube(e, C.CAV_F32), C.Params(Ra=ra)) for e, ra, _ in wl])
    b.init([s for _, _, s in wl])
    shapes, nb, _ = autotune.tune_batch(b, [e for e, _, _ in wl], C.CAV_F32, cache_path="/tmp/cavity_autotune.json")
    for e, (ti, kc) in shapes.items():
        assert ti in autotune.ti_candidates(C.CAV_F32) and kc in autotune.KC_CANDIDATES and kc < e
    assert nb in autotune.BLOCK_CANDIDATES
    b.init([s for _, _, s in wl])
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        gr = b.graph(100, nblocks=nb, stream=st)
        gr.launch(stream=st)
        st.synchronize()
        gr.destroy()
    pick = {}
    for m, (e, ra, _) in enumerate(wl):
        pick.setdefault(e, m)
    pick["lo"] = min(range(len(wl)), key=lambda m: wl[m][1])
    pick["hi"] = max(range(len(wl)), key=lambda m: wl[m][1])
    for m in sorted(set(pick.values())):
        e, ra, s = wl[m]
        g = C.Grid.cube(e, C.CAV_F32)
        cav = C.Cavity(g, C.Params(Ra=ra)).init(s)
        cav.step(100)
        say("  member", m, "edge", e, "Ra %.3g" % ra, "tile", C.batch_tile(C.CAV_F32, shapes[e][0]), "kc", shapes[e][1])
        got = interior(C, g, b.state(m))
        assert np.array_equal(got, interior(C, g, cav.q)), (m, e, ra)
        assert all(np.isfinite(b.norms(m)))
        # and against the FP64 oracle from the same (FP32-rounded) start
        P = O.Problem(e, Ra=ra)
        ref = O.init(P, s, 1e-3).astype(np.float32).astype(np.float64)
        O.step(P, ref, 100)
        want = P.interior(ref)
        err = [float(np.abs(got[f].astype(np.float64) - want[f]).max() / np.abs(want[f]).max()) for f in range(5)]
        say("    rel err vs FP64 oracle (p u v w T):", ["%.2e" % x for x in err])
        assert max(err) <= TOL_F32, (m, e, ra, err)


def test_graph_refuses_replay_after_odd_eager_step(C):
    """A graph replays the parity it was captured at: after an odd number of
    eager steps the launch is refused (nothing enqueued); one more eager step
    restores the parity and the replay is valid again."""
    import torch
    say("batch graph parity")
    a = build(C, 1).init(range(30, 30 + len(MEMBERS)))
    b = build(C, 1).init(range(30, 30 + len(MEMBERS)))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        gr = b.graph(2, stream=st)
        b.step(1, stream=st)
        with pytest.raises(C.CavError) as e:
            gr.launch(stream=st)
        assert e.value.code == C.CAV_EINVAL
        b.step(1, stream=st)
        gr.launch(stream=st)
        st.synchronize()
        gr.destroy()
    a.step(4)
    for m, (n, _) in enumerate(MEMBERS):
        g = C.Grid(*n, dtype=1)
        assert np.array_equal(interior(C, g, a.state(m)), interior(C, g, b.state(m))), m


@pytest.mark.parametrize("dtype", [0, 1])
def test_retile_keeps_states_and_parity(C, dtype):
    """Rebuilding the work list between steps (other tile widths and k
    chunks) changes nothing: 3 + 4 steps equal 7 steps, bit for bit."""
    say("batch retile", dtype)
    wide, narrow = C.BATCH_TILE_WIDTHS[dtype]
    a = build(C, dtype).init(range(20, 20 + len(MEMBERS)))
    b = build(C, dtype).init(range(20, 20 + len(MEMBERS)))
    a.step(7)
    b.step(3)
    b.retile([(kc, narrow if m % 2 else wide) for m, kc in enumerate((4, 0, 8, 3, 16, 5))])
    b.step(4)
    assert b.handle.parity == a.handle.parity
    # a live graph of the old work list blocks a rebuild of its table
    import torch
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        gr = b.graph(2, stream=st)
    st.synchronize()
    with pytest.raises(C.CavError):
        b.retile([(0, 0)] * len(MEMBERS))
    gr.destroy()
    b.retile([(0, 0)] * len(MEMBERS))
    for m, (n, _) in enumerate(MEMBERS):
        g = C.Grid(*n, dtype=dtype)
        assert np.array_equal(interior(C, g, a.state(m)), interior(C, g, b.state(m))), m
