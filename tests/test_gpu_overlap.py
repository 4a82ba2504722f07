"""GPU tests of the interior/exterior split step (cavity_step_overlap).

The split computes every cell with the same per-cell code as cavity_step, in
one of two launches, so the state must come out bit-identical to
cavity_step with the same halo; the norms are summed in another grouping and
agree to rounding (a cell computed twice or never would break one of the
two).  Checked on the parity grid, the paper's 256^3 share with its 1D, 2D
and 3D splits and both width sets, a ragged grid, FP32, and a hot-wall field,
on one stream and with the exchange on a second stream.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

CW, PW = (1, 2, 2, 2, 2), (2, 1, 1, 1, 1)


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
    G = g.ng
    return C.state_view(g, t)[:, G:G + g.nk, G:G + g.nj, G:G + g.ni].cpu().numpy()


def pair(C, g, prm, halo, seed):
    a = C.Cavity(g, prm, halo).init(seed)
    b = C.Cavity(g, prm, halo)
    b.q.copy_(a.q)
    return a, b


@pytest.mark.parametrize("n,split,width,dtype,steps", [
    ((16, 16, 16), (2, 2, 2), CW, 0, 9),
    ((256, 256, 256), (2, 2, 2), CW, 0, 4),
    ((256, 256, 256), (8, 1, 1), CW, 0, 3),
    ((256, 256, 256), (4, 2, 1), PW, 0, 3),
    ((64, 36, 24), (4, 3, 2), PW, 0, 5),
    ((96, 64, 32), (2, 4, 2), CW, 1, 6),
])
@pytest.mark.parametrize("two_streams", [False, True])
def test_split_step_is_bit_identical(C, n, split, width, dtype, steps, two_streams):
    import torch
    say("overlap", n, split, width, dtype, steps, two_streams)
    g = C.Grid(*n, dtype=dtype)
    halo = C.Halo(split, width)
    a, b = pair(C, g, C.Params(Ra=1e5), halo, 3)
    a.step(steps)
    b.q_tmp.fill_(float("nan"))
    comm = torch.cuda.Stream() if two_streams else None
    b.step_overlap(steps, comm_stream=comm)
    assert np.array_equal(interior(C, g, a.q), interior(C, g, b.q))
    np.testing.assert_allclose(b.norms(), a.norms(), rtol=1e-12 if dtype == 0 else 1e-6)


def test_split_with_wall_field_matches_oracle(C):
    import torch
    say("overlap wall field")
    n = (32, 24, 16)
    theta = 1.0 + 0.05 * np.random.default_rng(3).uniform(-1, 1, n[1] * n[2])
    P = O.Problem(*n, Ra=1e5, t_hot_field=theta)
    q0 = O.init(P, 5, 1e-3)
    split, width = (2, 2, 2), CW
    ref = q0.copy()
    O.step(P, ref, 12, halo=(split, width))
    g = C.Grid(*n)
    cav = C.Cavity(g, C.Params(Ra=1e5, t_hot_field=torch.from_numpy(theta).cuda()), C.Halo(split, width))
    C.state_view(g, cav.q).copy_(torch.from_numpy(q0))
    cav.step_overlap(12, comm_stream=torch.cuda.Stream())
    got = interior(C, g, cav.q)
    want = P.interior(ref)
    for f in range(5):
        assert np.abs(got[f] - want[f]).max() <= 1e-12 * np.abs(want[f]).max(), f


def test_split_rejects_thin_subdomains_and_missing_halo(C):
    say("overlap validation")
    g = C.Grid(16, 16, 16)
    cav = C.Cavity(g, C.Params(), C.Halo((4, 1, 1), CW))      # extent 4 < 2 * 3
    with pytest.raises(C.CavError) as e:
        cav.step_overlap(1)
    assert e.value.code == C.CAV_EINVAL
    cav = C.Cavity(g, C.Params(), None)
    with pytest.raises(C.CavError) as e:
        C.cavity_step_overlap(g, C.Params(), None, cav.q, cav.q_tmp, cav.ws, None, 1)
    assert e.value.code == C.CAV_EINVAL
