"""GPU test of cavity_step_noalloc, the step for callers that cannot
allocate: its norm partials live in the library's static device array
instead of a caller workspace.  It runs the same kernels as cavity_step, so
its state and norms must equal cavity_step's bit for bit; two calls in a
row (the second on a smaller grid) check that the shared array's leftover
contents from one call never reach the next.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def run_both(C, n, dtype, halo, steps, seed, Ra):
    """The same seeded start advanced by cavity_step (workspace) and by
    cavity_step_noalloc (static scratch); returns both states and norms."""
    import torch
    g = C.Grid(*n, dtype=dtype)
    prm = C.Params(Ra=Ra)
    h = C.Halo(*halo) if halo else None
    ref = C.Cavity(g, prm, h).init(seed, 1e-3)
    q = ref.q.clone()
    q_tmp = torch.full_like(ref.q_tmp, float("nan"))
    buf = None
    if h is not None:
        buf = torch.full_like(ref.buf, float("nan"))
    norms = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    ref.step(steps)
    C.cavity_step_noalloc(g, prm, h, q, q_tmp, buf, norms, steps)
    torch.cuda.synchronize()
    want_q = C.state_view(g, ref.q)[:, 2:-2, 2:-2, 2:-2].cpu().numpy()
    got_q = C.state_view(g, q)[:, 2:-2, 2:-2, 2:-2].cpu().numpy()
    return want_q, got_q, np.array(ref.norms()), norms.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    (((64, 48, 40), 0, ((2, 2, 1), (1, 2, 2, 2, 2)), 7, 2, 1e5),      # odd steps: the copy-back path
     ((24, 20, 16), 0, None, 4, 3, 1e3)),
    (((96, 64, 32), 1, ((4, 2, 1), (2, 1, 1, 1, 1)), 6, 4, 1e6),
     ((33, 17, 9), 1, None, 5, 5, 1e4)),
])
def test_noalloc_equals_cavity_step(C, first, second):
    for i, (n, dtype, halo, steps, seed, Ra) in enumerate((first, second)):
        say("noalloc call %d: %s dtype %d halo %s, %d steps" % (i + 1, n, dtype, halo, steps))
        want_q, got_q, want_n, got_n = run_both(C, n, dtype, halo, steps, seed, Ra)
        assert np.array_equal(got_q, want_q), "state differs from cavity_step's"
        assert np.array_equal(got_n, want_n), (got_n, want_n)


def test_noalloc_without_norms(C):
    """norms = NULL skips the norm pass; the state is still cavity_step's."""
    import torch
    n = (40, 24, 18)
    g, prm = C.Grid(*n), C.Params(Ra=1e5)
    ref = C.Cavity(g, prm).init(6, 1e-3)
    q = ref.q.clone()
    q_tmp = torch.zeros_like(ref.q_tmp)
    ref.step(3)
    C.cavity_step_noalloc(g, prm, None, q, q_tmp, None, None, 3)
    torch.cuda.synchronize()
    assert np.array_equal(C.state_view(g, q)[:, 2:-2, 2:-2, 2:-2].cpu().numpy(),
                          C.state_view(g, ref.q)[:, 2:-2, 2:-2, 2:-2].cpu().numpy())
