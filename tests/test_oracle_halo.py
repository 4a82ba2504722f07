"""Pins of the oracle's halo pack/unpack (Sec. 4.5, Listings 1-2) on the CPU.

The buffer is checked against a brute-force gather written from the layout
definition with numpy slicing, against the i-face orders of Listing 1 (two
layers of every field) and Listing 2 (pressure with two layers first, then
the other fields with one layer) built from numpy boxes, and for the round
trip unpack(pack(q)) == q, also after poisoning every segment cell.
"""
import itertools

import numpy as np
import pytest

import oracle as O

NG = O.NG
FACES = ((0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1))   # (axis, high) for -x,+x,-y,+y,-z,+z


def brute_gather(P, halo, q):
    split, width = halo
    n = (P.ni, P.nj, P.nk)
    e = [n[d] // split[d] for d in range(3)]
    out = []
    for c in range(split[2]):
        for b in range(split[1]):
            for a in range(split[0]):
                coord = (a, b, c)
                for axis, high in FACES:
                    if (not high and coord[axis] == 0) or (high and coord[axis] == split[axis] - 1):
                        continue
                    for f in range(5):
                        w = width[f]
                        if w == 0:
                            continue
                        lo = [coord[d] * e[d] for d in range(3)]
                        hi = [(coord[d] + 1) * e[d] for d in range(3)]
                        if high:
                            lo[axis] = hi[axis] - w
                        else:
                            hi[axis] = lo[axis] + w
                        box = q[f, NG + lo[2]:NG + hi[2], NG + lo[1]:NG + hi[1], NG + lo[0]:NG + hi[0]]
                        out.append(box.reshape(-1))
    return np.concatenate(out) if out else np.zeros(0)


def splits_of(n):
    return [s for s in itertools.product(range(1, 9), repeat=3)
            if np.prod(s) <= 8 and all(n[d] % s[d] == 0 for d in range(3))]


WIDTHS = [(2, 2, 2, 2, 2), (2, 1, 1, 1, 1), (1, 2, 2, 2, 2), (0, 1, 0, 2, 1), (1, 1, 1, 1, 1)]


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 8, 4), (12, 6, 10)])
def test_pack_matches_brute_force(orc, n):
    P = O.Problem(*n)
    q = np.random.default_rng(0).standard_normal(P.shape)
    for split in splits_of(n):
        for width in WIDTHS:
            if any(n[d] // split[d] < max(width) for d in range(3)):
                continue
            halo = (split, width)
            buf = O.halo_pack(P, halo, q)
            ref = brute_gather(P, halo, q)
            assert buf.size == ref.size == O.halo_elems(P, halo)
            assert np.array_equal(buf, ref), (split, width)


def test_element_count_closed_form(orc):
    """Count = sum over cut interfaces of width * face area: each of the
    (Pi-1) i-cuts carries two directions of (nj*nk) * sum(width) values."""
    P = O.Problem(16, 12, 8)
    for split in ((8, 1, 1), (4, 2, 1), (2, 2, 2), (1, 3, 4), (16, 1, 1)):
        for width in WIDTHS:
            Pi, Pj, Pk = split
            W = sum(width)
            expect = W * 2 * ((Pi - 1) * P.nj * P.nk + (Pj - 1) * P.ni * P.nk + (Pk - 1) * P.ni * P.nj)
            if min(P.ni // Pi, P.nj // Pj, P.nk // Pk) < max(width):
                continue
            assert O.halo_elems(P, (split, width)) == expect


def test_i_face_order_all_fields_two_layers(orc):
    """Sec. 4.5, Listing 1 (read 0-based): on an i face every field sends
    its two interior layers next to the cut, field after field, each as a
    (k, j, i) box with i fastest.  Expected here: the numpy box of the
    high block's -x face flattened in C order, which is that order."""
    ni, nj, nk = 8, 5, 3
    P = O.Problem(ni, nj, nk)
    q = np.random.default_rng(1).standard_normal(P.shape)
    buf = O.halo_pack(P, ((2, 1, 1), (2, 2, 2, 2, 2)), q)
    x0 = ni // 2
    low_sends = q[:, NG:NG + nk, NG:NG + nj, NG + x0 - 2:NG + x0].reshape(-1)    # +x face of block 0
    high_sends = q[:, NG:NG + nk, NG:NG + nj, NG + x0:NG + x0 + 2].reshape(-1)   # -x face of block 1
    assert np.array_equal(buf, np.concatenate([low_sends, high_sends]))
    # a planted slip (j fastest instead of i) is caught
    wrong = q[:, NG:NG + nk, NG:NG + nj, NG + x0:NG + x0 + 2].transpose(0, 1, 3, 2).reshape(-1)
    assert not np.array_equal(buf[buf.size // 2:], wrong)


def test_i_face_stencil_widths(orc):
    """Sec. 4.5, Listing 2: each field sends as many layers as its stencil
    reaches (p two, u v w T one), p's box first.  Expected here: the box of
    two p layers, then the one-layer boxes of u, v, w, T, each flattened in
    (k, j, i) order."""
    ni, nj, nk = 6, 4, 5
    P = O.Problem(ni, nj, nk)
    q = np.random.default_rng(2).standard_normal(P.shape)
    buf = O.halo_pack(P, ((2, 1, 1), (2, 1, 1, 1, 1)), q)
    back = buf[buf.size // 2:]                         # the -x face of the high block
    x0 = ni // 2
    p_box = q[0, NG:NG + nk, NG:NG + nj, NG + x0:NG + x0 + 2].reshape(-1)
    rest = [q[f, NG:NG + nk, NG:NG + nj, NG + x0:NG + x0 + 1].reshape(-1) for f in range(1, 5)]
    assert back.size == 2 * nk * nj + 4 * nk * nj
    assert np.array_equal(back, np.concatenate([p_box] + rest))


@pytest.mark.parametrize("split,width", [((2, 2, 2), (1, 2, 2, 2, 2)), ((8, 1, 1), (2, 1, 1, 1, 1)),
                                         ((1, 4, 2), (2, 2, 2, 2, 2))])
def test_unpack_round_trip_and_poison(orc, split, width):
    P = O.Problem(16)
    halo = (split, width)
    q = np.random.default_rng(3).standard_normal(P.shape)
    q0 = q.copy()
    buf = O.halo_pack(P, halo, q)
    O.halo_unpack(P, halo, buf, q)
    assert np.array_equal(q, q0)
    # poison every segment cell, then unpack restores them bit for bit
    mark = np.zeros(P.shape)
    O.halo_unpack(P, halo, np.ones(buf.size), mark)
    assert 0 < mark.sum() <= buf.size   # boxes of one sender may share corner cells
    q[mark == 1] = np.nan
    O.halo_unpack(P, halo, buf, q)
    assert np.array_equal(q, q0)


# ---------------------------------------------------------------------------
# Widths against the stencil reach (Sec. 3.1: p reads 2 cells, u v w T 1).
# With really separate subdomains a receiver sees only the w_f layers the
# exchange sent; whatever lies beyond them is stale.  Marking those cells NaN
# in the global array and evaluating the residual of one subdomain shows
# which widths suffice: the paper's stencil widths (p 2, others 1)
# reproduce the global residual exactly, while p = 1 (the widths of the
# single-array timed runs) or a zero width do not.
def _residual_seen_by(n, split_axis, w, seed=5):
    from oracle import tangent as TG
    ni, nj, nk = n
    P = O.Problem(ni, nj, nk, Ra=1e5)
    q = O.init(P, seed, 1e-2)
    C = TG.Case(ni, nj, nk, 1e5, np.full(nj * nk, 1.0))
    g = q.copy()
    TG.apply_bc(C, g)
    R_ref, _ = TG.residual(C, g)
    e = (ni, nj, nk)[split_axis] // 2          # one cut, at e
    seen = g.copy()
    for f in range(5):
        idx = [f, slice(None), slice(None), slice(None)]
        idx[3 - split_axis] = slice(O.NG + e + w[f], None)   # beyond the width, on the far side
        seen[tuple(idx)] = np.nan
    R, _ = TG.residual(C, seen)
    near = [slice(None), slice(None), slice(None), slice(None)]
    near[3 - split_axis] = slice(0, e)                          # the subdomain below the cut
    return R[tuple(near)], R_ref[tuple(near)]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_stencil_widths_suffice_for_separate_subdomains(axis):
    got, ref = _residual_seen_by((12, 10, 8), axis, (2, 1, 1, 1, 1))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("w", [(1, 2, 2, 2, 2), (2, 0, 1, 1, 1), (2, 1, 1, 1, 0)])
def test_narrower_widths_break_separate_subdomains(w):
    got, ref = _residual_seen_by((12, 10, 8), 0, w)
    assert not np.isfinite(got).all()
