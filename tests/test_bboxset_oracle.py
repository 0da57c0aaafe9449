"""Pins of the boolean-grid bboxset oracle (Sec. II-B, II-C) to things fixed outside it.

The worked examples of Sec. II-B (an L-shape stored as 6 points, a cuboid as
8) with hand-written corner coordinates, brute-force membership from box
lists in plain Python, Python set algebra on member tuples, the identities
the section states (derivatives commute, the anti-derivative recovers the
set, the xor of two sets is the xor of their derivatives), and hand-counted
ghost-exchange cases.  A derivative taken in the wrong direction, a dropped
axis, a wrong set operation or a wrong periodic image fails one of them.
"""

import json
import os
import random

import numpy as np
import pytest

import oracle.bboxset as B

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bboxset_examples.json")))


def random_boxes(rng, dim, k, span=12, maxlen=6):
    out = []
    for _ in range(k):
        lo = [rng.randrange(-span, span) for _ in range(dim)]
        hi = [l + rng.randrange(1, maxlen + 1) for l in lo]
        out.append((tuple(lo), tuple(hi)))
    return out


@pytest.mark.parametrize("name", ["l_shape", "cuboid", "frame"])
def test_worked_examples(name):
    ex = GOLD[name]
    boxes = [(tuple(lo), tuple(hi)) for lo, hi in ex["boxes"]]
    wlo, shape = B.window_of(boxes, ex["dim"])
    chi = B.rasterize(boxes, wlo, shape)
    assert int(chi.sum()) == ex["points"]
    kp = B.key_points(chi, wlo)
    assert len(kp) == ex["key_count"]
    assert kp == sorted(tuple(p) for p in ex["key_points"])


def test_interval_derivative_by_definition():
    # 1D, straight from (d R)(p) = R(p) xor R(p - 1), point by point
    for a, b in [(0, 1), (-3, 4), (5, 9)]:
        boxes = [((a,), (b,))]
        wlo, shape = B.window_of(boxes, 1)
        chi = B.rasterize(boxes, wlo, shape)
        want = [p for p in range(wlo[0], wlo[0] + shape[0])
                if B.contains_brute(boxes, (p,)) != B.contains_brute(boxes, (p - 1,))]
        assert want == [a, b]
        assert [p[0] for p in B.members(B.derivative(chi, 0), wlo)] == want


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_rasterize_and_translate_brute_force(dim):
    rng = random.Random(100 + dim)
    for _ in range(5):
        boxes = random_boxes(rng, dim, 4, span=5, maxlen=4)
        wlo, shape = B.window_of(boxes, dim, margin=3)
        chi = B.rasterize(boxes, wlo, shape)
        mem = set(B.members(chi, wlo))
        for off in np.ndindex(*shape):
            p = tuple(o + l for o, l in zip(off, wlo))
            assert (p in mem) == B.contains_brute(boxes, p)
        v = tuple(rng.randrange(-2, 3) for _ in range(dim))
        moved = set(B.members(B.translate(chi, v), wlo))
        assert moved == {tuple(x + d for x, d in zip(p, v)) for p in mem}


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_set_ops_match_python_sets(dim):
    rng = random.Random(200 + dim)
    for _ in range(6):
        r = random_boxes(rng, dim, 3)
        s = random_boxes(rng, dim, 3)
        wlo, shape = B.window_of(r + s, dim)
        R, S = B.rasterize(r, wlo, shape), B.rasterize(s, wlo, shape)
        mr, ms = set(B.members(R, wlo)), set(B.members(S, wlo))
        py = {"union": mr | ms, "intersection": mr & ms, "difference": mr - ms,
              "symmetric_difference": mr ^ ms}
        for name, f in B.SET_OPS.items():
            assert set(B.members(f(R, S), wlo)) == py[name], name


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_derivative_identities(dim):
    rng = random.Random(300 + dim)
    for _ in range(6):
        r = random_boxes(rng, dim, 4)
        s = random_boxes(rng, dim, 4)
        wlo, shape = B.window_of(r + s, dim, margin=2)  # room for two derivatives along one axis
        R, S = B.rasterize(r, wlo, shape), B.rasterize(s, wlo, shape)
        # derivatives commute
        for a in range(dim):
            for b in range(dim):
                assert np.array_equal(B.derivative(B.derivative(R, a), b), B.derivative(B.derivative(R, b), a))
        # the anti-derivative (a low-to-high scan) recovers the set, axis by axis and from the key points
        for a in range(dim):
            assert np.array_equal(B.antiderivative(B.derivative(R, a), a), R)
        D = B.full_derivative(R)
        for a in range(dim):
            D = B.antiderivative(D, a)
        assert np.array_equal(D, R)
        # the symmetric difference acts on derivatives directly
        assert np.array_equal(B.full_derivative(R ^ S), B.full_derivative(R) ^ B.full_derivative(S))


def test_key_points_count_boxes():
    # separated cuboids: 8 points each; touching along a full face: they merge into one cuboid
    far = [((0, 0, 0), (2, 3, 4)), ((10, 0, 0), (12, 2, 2)), ((0, 10, 5), (3, 13, 6))]
    wlo, shape = B.window_of(far, 3)
    assert len(B.key_points(B.rasterize(far, wlo, shape), wlo)) == 24
    glued = [((0, 0, 0), (2, 3, 4)), ((2, 0, 0), (7, 3, 4))]
    wlo, shape = B.window_of(glued, 3)
    assert B.key_points(B.rasterize(glued, wlo, shape), wlo) == sorted(
        (x, y, z) for x in (0, 7) for y in (0, 3) for z in (0, 4))


def test_expand_brute_force():
    rng = random.Random(400)
    for dim in (1, 2, 3):
        boxes = random_boxes(rng, dim, 3, span=4, maxlen=3)
        lo = [rng.randrange(0, 3) for _ in range(dim)]
        hi = [rng.randrange(0, 3) for _ in range(dim)]
        wlo, shape = B.window_of(boxes, dim, margin=3)
        chi = B.rasterize(boxes, wlo, shape)
        mem = B.members(chi, wlo)
        got = set(B.members(B.expand(chi, lo, hi), wlo))
        want = set()
        for p in mem:
            for d in np.ndindex(*[l + h + 1 for l, h in zip(lo, hi)]):
                want.add(tuple(x + di - l for x, di, l in zip(p, d, lo)))
        assert got == want


@pytest.mark.parametrize("n,g,w", [((5, 4, 3), 3, 2), ((2, 2, 2), 2, 2), ((6, 3, 4), 3, 1)])
def test_sync_mask_counts(n, g, w):
    full = B.sync_mask(n, g, w, "full")
    faces = B.sync_mask(n, g, w, "faces")
    assert int(full.sum()) == np.prod([m + 2 * w for m in n]) - np.prod(n)
    assert int(faces.sum()) == 2 * w * (n[1] * n[2] + n[0] * n[2] + n[0] * n[1])
    assert not (faces & ~full).any()


def test_sync_sources_two_slabs_by_hand():
    # domain 8 x 4 x 4 cut at x = 4; box 1 is box 0 moved by +4 in x
    lo, n, dom = [(0, 0, 0), (4, 0, 0)], [(4, 4, 4), (4, 4, 4)], (8, 4, 4)
    src = B.sync_sources(lo, n, 2, dom, 2, "full")
    for b in range(2):
        pts, who, s = src[b]
        table = {tuple(p): (int(w_), tuple(int(v) for v in q)) for p, w_, q in zip(pts, who, s)}
        other = 1 - b
        # x ghosts come from the other box (periodically on the far side), y and z ghosts from itself
        assert table[(-1, 0, 0)] == (other, (3, 0, 0))
        assert table[(-2, 1, 2)] == (other, (2, 1, 2))
        assert table[(4, 3, 3)] == (other, (0, 3, 3))
        assert table[(5, 0, 1)] == (other, (1, 0, 1))
        assert table[(0, -1, 0)] == (b, (0, 3, 0))
        assert table[(2, 1, 5)] == (b, (2, 1, 1))
        assert table[(-1, -2, 4)] == (other, (3, 2, 0))
        assert (who >= 0).all()


def test_sync_sources_partial_level():
    # one small box in a large periodic domain: no box covers any of its ghost points
    lo, n, dom = [(2, 2, 2)], [(3, 3, 3)], (10, 10, 10)
    pts, who, _ = B.sync_sources(lo, n, 2, dom, 2, "faces")[0]
    assert (who == -1).all() and len(who) == 2 * 2 * 27


def _two_slab_pieces():
    # hand-made exchange for the two-slab case, "faces", width 2
    P = []
    for b in range(2):
        o = 1 - b
        P.append((b, o, (-2, 0, 0), (2, 0, 0), (2, 4, 4)))   # low x face from the other box
        P.append((b, o, (4, 0, 0), (0, 0, 0), (2, 4, 4)))    # high x face
        P.append((b, b, (0, -2, 0), (0, 2, 0), (4, 2, 4)))   # y faces wrap onto the box itself
        P.append((b, b, (0, 4, 0), (0, 0, 0), (4, 2, 4)))
        P.append((b, b, (0, 0, -2), (0, 0, 2), (4, 4, 2)))   # z faces
        P.append((b, b, (0, 0, 4), (0, 0, 0), (4, 4, 2)))
    return P


def test_check_pieces_accepts_hand_schedule():
    lo, n, dom = [(0, 0, 0), (4, 0, 0)], [(4, 4, 4), (4, 4, 4)], (8, 4, 4)
    filled, unc = B.check_pieces(_two_slab_pieces(), lo, n, 2, dom, 2, "faces")
    assert unc == 0 and filled == 2 * 2 * 2 * 3 * 16


@pytest.mark.parametrize("k", range(4))
def test_check_pieces_rejects_planted_mistakes(k):
    lo, n, dom = [(0, 0, 0), (4, 0, 0)], [(4, 4, 4), (4, 4, 4)], (8, 4, 4)
    P = _two_slab_pieces()
    d, s, d0, s0, e = P[0]
    bad = [(d, d, d0, s0, e),                              # wrong source box
           (d, s, d0, (s0[0] - 1,) + s0[1:], e),          # source off by one
           (d, s, d0, s0, (1,) + e[1:]),                  # a layer missing
           (d, s, (d0[0] - 1,) + d0[1:], s0, e)][k]       # writes a point outside the mask
    P[0] = bad
    with pytest.raises(AssertionError):
        B.check_pieces(P, lo, n, 2, dom, 2, "faces")


def test_level_owner_rejects_overlap():
    with pytest.raises(AssertionError):
        B.level_owner([(0, 0, 0), (1, 0, 0)], [(2, 2, 2), (2, 2, 2)], (4, 4, 4))
    with pytest.raises(AssertionError):
        B.level_owner([(3, 0, 0)], [(2, 2, 2)], (4, 4, 4))


def test_sync_sources_open_axis_by_hand():
    # the two-slab level with x open: the outer x faces have no source, the inner ones face each other
    lo, n, dom = [(0, 0, 0), (4, 0, 0)], [(4, 4, 4), (4, 4, 4)], (0, 4, 4)
    src = B.sync_sources(lo, n, 2, dom, 2, "faces")
    t0 = {tuple(p): int(w) for p, w in zip(src[0][0], src[0][1])}
    t1 = {tuple(p): int(w) for p, w in zip(src[1][0], src[1][1])}
    assert t0[(-1, 0, 0)] == -1 and t0[(4, 0, 0)] == 1 and t0[(0, -1, 0)] == 0
    assert t1[(4, 2, 2)] == -1 and t1[(-2, 3, 1)] == 0
    assert sum(w == -1 for w in t0.values()) == 2 * 16 and sum(w == -1 for w in t1.values()) == 2 * 16
