"""The library's derivative bboxsets and level exchange schedule (host code,
no GPU) against the boolean-grid oracle: the same points, the same key
points, disjoint box decompositions, and a ghost-exchange schedule that
matches the brute-force source of every ghost point."""

import random

import numpy as np
import pytest

import oracle.bboxset as B
import paper_1308_1343_amd as S
import workload as W

from test_bboxset_oracle import GOLD, random_boxes


def grid_of(bset, wlo, shape):
    boxes = S.s4_bset_boxes(bset)
    chi = B.rasterize(boxes, wlo, shape)
    assert B.disjoint_cover(boxes, chi, wlo), "box decomposition is not disjoint"
    return chi


def check_same(bset, chi, wlo):
    info = S.s4_bset_info(bset)
    assert info["points"] == int(chi.sum())
    got = grid_of(bset, wlo, chi.shape)
    assert np.array_equal(got, chi)
    kp = B.key_points(chi, wlo)
    assert sorted(S.s4_bset_keys(bset)) == kp
    assert info["keys"] == len(kp)


@pytest.mark.parametrize("name", ["l_shape", "cuboid", "frame"])
def test_worked_examples(name):
    ex = GOLD[name]
    a = S.s4_bset_from_boxes(ex["dim"], [(tuple(l), tuple(h)) for l, h in ex["boxes"]])
    info = S.s4_bset_info(a)
    assert info["points"] == ex["points"] and info["keys"] == ex["key_count"]
    assert sorted(S.s4_bset_keys(a)) == sorted(tuple(p) for p in ex["key_points"])


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_union_of_boxes(dim):
    rng = random.Random(500 + dim)
    for k in (0, 1, 2, 5, 12):
        boxes = random_boxes(rng, dim, k)
        wlo, shape = B.window_of(boxes, dim)
        check_same(S.s4_bset_from_boxes(dim, boxes), B.rasterize(boxes, wlo, shape), wlo)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_set_operations(dim):
    rng = random.Random(600 + dim)
    for _ in range(8):
        r, s = random_boxes(rng, dim, 4), random_boxes(rng, dim, 4)
        wlo, shape = B.window_of(r + s, dim)
        R, Sg = B.rasterize(r, wlo, shape), B.rasterize(s, wlo, shape)
        a, b = S.s4_bset_from_boxes(dim, r), S.s4_bset_from_boxes(dim, s)
        for name, f in B.SET_OPS.items():
            check_same(S.s4_bset_op(name, a, b), f(R, Sg), wlo)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_shift_expand_derivative_contains(dim):
    rng = random.Random(700 + dim)
    for _ in range(5):
        r = random_boxes(rng, dim, 4, span=6, maxlen=5)
        wlo, shape = B.window_of(r, dim, margin=5)
        R = B.rasterize(r, wlo, shape)
        a = S.s4_bset_from_boxes(dim, r)
        v = [rng.randrange(-3, 4) for _ in range(dim)]
        check_same(S.s4_bset_shift(a, v), B.translate(R, v), wlo)
        lo = [rng.randrange(0, 3) for _ in range(dim)]
        hi = [rng.randrange(0, 3) for _ in range(dim)]
        check_same(S.s4_bset_expand(a, lo, hi), B.expand(R, lo, hi), wlo)
        for ax in range(dim):
            check_same(S.s4_bset_derivative(a, ax), B.derivative(R, ax), wlo)
        mem = set(B.members(R, wlo))
        for off in np.ndindex(*shape):
            p = tuple(o + l for o, l in zip(off, wlo))
            assert S.s4_bset_contains(a, p) == (p in mem)


def test_equality_is_set_equality():
    rng = random.Random(800)
    r, s = random_boxes(rng, 3, 5), random_boxes(rng, 3, 5)
    a, b = S.s4_bset_from_boxes(3, r), S.s4_bset_from_boxes(3, s)
    x = S.s4_bset_op("symmetric_difference", S.s4_bset_op("symmetric_difference", a, b), b)
    assert S.s4_bset_equal(x, a)
    # the same set from a different box list (its own decomposition)
    assert S.s4_bset_equal(S.s4_bset_from_boxes(3, S.s4_bset_boxes(a)), a)
    assert not S.s4_bset_equal(a, b)


def test_bset_errors():
    L = S.lib()
    with pytest.raises(S.Sten4Error) as e:
        S.s4_bset_from_boxes(4, [])
    assert e.value.code == S.S4_EINVAL
    with pytest.raises(S.Sten4Error):
        S.s4_bset_from_boxes(1, [((0,), (1 << 41,))])
    a2, a3 = S.s4_bset_from_boxes(2, [((0, 0), (1, 1))]), S.s4_bset_from_boxes(3, [((0, 0, 0), (1, 1, 1))])
    with pytest.raises(S.Sten4Error):
        S.s4_bset_op("union", a2, a3)
    with pytest.raises(S.Sten4Error):
        S.s4_bset_op(9, a2, a2)
    with pytest.raises(S.Sten4Error):
        S.s4_bset_derivative(a2, 2)
    with pytest.raises(S.Sten4Error):
        S.s4_bset_expand(a2, [-1, 0], [0, 0])
    assert L.s4_bset_op(0, None, None, None) == S.S4_EINVAL
    L.s4_bset_free(None)


# --------------------------------------------------------------------------- level schedule

def level_boxes(d):
    g = d["ghost"]
    boxes = []
    for b in d["boxes"]:
        nx, ny, nz = b["n"]
        sy = nx + 2 * g
        boxes.append(S.make_box(b["n"], g, (1, sy, sy * (ny + 2 * g)), d["dx"]))
    return boxes


def small_level(**kw):
    return W.level_tiling(counts=(3, 3, 2), smin=4, smax=9, **kw)


@pytest.mark.parametrize("shape", ["faces", "full"])
@pytest.mark.parametrize("width", [1, 2, 3])
def test_schedule_matches_brute_force(shape, width):
    d = small_level()
    lo = [b["lo"] for b in d["boxes"]]
    n = [b["n"] for b in d["boxes"]]
    L = S.s4_level_create(level_boxes(d), lo, d["domain"], width, shape)
    info = S.s4_level_info(L)
    filled, unc = B.check_pieces(S.s4_level_pieces(L), lo, n, d["ghost"], d["domain"], width, shape)
    assert unc == 0 and info["uncovered"] == 0
    assert info["filled"] == filled and info["points"] == int(np.prod(d["domain"]))


@pytest.mark.parametrize("domain_mask", [(1, 1, 1), (0, 1, 1), (0, 0, 0)])
def test_schedule_partial_and_open(domain_mask):
    d = small_level()
    keep = [i for i in range(len(d["boxes"])) if i % 3 != 1]  # holes between the boxes
    boxes = [level_boxes(d)[i] for i in keep]
    lo = [d["boxes"][i]["lo"] for i in keep]
    n = [d["boxes"][i]["n"] for i in keep]
    dom = tuple(v * m for v, m in zip(d["domain"], domain_mask))
    L = S.s4_level_create(boxes, lo, dom, 2, "full")
    info = S.s4_level_info(L)
    filled, unc = B.check_pieces(S.s4_level_pieces(L), lo, n, d["ghost"], dom, 2, "full")
    assert (info["filled"], info["uncovered"]) == (filled, unc) and unc > 0


def test_full_size_level_counts():
    d = W.level_tiling()
    boxes = level_boxes(d)
    lo = [b["lo"] for b in d["boxes"]]
    L = S.s4_level_create(boxes, lo, d["domain"], 2, "faces")
    info = S.s4_level_info(L)
    want = sum(2 * 2 * (b["n"][1] * b["n"][2] + b["n"][0] * b["n"][2] + b["n"][0] * b["n"][1]) for b in d["boxes"])
    assert info["uncovered"] == 0 and info["filled"] == want and info["boxes"] == 60
    assert info["points"] == int(np.prod(d["domain"]))
    assert S.s4_level_workspace_size(L, S.S4_OP_RK4) > S.s4_level_workspace_size(L, S.S4_OP_LEVEL_SYNC)


def test_level_errors():
    d = small_level()
    boxes, lo = level_boxes(d), [b["lo"] for b in d["boxes"]]

    def code(**kw):
        args = dict(boxes=boxes, lo=lo, domain=d["domain"], width=2, shape="faces")
        args.update(kw)
        with pytest.raises(S.Sten4Error) as e:
            S.s4_level_create(**args)
        return e.value.code

    bad_lo = list(lo)
    bad_lo[1] = lo[0]
    assert code(lo=bad_lo) == S.S4_EINVAL                          # overlap
    assert code(domain=(d["domain"][0] - 1,) + tuple(d["domain"][1:])) == S.S4_EINVAL  # outside
    assert code(width=4) == S.S4_EGHOST
    assert code(width=0) == S.S4_EGHOST
    assert code(shape=5) == S.S4_EINVAL
    other = list(boxes)
    other[2] = S.make_box(d["boxes"][2]["n"], d["ghost"], tuple(boxes[2].stride), 0.5)
    assert code(boxes=other) == S.S4_EINVAL                        # two spacings on one level


@pytest.mark.parametrize("shape", ["faces", "full"])
def test_schedule_many_small_boxes(shape):
    # 216 boxes of sides 3..8: boxes narrower than the ghost zone reach past their neighbours
    d = W.level_tiling(counts=(6, 6, 6), smin=3, smax=8)
    lo = [b["lo"] for b in d["boxes"]]
    n = [b["n"] for b in d["boxes"]]
    L = S.s4_level_create(level_boxes(d), lo, d["domain"], 3, shape)
    info = S.s4_level_info(L)
    filled, unc = B.check_pieces(S.s4_level_pieces(L), lo, n, d["ghost"], d["domain"], 3, shape)
    assert unc == 0 and info["uncovered"] == 0 and info["filled"] == filled
