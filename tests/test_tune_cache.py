"""Tuning cache files (S4_TUNE_CACHE) read on the host: an entry names its
candidate by parameters, and an entry that names no candidate of this build,
or one the loop setup's op cannot run on its boxes, is ignored (the context
then falls back to its heuristic).  s4_tune_cache_lookup reads a file the
way s4_create does, without a device."""
import json

import paper_1308_1343_amd as S

DEV = "gfx950"


def box(n, g=2):
    nx, ny, nz = n
    sy = nx + 2 * g
    return S.make_box(n, g, (1, sy, sy * (ny + 2 * g)), 1.0 / nx)


def key(op, boxes, c2=False, level=0):
    """The loop-setup key format documented beside S4_TUNE_CACHE."""
    k = f"op{op}|{DEV}|{len(boxes)}"
    for b in boxes:
        k += f"|{b.n[0]},{b.n[1]},{b.n[2]},g{b.ghost},s{b.stride[1]},{b.stride[2]}"
    return k + ("|c2" if c2 else "") + {0: "", 1: "|level", 2: "|level4"}[level]


def lookup(tmp_path, entries, op, boxes, level=0):
    p = tmp_path / "tune.json"
    p.write_text(entries if isinstance(entries, str) else json.dumps(entries))
    return S.s4_tune_cache_lookup(str(p), DEV, op, boxes, level)


WHOLE = "v4 x32 w8 z32 r0"     # whole-step kernels: RK4 only
PAIR1 = "v1 x32 w8 z32 r0"     # widened-tile stage pairs: RK4 on one box only
TILES = "v0 x64 w8 z64 r0"     # tile traversal: every op


def test_tags_name_distinct_candidates(tmp_path):
    b = [box((64, 64, 64))]
    got = {t: lookup(tmp_path, {key(S.S4_OP_RK4, b): t}, S.S4_OP_RK4, b) for t in (WHOLE, PAIR1, TILES)}
    assert all(v >= 0 for v in got.values()), got
    assert len(set(got.values())) == 3


def test_index_written_by_an_older_build_is_ignored(tmp_path):
    b = [box((64, 64, 64))]
    assert lookup(tmp_path, {key(S.S4_OP_RK4, b): 79}, S.S4_OP_RK4, b) == -1
    # a valid entry beside it is still read
    e = '{"%s": 79, "%s": "%s"}' % (key(S.S4_OP_WAVE_RHS, b), key(S.S4_OP_RK4, b), WHOLE)
    assert lookup(tmp_path, e, S.S4_OP_WAVE_RHS, b) == -1
    assert lookup(tmp_path, e, S.S4_OP_RK4, b) >= 0


def test_unknown_candidate_is_ignored(tmp_path):
    b = [box((64, 64, 64))]
    assert lookup(tmp_path, {key(S.S4_OP_RK4, b): "v4 x48 w8 z32 r0"}, S.S4_OP_RK4, b) == -1
    assert lookup(tmp_path, {key(S.S4_OP_RK4, b): "v9 x32 w8 z32 r0"}, S.S4_OP_RK4, b) == -1


def test_candidate_the_op_cannot_run_is_ignored(tmp_path):
    one = [box((64, 64, 64))]
    two = [box((32, 32, 32)), box((40, 24, 16))]
    # whole-step kernels do not compute a plain RHS
    assert lookup(tmp_path, {key(S.S4_OP_WAVE_RHS, one): WHOLE}, S.S4_OP_WAVE_RHS, one) == -1
    assert lookup(tmp_path, {key(S.S4_OP_WAVE_RHS, one): TILES}, S.S4_OP_WAVE_RHS, one) >= 0
    # the widened-tile stage pairs run on one box only
    assert lookup(tmp_path, {key(S.S4_OP_RK4, two): PAIR1}, S.S4_OP_RK4, two) == -1
    assert lookup(tmp_path, {key(S.S4_OP_RK4, two): WHOLE}, S.S4_OP_RK4, two) >= 0
    # a level runs only kernel sets that read radius-2 ghost zones
    lk = key(S.S4_OP_RK4, two, level=1)
    assert lookup(tmp_path, {lk: WHOLE}, S.S4_OP_RK4, two, level=1) == -1
    assert lookup(tmp_path, {lk: TILES}, S.S4_OP_RK4, two, level=1) >= 0
    # a wide level (exchanges of width 4) runs whole steps, never the widened-tile pairs
    wk = key(S.S4_OP_RK4, two, level=2)
    assert lookup(tmp_path, {wk: WHOLE}, S.S4_OP_RK4, two, level=2) >= 0
    assert lookup(tmp_path, {wk: PAIR1}, S.S4_OP_RK4, two, level=2) == -1
    assert lookup(tmp_path, {lk: WHOLE}, S.S4_OP_RK4, two, level=2) == -1  # keys differ


def test_whole_steps_need_z_planes_below_2gib(tmp_path):
    big = [box((16384, 16384, 4))]  # one z plane of 2.1 GB
    assert lookup(tmp_path, {key(S.S4_OP_RK4, big): WHOLE}, S.S4_OP_RK4, big) == -1


def test_c2_setup_has_its_own_key(tmp_path):
    b = [box((64, 64, 64))]
    e = {key(S.S4_OP_RK4, b, c2=True): WHOLE}
    assert lookup(tmp_path, e, S.S4_OP_RK4 | S.S4_WITH_C2, b) >= 0
    assert lookup(tmp_path, e, S.S4_OP_RK4, b) == -1


def test_other_device_and_garbage(tmp_path):
    b = [box((64, 64, 64))]
    e = {key(S.S4_OP_RK4, b).replace(DEV, "gfx942"): WHOLE}
    assert lookup(tmp_path, e, S.S4_OP_RK4, b) == -1
    assert lookup(tmp_path, "not json at all", S.S4_OP_RK4, b) == -1
    assert lookup(tmp_path, '{"unterminated": "v4 x32', S.S4_OP_RK4, b) == -1
    try:
        S.s4_tune_cache_lookup(str(tmp_path / "missing.json"), DEV, S.S4_OP_RK4, b)
        assert False, "missing file accepted"
    except S.Sten4Error as e:
        assert e.code == S.S4_EINVAL
