"""HIP path against the FP64 oracle, through the C ABI.

Tolerance: max-norm relative error over interior points <= 1e-12 (the kernels
fuse multiply-adds and scale by precomputed 1/(12 h^2), the oracle divides
and does not fuse, so results agree to rounding, not bit for bit).  Integer
and copy work (ghost fill) is compared bit for bit; tile shapes and launch
modes of the HIP path are compared with each other bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1308_1343_amd as S
import workload as W
from _gpu import cands_by_kind, NAN, dev, dev_full, ghosts_untouched, host, inner, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    return S.Context(0)


def rand_box(n, g, seed, stream):
    nx, ny, nz = n
    return O.embed(W.uniform_pm1(seed, stream, (nz, ny, nx)), g)


SHAPES = [((32, 32, 32), 2), ((37, 19, 23), 2), ((5, 7, 6), 3), ((70, 9, 5), 3), ((1, 3, 2), 2), ((64, 64, 16), 2)]


@pytest.mark.parametrize("n,g", SHAPES)
@pytest.mark.parametrize("pad", [True, False])
def test_fill_bitexact(ctx, n, g, pad):
    a = rand_box(n, g, 1, 1)
    t = dev(a, g, pad)
    if min(n) < g:
        # a periodic fill copies g layers from an interior of fewer points:
        # rejected on the host before any launch, the field left as it was
        before = host(t)
        with pytest.raises(S.Sten4Error) as e:
            S.s4_fill_ghosts_periodic(ctx, S.box_of(t, g, 0.1), [t])
        assert e.value.code == S.S4_EGHOST
        np.testing.assert_array_equal(host(t), before)
        return
    S.s4_fill_ghosts_periodic(ctx, S.box_of(t, g, 0.1), [t])
    want = O.fill_ghosts_periodic(a.copy(), g)
    np.testing.assert_array_equal(host(t), want)


@pytest.mark.parametrize("n,g", SHAPES)
@pytest.mark.parametrize("with_c2", [False, True])
def test_wave_rhs_parity(ctx, n, g, with_c2):
    dx = (1.0 / 32, 1.0 / 24, 1.0 / 40)
    a = O.fill_ghosts_periodic(rand_box(n, g, 2, 1), g)
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(2, 2, n[::-1]), g) if with_c2 else None
    u = dev_full(a, g)
    c2d = dev(c2, g) if with_c2 else None
    out = S.alloc_field(n, g, fill=NAN)
    b = S.box_of(u, g, dx)
    S.s4_wave_rhs(ctx, b, [u], None if c2d is None else [c2d], [out])
    got = host(out)
    want = O.wave_rhs(a, g, dx, c2)
    assert rel(got, want, g) <= TOL
    assert np.all(np.isfinite(inner(got, g))) and ghosts_untouched(got, g)


def test_wave32_rhs_and_candidates_bitwise(ctx):
    d = W.wave32()
    g = d["ghost"]
    a = O.fill_ghosts_periodic(O.embed(d["u"], g), g)
    u = dev_full(a, g)
    b = S.box_of(u, g, d["dx"])
    want = O.wave_rhs(a, g, d["dx"])
    ref = None
    k = cands_by_kind(ctx, S.S4_OP_WAVE_RHS, b)
    assert k["pairs"] and not k["fused"]
    for cand in k["tiles"] + k["rows"] + k["pairs"]:
        S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, b, cand)
        out = S.alloc_field(d["n"], g, fill=NAN)
        S.s4_wave_rhs(ctx, b, [u], None, [out])
        got = host(out)
        if ref is None:
            ref = got
            assert rel(got, want, g) <= TOL
        np.testing.assert_array_equal(got, ref, err_msg=f"candidate {cand}")
    S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, b, -1)


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
def test_wave32_rk4_parity(ctx, mode):
    d = W.wave32()
    g = d["ghost"]
    u0, r0 = O.embed(d["u"], g), O.embed(d["rho"], g)
    wu, wr = O.rk4(u0, r0, g, d["dx"], d["dt"], d["nsteps"])
    u, r = dev(u0, g), dev(r0, g)
    b = S.box_of(u, g, d["dx"])
    S.s4_rk4(ctx, b, [u], [r], None, d["dt"], d["nsteps"], mode)
    gu, gr = host(u), host(r)
    assert rel(gu, wu, g) <= TOL and rel(gr, wr, g) <= TOL
    assert ghosts_untouched(gu, g) and ghosts_untouched(gr, g)


def test_rk4_modes_and_candidates_bitwise(ctx):
    n, g = (37, 19, 23), 2
    dx = (1 / 37, 1 / 19, 1 / 23)
    dt = 0.2 / 37
    u0, r0 = rand_box(n, g, 3, 1), rand_box(n, g, 3, 2)
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(3, 3, n[::-1]), g)
    wu, wr = O.rk4(u0, r0, g, dx, dt, 3, c2)
    c2d = dev(c2, g)
    ref = None
    b = None
    nc = None
    kinds = None
    for cand in [None, 0, 7, 13, 21, 29, "rows", "fused"]:
        for mode in ["perbox", "graph"]:
            u, r = dev(u0, g), dev(r0, g)
            b = S.box_of(u, g, dx)
            if kinds is None:
                kinds = cands_by_kind(ctx, S.S4_OP_RK4, b)
            cl = kinds[cand] if isinstance(cand, str) else [cand]
            for cc in cl:
                u, r = dev(u0, g), dev(r0, g)
                if cc is not None:
                    S.s4_set_choice(ctx, S.S4_OP_RK4, b, cc)
                S.s4_rk4(ctx, b, [u], [r], [c2d], dt, 3, mode)  # odd: fused pair + one stage-kernel step
                got = (host(u), host(r))
                if ref is None:
                    ref = got
                    assert rel(got[0], wu, g) <= TOL and rel(got[1], wr, g) <= TOL
                np.testing.assert_array_equal(got[0], ref[0], err_msg=f"candidate {cc} {mode}")
                np.testing.assert_array_equal(got[1], ref[1], err_msg=f"candidate {cc} {mode}")
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, -1)
    # even step counts end in the caller's buffers after fused pairs only
    wu4, wr4 = O.rk4(u0, r0, g, dx, dt, 4, c2)
    res = []
    for cc in [0, kinds["rows"][0], kinds["rows"][-1], kinds["fused"][0], kinds["fused"][-1]]:
        u, r = dev(u0, g), dev(r0, g)
        S.s4_set_choice(ctx, S.S4_OP_RK4, b, cc)
        S.s4_rk4(ctx, b, [u], [r], [c2d], dt, 4, "graph")
        res.append((host(u), host(r)))
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, -1)
    assert rel(res[0][0], wu4, g) <= TOL and rel(res[0][1], wr4, g) <= TOL
    for a in res[1:]:
        np.testing.assert_array_equal(a[0], res[0][0])
        np.testing.assert_array_equal(a[1], res[0][1])
        assert ghosts_untouched(a[0], g) and ghosts_untouched(a[1], g)


def small_bboxset(seed=7, nbox=9):
    seq = W.Sequence(seed, 1)
    boxes = []
    for i in range(nbox):
        n = tuple(seq.integer(5, 40) for _ in range(3))
        lev = i % 3
        h = (1.0 / 32) / 2 ** lev
        boxes.append(dict(n=n, level=lev, dx=(h, h, h)))
    return boxes


def run_bboxset(ctx, boxes, g, dt, nsteps, mode, seed=8, ws=None):
    us, rs, bs = [], [], []
    for i, bx in enumerate(boxes):
        u0, r0 = rand_box(bx["n"], g, seed, 2 * i), rand_box(bx["n"], g, seed, 2 * i + 1)
        u, r = dev(u0, g), dev(r0, g)
        us.append(u)
        rs.append(r)
        bs.append(S.box_of(u, g, bx["dx"], bx["level"]))
    S.s4_rk4(ctx, bs, us, rs, None, dt, nsteps, mode, ws=ws)
    return [host(u) for u in us], [host(r) for r in rs]


def test_bboxset_modes_match_oracle(ctx):
    boxes = small_bboxset()
    g, dt = 3, 0.25 / 128
    res = {m: run_bboxset(ctx, boxes, g, dt, 2, m) for m in ["perbox", "batched", "graph"]}
    for m in ["batched", "graph"]:
        for a, b in zip(res[m][0] + res[m][1], res["perbox"][0] + res["perbox"][1]):
            np.testing.assert_array_equal(a, b)
    for i, bx in enumerate(boxes):
        u0, r0 = rand_box(bx["n"], g, 8, 2 * i), rand_box(bx["n"], g, 8, 2 * i + 1)
        wu, wr = O.rk4(u0, r0, g, bx["dx"], dt, 2)
        assert rel(res["graph"][0][i], wu, g) <= TOL and rel(res["graph"][1][i], wr, g) <= TOL


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
@pytest.mark.parametrize("nsteps", [2, 3])
def test_bboxset_stage_pairs_bitwise(ctx, mode, nsteps):
    """Stage-pair and whole-step candidates on a set of self-periodic boxes, some with c^2 and
    some without, bit for bit against the per-stage tile kernels (odd counts end with one
    per-stage step)."""
    boxes = small_bboxset(13, 7)
    g, dt = 3, 0.25 / 128

    def run(cand):
        us, rs, cs, bs = [], [], [], []
        for i, bx in enumerate(boxes):
            us.append(dev(rand_box(bx["n"], g, 14, 2 * i), g))
            rs.append(dev(rand_box(bx["n"], g, 14, 2 * i + 1), g))
            cs.append(dev(O.embed(1.0 + 0.5 * W.uniform_pm1(14, 100 + i, bx["n"][::-1]), g), g) if i % 2 else None)
            bs.append(S.box_of(us[-1], g, bx["dx"], bx["level"]))
        S.s4_set_choice(ctx, S.S4_OP_RK4, bs, cand)
        S.s4_rk4(ctx, bs, us, rs, cs, dt, nsteps, mode)
        S.s4_set_choice(ctx, S.S4_OP_RK4, bs, -1)
        return [host(t) for t in us + rs], bs

    ref, bs = run(2)
    pairs = cands_by_kind(ctx, S.S4_OP_RK4, bs)["fused"]
    assert pairs and all(S.s4_get_choice(ctx, S.S4_OP_RK4, bs)["ncandidates"] > c for c in pairs)
    whole = [c for c in pairs if (S.s4_set_choice(ctx, S.S4_OP_RK4, bs, c) or True)
             and S.s4_get_choice(ctx, S.S4_OP_RK4, bs)["kernel_op"] == 102]
    S.s4_set_choice(ctx, S.S4_OP_RK4, bs, -1)
    assert whole  # whole RK4 steps run on sets of periodic boxes too
    for cand in sorted({pairs[0], pairs[len(pairs) // 2], pairs[-1], whole[0], whole[len(whole) // 2]}):
        got, _ = run(cand)
        for a, b_ in zip(got, ref):
            np.testing.assert_array_equal(a, b_, err_msg=f"candidate {cand}")
    # and against the oracle box by box
    for i, bx in enumerate(boxes):
        c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(14, 100 + i, bx["n"][::-1]), g) if i % 2 else None
        wu, wr = O.rk4(rand_box(bx["n"], g, 14, 2 * i), rand_box(bx["n"], g, 14, 2 * i + 1), g, bx["dx"], dt,
                       nsteps, c2)
        assert rel(ref[i], wu, g) <= TOL and rel(ref[len(boxes) + i], wr, g) <= TOL


def test_rk4_step_to_matches_in_place(ctx):
    """The out-of-place step equals s4_rk4 on a copy, bit for bit, in every kernel set."""
    n, g = (37, 19, 23), 2
    dx = (1 / 37, 1 / 19, 1 / 23)
    dt = 0.2 / 37
    u0, r0 = rand_box(n, g, 15, 1), rand_box(n, g, 15, 2)
    c2 = dev(O.embed(1.0 + 0.5 * W.uniform_pm1(15, 3, n[::-1]), g), g)
    ui, ri = dev(u0, g), dev(r0, g)
    b = S.box_of(ui, g, dx)
    kinds = cands_by_kind(ctx, S.S4_OP_RK4, b)
    for cand in (kinds["tiles"][3], kinds["rows"][0], kinds["fused"][0], kinds["fused"][-1]):
        S.s4_set_choice(ctx, S.S4_OP_RK4, b, cand)
        u, r = dev(u0, g), dev(r0, g)
        S.s4_rk4(ctx, b, [u], [r], [c2], dt, 1, "perbox")
        uo, ro = S.alloc_field(n, g, fill=NAN), S.alloc_field(n, g, fill=NAN)
        S.s4_rk4_step_to(ctx, b, ui, ri, c2, dt, uo, ro)
        np.testing.assert_array_equal(inner(host(uo), g), inner(host(u), g), err_msg=f"candidate {cand}")
        np.testing.assert_array_equal(inner(host(ro), g), inner(host(r), g), err_msg=f"candidate {cand}")
        assert ghosts_untouched(host(uo), g)
        np.testing.assert_array_equal(inner(host(ui), g), inner(u0, g))  # input untouched
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, -1)
    with pytest.raises(S.Sten4Error) as e:
        S.s4_rk4_step_to(ctx, b, ui, ri, None, dt, ui, ro)
    assert e.value.code == S.S4_EALIAS


def test_graph_replays_match_eager(ctx):
    """One captured step replayed several times, with eager work in between."""
    boxes = small_bboxset(11, 5)
    g, dt = 3, 0.25 / 128
    us, rs, bs = [], [], []
    for i, bx in enumerate(boxes):
        u, r = dev(rand_box(bx["n"], g, 12, 2 * i), g), dev(rand_box(bx["n"], g, 12, 2 * i + 1), g)
        us.append(u); rs.append(r); bs.append(S.box_of(u, g, bx["dx"]))
    ue = [dev(host(u), g) for u in us]
    re_ = [dev(host(r), g) for r in rs]
    ws = S.workspace(S.s4_workspace_size(bs, S.S4_OP_RK4, S.S4_GRAPH))
    wse = S.workspace(S.s4_workspace_size(bs, S.S4_OP_RK4, S.S4_BATCHED))
    for rep in range(4):
        S.s4_rk4(ctx, bs, us, rs, None, dt, 1, "graph", ws=ws)
        S.s4_rk4(ctx, [S.box_of(u, g, bx["dx"]) for u, bx in zip(ue, boxes)], ue, re_, None, dt, 1, "batched", ws=wse)
        torch.cuda.synchronize()
        for a, b in zip(us + rs, ue + re_):
            np.testing.assert_array_equal(host(a), host(b), err_msg=f"replay {rep}")


@pytest.mark.parametrize("with_c2", [False, True])
def test_adjoint_rhs_parity_and_identity(ctx, with_c2):
    n, g = (12, 10, 14), 2
    dx = (0.1, 0.12, 0.08)
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(4, 1, n[::-1]), g) if with_c2 else None
    lu, lr = rand_box(n, g, 4, 2), rand_box(n, g, 4, 3)
    wu, wr = O.wave_adjoint_rhs(lu, lr, g, dx, c2)
    ou, orr = S.alloc_field(n, g, fill=NAN), S.alloc_field(n, g, fill=NAN)
    lud, lrd = dev(lu, g), dev(lr, g)
    c2d = [dev(c2, g)] if with_c2 else None
    b = S.box_of(lud, g, dx)
    S.s4_wave_adjoint_rhs(ctx, b, [lud], [lrd], c2d, [ou], [orr])
    gu, gr = host(ou), host(orr)
    assert rel(gu, wu, g) <= TOL
    np.testing.assert_array_equal(inner(gr, g), inner(wr, g))
    # <A v, w> = <v, A^T w> with A v = (rho, c^2 L_p u) from the forward kernels
    v_u = O.fill_ghosts_periodic(rand_box(n, g, 4, 5), g)
    v_r = rand_box(n, g, 4, 6)
    rt = S.alloc_field(n, g, fill=NAN)
    S.s4_wave_rhs(ctx, b, [dev_full(v_u, g)], c2d, [rt])
    Av_r = host(rt)
    lhs = np.sum(inner(v_r, g) * inner(lu, g)) + np.sum(inner(Av_r, g) * inner(lr, g))
    rhs = np.sum(inner(v_u, g) * inner(gu, g)) + np.sum(inner(v_r, g) * inner(gr, g))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sum(np.abs(inner(Av_r, g) * inner(lr, g))))


@pytest.mark.parametrize("with_c2", [False, True])
def test_adjoint_step_parity(ctx, with_c2):
    n, g = (10, 12, 9), 2
    dx = (1 / 10, 1 / 12, 1 / 9)
    dt = 0.02
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(5, 1, n[::-1]), g) if with_c2 else None
    un, rn = rand_box(n, g, 5, 2), rand_box(n, g, 5, 3)
    lu, lr = rand_box(n, g, 5, 4), rand_box(n, g, 5, 5)
    cb0 = rand_box(n, g, 5, 6) if with_c2 else None
    wu, wr, wc = O.rk4_adjoint_step(un, rn, lu, lr, g, dx, dt, c2, cb0)
    und, rnd = dev(un, g), dev(rn, g)
    lud, lrd = dev(lu, g), dev(lr, g)
    c2d = dev(c2, g) if with_c2 else None
    cbd = dev(cb0, g) if with_c2 else None
    b = S.box_of(und, g, dx)
    S.s4_rk4_adjoint_step(ctx, b, und, rnd, c2d, dt, lud, lrd, cbd)
    assert rel(host(lud), wu, g) <= TOL
    assert rel(host(lrd), wr, g) <= TOL
    if with_c2:
        assert rel(host(cbd), wc, g) <= TOL
    # inputs untouched
    np.testing.assert_array_equal(inner(host(und), g), inner(un, g))


def test_tune_records_choice(ctx):
    n, g = (40, 24, 20), 2
    u = S.alloc_field(n, g, fill=0.0)
    b = S.box_of(u, g, 0.05)
    assert S.s4_get_choice(ctx, S.S4_OP_RK4, b)["tuned"] == 0
    S.s4_tune(ctx, S.S4_OP_RK4, b, flags=0)
    ch = S.s4_get_choice(ctx, S.S4_OP_RK4, b)
    assert ch["tuned"] == 1 and 0 <= ch["candidate"] < ch["ncandidates"]


def test_copy_probe(ctx):
    src = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    S.s4_copy(ctx, dst, src)
    assert torch.equal(dst, src)


def test_fused_candidates_only_for_single_box_rk4(ctx):
    n, g = (16, 16, 16), 2
    u = S.alloc_field(n, g, fill=0.0)
    b = S.box_of(u, g, 0.1)
    nc = S.s4_get_choice(ctx, S.S4_OP_RK4, b)["ncandidates"]
    for op in (S.S4_OP_WAVE_RHS, S.S4_OP_DERIV_MIXED, S.S4_OP_ADJOINT_STEP):
        with pytest.raises(S.Sten4Error) as e:
            S.s4_set_choice(ctx, op, b, nc - 1)
        assert e.value.code == S.S4_ENOTSUP
    with pytest.raises(S.Sten4Error) as e:
        S.s4_set_choice(ctx, S.S4_OP_RK4, [b, b], nc - 1)
    assert e.value.code == S.S4_ENOTSUP
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, nc - 1)
    assert S.s4_get_choice(ctx, S.S4_OP_RK4, b)["kernel_op"] == 100  # widened stage pairs: one box only
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, -1)
    # whole steps and per-tap pairs: RK4 on any number of boxes, no other op
    kinds = cands_by_kind(ctx, S.S4_OP_RK4, [b, b])
    assert {S.s4_set_choice(ctx, S.S4_OP_RK4, [b, b], c) or S.s4_get_choice(ctx, S.S4_OP_RK4, [b, b])["kernel_op"]
            for c in kinds["fused"]} == {101, 102}
    S.s4_set_choice(ctx, S.S4_OP_RK4, [b, b], -1)
    for op in (S.S4_OP_WAVE_RHS, S.S4_OP_ADJOINT_STEP):
        with pytest.raises(S.Sten4Error) as e:
            S.s4_set_choice(ctx, op, b, kinds["fused"][-1])
        assert e.value.code == S.S4_ENOTSUP
    # row-register candidates: RHS and RK4 only (any number of boxes)
    rows = cands_by_kind(ctx, S.S4_OP_RK4, b)["rows"]
    assert rows and rows == cands_by_kind(ctx, S.S4_OP_WAVE_RHS, b)["rows"]
    assert cands_by_kind(ctx, S.S4_OP_RK4, [b, b])["rows"] == rows
    for op in (S.S4_OP_DERIV_MIXED, S.S4_OP_ADJOINT_STEP, S.S4_OP_ADJOINT_RHS):
        with pytest.raises(S.Sten4Error) as e:
            S.s4_set_choice(ctx, op, b, rows[0])
        assert e.value.code == S.S4_ENOTSUP


def test_heuristic_kernel_sets(ctx):
    """Untuned RK4 starts on whole steps (one box or a set), and on the per-tap
    stage pairs where a z plane reaches 2 GiB (the whole-step stores address a
    plane with 31-bit byte offsets); the RHS on pair-lane tiles where they fit
    and fill the device; the multi-field kernel on small workgroups.
    Descriptors only: nothing is allocated."""
    fresh = S.Context(0)
    b = S.make_box((256, 256, 256), 2, (1, 272, 272 * 260), 1 / 256)
    assert S.s4_get_choice(fresh, S.S4_OP_RK4, b)["kernel_op"] == 102
    assert S.s4_get_choice(fresh, S.S4_OP_RK4, [b, b])["kernel_op"] == 102
    # 128^3: 32-plane chunks of 28 x 12 output tiles leave CUs idle (220 items);
    # 16-plane chunks fit one round of resident workgroups
    c128 = S.make_box((128, 128, 128), 2, (1, 144, 144 * 132), 1 / 128)
    ch = S.s4_get_choice(fresh, S.S4_OP_RK4, c128)
    assert (ch["kernel_op"], ch["tile_x"], ch["tile_y"], ch["z_chunk"]) == (102, 32, 16, 16), ch
    # 256^3: 68 x 15 lanes, whose 64-point output rows cover x in four tiles,
    # in 32-plane chunks (96 tiles x 8 chunks: three rounds of one workgroup per CU)
    ch = S.s4_get_choice(fresh, S.S4_OP_RK4, b)
    assert (ch["kernel_op"], ch["tile_x"], ch["tile_y"], ch["z_chunk"]) == (102, 68, 15, 32), ch
    big = S.make_box((16384, 16384, 4), 2, (1, 16400, 16400 * 16388), 1.0)
    assert S.s4_get_choice(fresh, S.S4_OP_RK4, big)["kernel_op"] == 101
    assert S.s4_get_choice(fresh, S.S4_OP_RK4, [b, big])["kernel_op"] == 101
    # the RHS on pair-lane tiles where rows and strides are even, else one point per lane
    ch = S.s4_get_choice(fresh, S.S4_OP_WAVE_RHS, b)
    assert (ch["kernel_op"], ch["tile_x"], ch["tile_y"], ch["z_chunk"]) == (300, 128, 8, 32), ch
    odd = S.make_box((255, 256, 256), 2, (1, 259, 259 * 260), 1 / 256)
    assert S.s4_get_choice(fresh, S.S4_OP_WAVE_RHS, odd)["kernel_op"] == 0
    small = S.make_box((32, 32, 32), 2, (1, 48, 48 * 36), 1 / 32)
    assert S.s4_get_choice(fresh, S.S4_OP_WAVE_RHS, small)["kernel_op"] == 0
    # the multi-field kernel: 32 x 8 lanes, the longest z chunk giving each CU one item per field
    m = S.make_box((192, 192, 192), 2, (1, 208, 208 * 196), 1 / 192)
    ch = S.s4_get_choice(fresh, S.S4_OP_DERIV_MIXED, m)
    assert (ch["tile_x"], ch["tile_y"], ch["z_chunk"]) == (32, 8, 64), ch


def test_errors_on_device_calls(ctx):
    n, g = (8, 8, 8), 2
    u = S.alloc_field(n, g, fill=0.0)
    b = S.box_of(u, g, 0.1)
    with pytest.raises(S.Sten4Error) as e:
        S.s4_wave_rhs(ctx, b, [u], None, [u])  # output aliases the stencil input
    assert e.value.code == S.S4_EALIAS
    r = S.alloc_field(n, g, fill=0.0)
    small = S.workspace(1024)
    with pytest.raises(S.Sten4Error) as e:
        S.s4_rk4(ctx, b, [u], [r], None, 0.01, 1, "perbox", ws=small)
    assert e.value.code == S.S4_ENOMEM
    with pytest.raises(S.Sten4Error) as e:
        S.s4_rk4(ctx, b, [u], [r], None, -0.01, 1, "perbox")
    assert e.value.code == S.S4_EINVAL


# --------------------------------------------------------------------------- multi-field kernel

@pytest.mark.parametrize("n,g", [((20, 17, 13), 2), ((33, 9, 12), 3), ((8, 40, 6), 2), ((70, 5, 4), 2)])
@pytest.mark.parametrize("symmetric", [True, False])
def test_mixed_parity(ctx, n, g, symmetric):
    dx = (1.0 / n[0], 1.3 / n[1], 0.9 / n[2])
    fs = [O.fill_ghosts_periodic(rand_box(n, g, 6, k), g) for k in range(3)]
    A = W.random_symmetric3(6, 9)
    if not symmetric:
        A[0, 1] += 0.3
        A[2, 0] -= 0.2
    gd = [dev_full(f, g) for f in fs]
    outs = [S.alloc_field(n, g, fill=NAN) for _ in fs]
    b = S.box_of(gd[0], g, dx)
    S.s4_deriv_mixed(ctx, b, gd, A, outs)
    for k, f in enumerate(fs):
        got = host(outs[k])
        want = O.deriv_mixed(f, g, dx, A)
        assert rel(got, want, g) <= TOL, k
        assert ghosts_untouched(got, g)


def test_mixed_candidates_bitwise_and_many_fields(ctx):
    n, g = (40, 24, 20), 2
    dx = (0.025, 0.04, 0.05)
    fs = [O.fill_ghosts_periodic(rand_box(n, g, 7, k), g) for k in range(10)]  # > 8: two launches
    A = W.random_symmetric3(7, 99)
    gd = [dev_full(f, g) for f in fs]
    b = S.box_of(gd[0], g, dx)
    ref = None
    nc = S.s4_get_choice(ctx, S.S4_OP_DERIV_MIXED, b)["ncandidates"]
    for cand in list(range(0, nc, 3)) + [nc - 1]:
        S.s4_set_choice(ctx, S.S4_OP_DERIV_MIXED, b, cand)
        outs = [S.alloc_field(n, g, fill=NAN) for _ in fs]
        S.s4_deriv_mixed(ctx, b, gd, A, outs)
        got = [host(o) for o in outs]
        if ref is None:
            ref = got
            for k, f in enumerate(fs):
                assert rel(got[k], O.deriv_mixed(f, g, dx, A), g) <= TOL
        for a, r in zip(got, ref):
            np.testing.assert_array_equal(a, r, err_msg=f"candidate {cand}")
    S.s4_set_choice(ctx, S.S4_OP_DERIV_MIXED, b, -1)


def test_mixed192_full_size(ctx):
    """The 6-field workload at its full size (192^3 + 2 ghosts, sine-mode fields)."""
    d = W.mixed_fields()
    g = d["ghost"]
    fs = [O.fill_ghosts_periodic(O.embed(f, g), g) for f in d["fields"]]
    gd = [dev_full(f, g) for f in fs]
    outs = [S.alloc_field(d["n"], g, fill=NAN) for _ in fs]
    b = S.box_of(gd[0], g, d["dx"])
    S.s4_deriv_mixed(ctx, b, gd, d["A"], outs)
    for k, f in enumerate(fs):
        got = host(outs[k])
        assert rel(got, O.deriv_mixed(f, g, d["dx"], d["A"]), g) <= TOL, k
        assert ghosts_untouched(got, g)


@pytest.mark.parametrize("with_c2", [False, True])
def test_pair_lane_rhs_candidates(ctx, with_c2):
    """The pair-lane RHS tiles (two x points per lane) on a box with even rows:
    every shape against the oracle, with and without c^2, and bit for bit
    against the one-point tiles; fields whose interior rows are not 16-byte
    aligned run the same shape on the one-point tiles."""
    n, g = (64, 40, 24), 2
    dx = (1 / 64, 1 / 40, 1 / 24)
    a = O.fill_ghosts_periodic(rand_box(n, g, 12, 1), g)
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(12, 2, n[::-1]), g) if with_c2 else None
    u = dev_full(a, g)
    c2d = dev(c2, g) if with_c2 else None
    b = S.box_of(u, g, dx)
    want = O.wave_rhs(a, g, dx, c2)
    kinds = cands_by_kind(ctx, S.S4_OP_WAVE_RHS, b)
    assert len(kinds["pairs"]) == 12
    ref = None
    for cand in [kinds["tiles"][1]] + kinds["pairs"]:
        out = S.alloc_field(n, g, fill=NAN)
        S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, b, cand)
        S.s4_wave_rhs(ctx, b, [u], None if c2d is None else [c2d], [out])
        got = host(out)
        assert rel(got, want, g) <= TOL, f"candidate {cand}"
        assert ghosts_untouched(got, g)
        if ref is None:
            ref = got
        np.testing.assert_array_equal(inner(got, g), inner(ref, g), err_msg=f"candidate {cand}")
    # misaligned fields: views shifted by one element (8-byte aligned, not 16)
    span = u.stride()[0] * u.shape[0]
    flat = torch.empty(span + 64, dtype=torch.float64, device="cuda")
    shifted = flat[1:].as_strided(u.shape, u.stride())
    shifted.copy_(u)
    outs = torch.full_like(flat, NAN)[1:].as_strided(u.shape, u.stride())
    bs = S.box_of(shifted, g, dx)
    S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, bs, kinds["pairs"][0])
    c2s = None
    if with_c2:
        cflat = torch.full_like(flat, NAN)
        c2s = cflat[1:].as_strided(u.shape, u.stride())
        c2s.copy_(c2d)
    S.s4_wave_rhs(ctx, bs, [shifted], None if c2s is None else [c2s], [outs])
    np.testing.assert_array_equal(inner(host(outs), g), inner(ref, g))
    S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, b, -1)
    S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, bs, -1)
