"""Same-level ghost exchange and RK4 on a level of boxes that tile a periodic
domain, against the oracle: every exchanged ghost point bit for bit against
the brute-force source map, untouched points left alone, and the level's
RK4 against the oracle's RK4 on one box spanning the whole domain (and bit
for bit against the library's own single-box RK4 on that box)."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.bboxset as B
import paper_1308_1343_amd as S
import workload as W
from _gpu import NAN, host

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    return S.Context(0)


def level_of(d, keep=None, domain=None, width=2, shape="faces", fields=()):
    """Level handle, device fields (one list per global array in `fields`) and the
    kept box records.  Interiors hold the global arrays' slices, ghosts NaN."""
    g = d["ghost"]
    idx = list(range(len(d["boxes"]))) if keep is None else keep
    recs = [d["boxes"][i] for i in idx]
    out = []
    for arr in fields:
        fs = []
        for b in recs:
            t = S.alloc_field(b["n"], g, fill=NAN)
            S.interior(t, g).copy_(torch.from_numpy(np.ascontiguousarray(arr[W.box_slice(b)])))
            fs.append(t)
        out.append(fs)
    boxes = [S.box_of(t, g, d["dx"]) for t in (out[0] if out else
                                               [S.alloc_field(b["n"], g) for b in recs])]
    dom = d["domain"] if domain is None else domain
    L = S.s4_level_create(boxes, [b["lo"] for b in recs], dom, width, shape)
    return L, boxes, out, recs


def check_exchange(fs, recs, glob, g, domain, width, shape):
    src = B.sync_sources([b["lo"] for b in recs], [b["n"] for b in recs], g, domain, width, shape)
    for k, (t, b) in enumerate(zip(fs, recs)):
        h = host(t)                              # (z, y, x) ghosted
        pts, who, sp = src[k]
        ix = (pts[:, 2] + g, pts[:, 1] + g, pts[:, 0] + g)
        got = h[ix]
        cov = who >= 0
        lo_o = np.asarray([recs[w]["lo"] for w in who[cov]]).reshape(-1, 3)
        gp = lo_o + sp[cov]                      # global (x, y, z) of the source
        want = glob[gp[:, 2], gp[:, 1], gp[:, 0]]
        assert np.array_equal(got[cov].view(np.int64), want.view(np.int64)), f"box {k}: wrong ghost values"
        assert np.isnan(got[~cov]).all(), f"box {k}: an uncovered ghost point was written"
        m = np.zeros(h.shape, bool)
        m[ix] = True
        m[g:-g, g:-g, g:-g] = True
        assert np.isnan(h[~m]).all(), f"box {k}: a ghost point outside the exchange was written"
        assert np.array_equal(h[g:-g, g:-g, g:-g], glob[W.box_slice(b)]), f"box {k}: interior changed"


SMALL = dict(counts=(3, 3, 2), smin=6, smax=20)


@pytest.mark.parametrize("shape,width", [("faces", 2), ("full", 3), ("full", 1), ("faces", 3)])
def test_exchange_tiled_level(ctx, shape, width):
    d = W.level_tiling(**SMALL)
    L, boxes, (fs,), recs = level_of(d, width=width, shape=shape, fields=(d["u"],))
    S.s4_level_sync(ctx, L, fs)
    check_exchange(fs, recs, d["u"], d["ghost"], d["domain"], width, shape)


@pytest.mark.parametrize("mask", [(1, 1, 1), (0, 1, 1), (0, 0, 0)])
def test_exchange_partial_level(ctx, mask):
    d = W.level_tiling(**SMALL)
    keep = [i for i in range(len(d["boxes"])) if i % 3 != 1]
    dom = tuple(v * m for v, m in zip(d["domain"], mask))
    L, boxes, (fs,), recs = level_of(d, keep=keep, domain=dom, width=2, shape="full", fields=(d["u"],))
    assert S.s4_level_info(L)["uncovered"] > 0
    S.s4_level_sync(ctx, L, fs)
    check_exchange(fs, recs, d["u"], d["ghost"], dom, 2, "full")


def test_exchange_full_size_level(ctx):
    d = W.level_tiling()
    L, boxes, (fs,), recs = level_of(d, width=2, shape="faces", fields=(d["u"],))
    ws = S.s4_level_sync(ctx, L, fs)
    S.s4_level_sync(ctx, L, fs, ws=ws)           # again, reusing the workspace: same result
    check_exchange(fs, recs, d["u"], d["ghost"], d["domain"], 2, "faces")


def level_rk4_case(ctx, d, nsteps, mode, c2glob=None, shape="faces"):
    fields = (d["u"], d["rho"]) + ((c2glob,) if c2glob is not None else ())
    L, boxes, fl, recs = level_of(d, width=2, shape=shape, fields=fields)
    u, r = fl[0], fl[1]
    c2 = fl[2] if c2glob is not None else None
    S.s4_level_rk4(ctx, L, u, r, c2, d["dt"], nsteps, mode)
    return [host(t) for t in u], [host(t) for t in r], recs


def oracle_level(d, nsteps, c2glob=None):
    g = 2
    c2 = O.embed(c2glob, g) if c2glob is not None else None
    return O.rk4(O.embed(d["u"], g), O.embed(d["rho"], g), g, d["dx"], d["dt"], nsteps, c2=c2)


def compare(level_u, level_r, recs, ou, orho, gl=3, go=2):
    ou_i, or_i = O.interior(ou, go), O.interior(orho, go)
    su, sr = max(np.abs(ou_i).max(), 1e-300), max(np.abs(or_i).max(), 1e-300)
    eu = er = 0.0
    for hu, hr, b in zip(level_u, level_r, recs):
        sl = W.box_slice(b)
        eu = max(eu, np.abs(hu[gl:-gl, gl:-gl, gl:-gl] - ou_i[sl]).max() / su)
        er = max(er, np.abs(hr[gl:-gl, gl:-gl, gl:-gl] - or_i[sl]).max() / sr)
    return eu, er


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
def test_level_rk4_vs_oracle(ctx, mode):
    d = W.level_tiling(**SMALL)
    lu, lr, recs = level_rk4_case(ctx, d, 4, mode)
    ou, orho = oracle_level(d, 4)
    eu, er = compare(lu, lr, recs, ou, orho)
    assert eu <= TOL and er <= TOL, (eu, er)


def test_level_rk4_variable_c2_full_shape(ctx):
    d = W.level_tiling(**SMALL)
    c2 = 0.5 + W.uniform01(d["seed"], 9, d["u"].shape)
    lu, lr, recs = level_rk4_case(ctx, d, 3, "graph", c2glob=c2, shape="full")
    ou, orho = oracle_level(d, 3, c2glob=c2)
    eu, er = compare(lu, lr, recs, ou, orho)
    assert eu <= TOL and er <= TOL, (eu, er)


def test_level_rk4_equals_single_box_bitwise(ctx):
    """The level's boxes compute every point exactly as one box over the whole domain does."""
    d = W.level_tiling(**SMALL)
    lu, lr, recs = level_rk4_case(ctx, d, 5, "batched")
    n = d["domain"]
    u = S.alloc_field(n, 2, fill=0.0)
    r = S.alloc_field(n, 2, fill=0.0)
    S.interior(u, 2).copy_(torch.from_numpy(d["u"]))
    S.interior(r, 2).copy_(torch.from_numpy(d["rho"]))
    S.s4_rk4(ctx, S.box_of(u, 2, d["dx"]), [u], [r], None, d["dt"], 5, "perbox")
    gu, gr = S.interior(u, 2).cpu().numpy(), S.interior(r, 2).cpu().numpy()
    for hu, hr, b in zip(lu, lr, recs):
        np.testing.assert_array_equal(hu[3:-3, 3:-3, 3:-3], gu[W.box_slice(b)])
        np.testing.assert_array_equal(hr[3:-3, 3:-3, 3:-3], gr[W.box_slice(b)])


def test_level_rk4_graph_replays(ctx):
    """A captured step replayed across calls (cache hit) equals per-box launches."""
    d = W.level_tiling(**SMALL)
    L, boxes, (u, r), recs = level_of(d, fields=(d["u"], d["rho"]))
    ws = S.s4_level_rk4(ctx, L, u, r, None, d["dt"], 2, "graph")
    torch.cuda.synchronize()
    S.s4_level_rk4(ctx, L, u, r, None, d["dt"], 3, "graph", ws=ws)
    L2, _, (u2, r2), _ = level_of(d, fields=(d["u"], d["rho"]))
    S.s4_level_rk4(ctx, L2, u2, r2, None, d["dt"], 5, "perbox")
    for a, b in zip(u + r, u2 + r2):
        np.testing.assert_array_equal(S.interior(a, 3).cpu().numpy(), S.interior(b, 3).cpu().numpy())


def test_level60_rk4_vs_oracle(ctx):
    """The 60-box level (280 x 224 x 168 periodic domain), in the benchmark's graph mode."""
    d = W.level_tiling()
    lu, lr, recs = level_rk4_case(ctx, d, 2, "graph")
    ou, orho = oracle_level(d, 2)
    eu, er = compare(lu, lr, recs, ou, orho)
    assert eu <= TOL and er <= TOL, (eu, er)


def test_level_rk4_rejects_uncovered_and_narrow(ctx):
    d = W.level_tiling(**SMALL)
    keep = [i for i in range(len(d["boxes"])) if i != 4]
    L, boxes, (u, r), _ = level_of(d, keep=keep, fields=(d["u"], d["rho"]))
    with pytest.raises(S.Sten4Error) as e:
        S.s4_level_rk4(ctx, L, u, r, None, d["dt"], 1, "perbox")
    assert e.value.code == S.S4_EGHOST
    L1, _, (u1, r1), _ = level_of(d, width=1, fields=(d["u"], d["rho"]))
    with pytest.raises(S.Sten4Error) as e:
        S.s4_level_rk4(ctx, L1, u1, r1, None, d["dt"], 1, "perbox")
    assert e.value.code == S.S4_EGHOST


def test_level_sync_argument_errors(ctx):
    d = W.level_tiling(**SMALL)
    L, boxes, (fs,), _ = level_of(d, fields=(d["u"],))
    need = S.s4_level_workspace_size(L, S.S4_OP_LEVEL_SYNC)
    with pytest.raises(S.Sten4Error) as e:
        S.s4_level_sync(ctx, L, fs, ws=S.workspace(need - 256))
    assert e.value.code == S.S4_ENOMEM
    with pytest.raises(S.Sten4Error) as e:
        S.s4_level_sync(ctx, L, [fs[0]] * len(fs))
    assert e.value.code == S.S4_EALIAS


def test_level_choice_after_tuning(ctx):
    """s4_tune on a level's boxes keeps, besides the fastest setting, the fastest
    level-capable one, which the level then runs (reported by s4_level_choice)."""
    d = W.level_tiling(**SMALL)
    L, boxes, (u, r), _ = level_of(d, fields=(d["u"], d["rho"]))
    tctx = S.Context(0)
    S.s4_tune(tctx, S.S4_OP_RK4, boxes, flags=0)
    bc, lc = S.s4_get_choice(tctx, S.S4_OP_RK4, boxes), S.s4_level_choice(tctx, L)
    assert bc["tuned"] == 1 and lc["tuned"] == 1
    assert lc["kernel_op"] not in (100, 102)
    if bc["kernel_op"] not in (100, 102):
        assert lc["candidate"] == bc["candidate"]
    S.s4_level_rk4(tctx, L, u, r, None, d["dt"], 2, "graph")
    # interiors only: ghost points the face exchange does not fill keep their NaN canaries
    assert all(bool(torch.isfinite(t[3:-3, 3:-3, 3:-3]).all()) for t in u + r)


def test_level_refuses_whole_steps(ctx):
    """A whole-step choice for the boxes (radius-4 widened tiles) is replaced on a
    level by a level-capable one, and the level's result is unchanged by it."""
    from _gpu import cands_by_kind
    d = W.level_tiling(**SMALL)
    L, boxes, (u, r), _ = level_of(d, fields=(d["u"], d["rho"]))
    S.s4_level_rk4(ctx, L, u, r, None, d["dt"], 2, "batched")
    ref = [host(t) for t in u + r]
    whole = [c for c in cands_by_kind(ctx, S.S4_OP_RK4, boxes)["fused"]
             if (S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, c) or True)
             and S.s4_get_choice(ctx, S.S4_OP_RK4, boxes)["kernel_op"] == 102]
    assert whole
    for c in (whole[0], whole[-1]):
        L, boxes, (u, r), _ = level_of(d, fields=(d["u"], d["rho"]))
        S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, c)
        assert S.s4_get_choice(ctx, S.S4_OP_RK4, boxes)["kernel_op"] == 102
        lc = S.s4_level_choice(ctx, L)
        assert lc["kernel_op"] not in (100, 102) and lc["candidate"] != c
        S.s4_level_rk4(ctx, L, u, r, None, d["dt"], 2, "batched")
        for a, b_ in zip([host(t) for t in u + r], ref):
            np.testing.assert_array_equal(a[3:-3, 3:-3, 3:-3], b_[3:-3, 3:-3, 3:-3])
    S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, -1)


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
@pytest.mark.parametrize("kind,nsteps", [("rows", 3), ("fused", 3), ("fused", 4)])
def test_level_rk4_kernel_sets_bitwise(ctx, mode, kind, nsteps):
    """The row-register stage kernels and the stage pairs, with ghost addressing and the
    exchanges they need, give the per-stage tile kernels' result bit for bit."""
    from _gpu import cands_by_kind
    d = W.level_tiling(**SMALL)
    L, boxes, (u, r), _ = level_of(d, fields=(d["u"], d["rho"]))
    S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, 2)
    S.s4_level_rk4(ctx, L, u, r, None, d["dt"], nsteps, mode)
    S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, -1)
    ref_u, ref_r = [host(t) for t in u], [host(t) for t in r]
    cl = cands_by_kind(ctx, S.S4_OP_RK4, boxes)[kind]
    if kind == "fused":  # the per-tap stage pairs; whole steps cannot run on a level
        cl = [c for c in cl if (S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, c) or True)
              and S.s4_get_choice(ctx, S.S4_OP_RK4, boxes)["kernel_op"] == 101]
        S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, -1)
    for cand in (cl[0], cl[len(cl) // 2], cl[-1]):
        L, boxes, (u, r), _ = level_of(d, fields=(d["u"], d["rho"]))
        S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, cand)
        assert S.s4_level_choice(ctx, L)["candidate"] == cand
        S.s4_level_rk4(ctx, L, u, r, None, d["dt"], nsteps, mode)
        for a, b_ in zip([host(t) for t in u] + [host(t) for t in r], ref_u + ref_r):
            np.testing.assert_array_equal(a[3:-3, 3:-3, 3:-3], b_[3:-3, 3:-3, 3:-3], err_msg=f"candidate {cand}")
        S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, -1)


# ---------------------------------------------------------------------------
# wide levels: a full-shell exchange of width 4 over boxes with 4 ghost layers
# lets a whole RK4 step read its radius-4 neighbourhood from the ghost zones

def wide_level_case(ctx, d, nsteps, mode, cand=None, c2glob=None):
    fields = (d["u"], d["rho"]) + ((c2glob,) if c2glob is not None else ())
    L, boxes, fl, recs = level_of(d, width=4, shape="full", fields=fields)
    if cand is not None:
        S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, cand)
    ch = S.s4_level_choice(ctx, L)
    S.s4_level_rk4(ctx, L, fl[0], fl[1], fl[2] if c2glob is not None else None, d["dt"], nsteps, mode)
    if cand is not None:
        S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, -1)
    return [host(t) for t in fl[0]], [host(t) for t in fl[1]], recs, ch


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
@pytest.mark.parametrize("nsteps", [3, 4])
def test_wide_level_whole_steps(ctx, mode, nsteps):
    """Whole steps (the default on a wide level) against the oracle, and bit for
    bit against the per-stage kernels on the same level; an odd count ends with
    one per-stage step."""
    d = W.level_tiling(**SMALL, ghost=4)
    lu, lr, recs, ch = wide_level_case(ctx, d, nsteps, mode)
    assert ch["kernel_op"] == 102
    ou, orho = oracle_level(d, nsteps)
    eu, er = compare(lu, lr, recs, ou, orho, gl=4)
    assert eu <= TOL and er <= TOL, (eu, er)
    su, sr, _, ch2 = wide_level_case(ctx, d, nsteps, mode, cand=2)
    assert ch2["candidate"] == 2
    for a, b_ in zip(lu + lr, su + sr):
        np.testing.assert_array_equal(a[4:-4, 4:-4, 4:-4], b_[4:-4, 4:-4, 4:-4])


def test_wide_level_every_whole_step_shape(ctx):
    from _gpu import cands_by_kind
    d = W.level_tiling(**SMALL, ghost=4)
    L, boxes, _, _ = level_of(d, width=4, shape="full", fields=(d["u"],))
    whole = [c for c in cands_by_kind(ctx, S.S4_OP_RK4, boxes)["fused"]
             if (S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, c) or True)
             and S.s4_get_choice(ctx, S.S4_OP_RK4, boxes)["kernel_op"] == 102]
    S.s4_set_choice(ctx, S.S4_OP_RK4, boxes, -1)
    ref = None
    for c in whole:
        lu, lr, _, ch = wide_level_case(ctx, d, 2, "batched", cand=c)
        assert ch["candidate"] == c
        if ref is None:
            ref = (lu, lr)
        for a, b_ in zip(lu + lr, ref[0] + ref[1]):
            np.testing.assert_array_equal(a[4:-4, 4:-4, 4:-4], b_[4:-4, 4:-4, 4:-4], err_msg=f"candidate {c}")


def test_wide_level_variable_c2(ctx):
    d = W.level_tiling(**SMALL, ghost=4)
    c2 = 0.5 + W.uniform01(d["seed"], 9, d["u"].shape)
    lu, lr, recs, ch = wide_level_case(ctx, d, 4, "graph", c2glob=c2)
    assert ch["kernel_op"] == 102
    ou, orho = oracle_level(d, 4, c2glob=c2)
    eu, er = compare(lu, lr, recs, ou, orho, gl=4)
    assert eu <= TOL and er <= TOL, (eu, er)


def test_level60_wide_whole_steps_vs_oracle(ctx):
    """The 60-box level with 4 ghost layers and a full exchange of width 4, in
    the benchmark's graph mode, against the oracle."""
    d = W.level_tiling(ghost=4)
    lu, lr, recs, ch = wide_level_case(ctx, d, 2, "graph")
    assert ch["kernel_op"] == 102
    ou, orho = oracle_level(d, 2)
    eu, er = compare(lu, lr, recs, ou, orho, gl=4)
    assert eu <= TOL and er <= TOL, (eu, er)
