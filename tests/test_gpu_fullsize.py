"""Full-size workloads, in the launch configuration the benchmark times:
256^3 wave RK4 for all 100 steps against the oracle, the pure-mode closed
form at 256^3, the 60-box bboxset steps in all three launch modes, and
large single cubes in their untuned setting."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1308_1343_amd as S
import workload as W
from _gpu import cands_by_kind, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return S.Context(0)


def to_dev(a, n, g, fill=0.0):
    t = S.alloc_field(n, g, fill=fill)
    S.interior(t, g).copy_(torch.from_numpy(a))
    return t


def test_wave256_rk4_100_steps_vs_oracle(ctx):
    d = W.wave256()
    g, n = d["ghost"], d["n"]
    u, r = to_dev(d["u"], n, g), to_dev(d["rho"], n, g)
    b = S.box_of(u, g, d["dx"])
    S.s4_rk4(ctx, b, [u], [r], None, d["dt"], d["nsteps"], "graph")
    wu, wr = O.rk4(O.embed(d["u"], g), O.embed(d["rho"], g), g, d["dx"], d["dt"], d["nsteps"])
    assert rel(host(u), wu, g) <= 1e-12
    assert rel(host(r), wr, g) <= 1e-12


def find_cand(ctx, op, b, kind, tile_x, threads, z_chunk):
    """Index of the candidate with these parameters (as s4_get_choice reports
    them); kind "tiles" (the tile traversal: kernel op below 100), "pairs"
    (pair-lane tiles: 300 and up) or "whole" (the whole-step kernels: 102)."""
    nc = S.s4_get_choice(ctx, op, b)["ncandidates"]
    try:
        for c in range(nc):
            try:
                S.s4_set_choice(ctx, op, b, c)
            except S.Sten4Error:
                continue  # a kernel set this op does not use
            ch = S.s4_get_choice(ctx, op, b)
            k = ch["kernel_op"]
            want = k < 100 if kind == "tiles" else k >= 300 if kind == "pairs" else k == 102
            if want and \
                    (ch["tile_x"], ch["threads"], ch["z_chunk"]) == (tile_x, threads, z_chunk):
                return c
    finally:
        S.s4_set_choice(ctx, op, b, -1)
    raise AssertionError(f"no candidate {kind, tile_x, threads, z_chunk}")


def test_wave256_rhs_benchmarked_tile_vs_oracle(ctx):
    """The 256^3 RHS in the tile the sweep picks for the benchmark (pair-lane
    tiles of 64 x 8 points on 256 lanes, 64-plane chunks) and in every other
    RHS candidate, against the oracle and bit for bit against each other."""
    d = W.wave256()
    g, n = d["ghost"], d["n"]
    uf = O.fill_ghosts_periodic(O.embed(d["u"], g), g)
    u = S.alloc_field(n, g, fill=float("nan"))
    u.copy_(torch.from_numpy(uf))
    b = S.box_of(u, g, d["dx"])
    want = O.wave_rhs(uf, g, d["dx"])
    tuned = find_cand(ctx, S.S4_OP_WAVE_RHS, b, "pairs", 64, 256, 64)
    k = cands_by_kind(ctx, S.S4_OP_WAVE_RHS, b)
    ref = None
    for cand in [tuned] + [c for c in k["tiles"] + k["rows"] + k["pairs"] if c != tuned]:
        out = S.alloc_field(n, g, fill=float("nan"))
        S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, b, cand)
        S.s4_wave_rhs(ctx, b, [u], None, [out])
        got = host(out)
        assert rel(got, want, g) <= 1e-12, f"candidate {cand}"
        if ref is None:
            ref = got
        else:
            np.testing.assert_array_equal(got[g:-g, g:-g, g:-g], ref[g:-g, g:-g, g:-g], err_msg=f"candidate {cand}")
    S.s4_set_choice(ctx, S.S4_OP_WAVE_RHS, b, -1)


@pytest.mark.parametrize("tile_x,z_chunk", [(68, 32), (64, 128)])
def test_wave256_rk4_c2_benchmarked_setting_vs_oracle(ctx, tile_x, z_chunk):
    """The 256^3 RK4 with variable c^2 in the settings its sweep picks for the
    benchmark: whole steps on 68 x 15 lanes in 32-plane chunks, and on 64 x 16
    lanes (loads two planes ahead) in 128-plane chunks; 20 steps against the
    oracle and bit for bit against the per-stage kernels."""
    d = W.wave256()
    g, n = d["ghost"], d["n"]
    c2h = 1.0 + 0.5 * W.uniform_pm1(d["seed"], 99, tuple(n[::-1]))
    u, r = to_dev(d["u"], n, g), to_dev(d["rho"], n, g)
    c2 = to_dev(c2h, n, g, fill=float("nan"))  # read at interior points only
    b = S.box_of(u, g, d["dx"])
    op = S.S4_OP_RK4 | S.S4_WITH_C2
    whole = find_cand(ctx, op, b, "whole", tile_x, 1024, z_chunk)
    S.s4_set_choice(ctx, op, b, whole)
    S.s4_rk4(ctx, b, [u], [r], [c2], d["dt"], 20, "graph")
    S.s4_set_choice(ctx, op, b, -1)
    wu, wr = O.rk4(O.embed(d["u"], g), O.embed(d["rho"], g), g, d["dx"], d["dt"], 20, O.embed(c2h, g, 1.0))
    gu, gr = host(u), host(r)
    assert rel(gu, wu, g) <= 1e-12
    assert rel(gr, wr, g) <= 1e-12
    # the per-stage tile kernels (candidate 2) from the same inputs, bit for bit
    u2, r2 = to_dev(d["u"], n, g), to_dev(d["rho"], n, g)
    S.s4_set_choice(ctx, op, b, 2)
    S.s4_rk4(ctx, b, [u2], [r2], [c2], d["dt"], 20, "graph")
    S.s4_set_choice(ctx, op, b, -1)
    sl = (slice(g, -g),) * 3
    np.testing.assert_array_equal(host(u2)[sl], gu[sl])
    np.testing.assert_array_equal(host(r2)[sl], gr[sl])


def test_wave256_fused_pairs_match_stage_kernels(ctx):
    """Every fused stage-pair and row-register candidate against the per-stage tile kernels, bit for bit, at 256^3."""
    d = W.wave256()
    g, n = d["ghost"], d["n"]
    u, r = to_dev(d["u"], n, g), to_dev(d["rho"], n, g)
    b = S.box_of(u, g, d["dx"])
    kinds = cands_by_kind(ctx, S.S4_OP_RK4, b)
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, 2)
    S.s4_rk4(ctx, b, [u], [r], None, d["dt"], 6, "graph")
    ref = (host(u), host(r))
    for cand in kinds["fused"] + kinds["rows"]:
        u, r = to_dev(d["u"], n, g), to_dev(d["rho"], n, g)
        S.s4_set_choice(ctx, S.S4_OP_RK4, b, cand)
        S.s4_rk4(ctx, b, [u], [r], None, d["dt"], 6, "graph")
        np.testing.assert_array_equal(host(u), ref[0], err_msg=f"candidate {cand}")
        np.testing.assert_array_equal(host(r), ref[1], err_msg=f"candidate {cand}")
    S.s4_set_choice(ctx, S.S4_OP_RK4, b, -1)


def test_wave256_pure_mode_closed_form(ctx):
    """u0 = sin(2 pi x) sin(2 pi y) sin(2 pi z), rho0 = 0: after N steps
    (u, rho) = P^N (1, 0) S with P the RK4 polynomial of dt [[0, 1], [lam, 0]]
    and lam the discrete symbol of the 4th-order Laplacian."""
    n, g, N = 256, 2, 100
    h = 1.0 / n
    dt = 0.25 * h
    th = 2 * math.pi * h
    lam = 3 * (-2 * math.cos(2 * th) + 32 * math.cos(th) - 30) / (12 * h * h)
    Z = dt * np.array([[0.0, 1.0], [lam, 0.0]])
    P = np.eye(2)
    T = np.eye(2)
    for k in range(1, 5):
        T = T @ Z / k
        P = P + T
    PN = np.linalg.matrix_power(P, N)
    Smode = W.sine_mode_111(n)
    u = to_dev(Smode, (n, n, n), g)
    r = to_dev(np.zeros_like(Smode), (n, n, n), g)
    b = S.box_of(u, g, h)
    S.s4_rk4(ctx, b, [u], [r], None, dt, N, "graph")
    su = S.interior(u, g).cpu().numpy()
    sr = S.interior(r, g).cpu().numpy()
    assert np.max(np.abs(su - PN[0, 0] * Smode)) <= 1e-12
    assert np.max(np.abs(sr - PN[1, 0] * Smode)) <= 1e-12 * math.sqrt(-lam)


@pytest.mark.parametrize("nsteps", [1, 2])
def test_bboxset60_step_all_modes_vs_oracle(ctx, nsteps):
    """The 60-box set in its default kernel set (whole steps for even step
    counts, as the benchmark times it; an odd count ends with one per-stage
    step), every launch mode, against the oracle box by box."""
    d = W.bboxset()
    g = d["ghost"]
    res = {}
    for mode in ("perbox", "batched", "graph"):
        us, rs, bs = [], [], []
        for i, bx in enumerate(d["boxes"]):
            u, r = to_dev(d["u"][i], bx["n"], g), to_dev(d["rho"][i], bx["n"], g)
            us.append(u)
            rs.append(r)
            bs.append(S.box_of(u, g, bx["dx"], bx["level"]))
        if mode == "perbox":
            assert S.s4_get_choice(ctx, S.S4_OP_RK4, bs)["kernel_op"] == 102
        S.s4_rk4(ctx, bs, us, rs, None, d["dt"], nsteps, mode)
        res[mode] = ([S.interior(u, g).cpu().numpy() for u in us], [S.interior(r, g).cpu().numpy() for r in rs])
    for mode in ("batched", "graph"):
        for a, b in zip(res[mode][0] + res[mode][1], res["perbox"][0] + res["perbox"][1]):
            np.testing.assert_array_equal(a, b)
    for i, bx in enumerate(d["boxes"]):
        wu, wr = O.rk4(O.embed(d["u"][i], g), O.embed(d["rho"][i], g), g, bx["dx"], d["dt"], nsteps)
        wi = wu[g:-g, g:-g, g:-g]
        ri = wr[g:-g, g:-g, g:-g]
        assert np.max(np.abs(res["graph"][0][i] - wi)) <= 1e-12 * np.max(np.abs(wi))
        assert np.max(np.abs(res["graph"][1][i] - ri)) <= 1e-12 * np.max(np.abs(ri))


@pytest.mark.parametrize("n,shape", [(224, (32, 32)), (272, (64, 16)), (320, (68, 15))])
def test_large_cubes_default_setting_vs_oracle(n, shape):
    """Two steps on single periodic cubes whose untuned whole-step setting is a
    1024-lane shape (28 x 28 output tiles dividing 224^3 exactly, in equal
    runs; 60 x 12 tiles in equal runs at 272^3; 64 x 11 tiles of 68-point
    rows, four idle lanes per workgroup, in 64-plane chunks at 320^3),
    against the oracle."""
    fresh = S.Context(0)
    g, nn = 2, (n, n, n)
    u0, r0 = W.uniform_pm1(7, 1, nn), W.uniform_pm1(7, 2, nn)
    u, r = to_dev(u0, nn, g), to_dev(r0, nn, g)
    b = S.box_of(u, g, 1.0 / n)
    ch = S.s4_get_choice(fresh, S.S4_OP_RK4, b)
    assert ch["kernel_op"] == 102 and (ch["tile_x"], ch["tile_y"]) == shape, ch
    dt = 0.25 / n
    S.s4_rk4(fresh, b, [u], [r], None, dt, 2, "graph")
    wu, wr = O.rk4(O.embed(u0, g), O.embed(r0, g), g, (1.0 / n,) * 3, dt, 2)
    assert rel(host(u), wu, g) <= 1e-12
    assert rel(host(r), wr, g) <= 1e-12
