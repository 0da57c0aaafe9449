"""The on-line tuner's search (the paper's random-restart hill climbing,
Sec. III-B), driven on the host against synthetic per-candidate costs
through s4_online_simulate: it converges on a smooth landscape, leaves a
local optimum only through random restarts, keeps the cost of its
excursions small, tolerates timing noise and is deterministic per seed."""
import numpy as np

import paper_1308_1343_amd as S

# the library's candidate list, in its order (variant, tx, nw, tz, ry): one kernel per stage
# on the tile traversal, on the row-register traversal, stage pairs per tap, whole steps,
# widened stage pairs, pair-lane tiles (RHS only)
CANDS = [(0, tx, nw, tz, 0) for tx in (64, 32, 16) for nw in (8, 4) for tz in (0, 64, 32, 16, 8)] + \
        [(2, tx, 4, tz, ry) for tx in (256, 128, 64) for ry in (4, 2) for tz in (64, 32, 16)] + \
        [(3, tx, nw, tz, 0) for tx, nw in ((64, 4), (64, 8), (32, 8), (32, 4), (16, 8), (16, 4))
         for tz in (64, 32, 16)] + \
        [(4, tx, nw, tz, 0) for tx, nw in ((64, 16), (32, 16), (32, 8), (68, 16)) for tz in (0, 128, 64, 32, 16)] + \
        [(1, tx, nw, tz, 0) for tx, nw in ((32, 8), (64, 8), (64, 16), (32, 16)) for tz in (64, 32, 16)] + \
        [(5, tx, nw, tz, 0) for tx in (64, 32) for nw in (8, 4) for tz in (64, 32, 16)]
ORD_TX = {16: 0, 32: 1, 64: 2, 68: 2, 128: 3, 256: 4}
ORD_NW = {4: 0, 8: 1, 16: 2}
ORD_TZ = {8: 0, 16: 1, 32: 2, 64: 3, 128: 4, 0: 5}
ORD_RY = {0: 0, 2: 0, 4: 1}
BOX = S.make_box((256, 256, 256), 2, (1, 272, 272 * 260), 1 / 256)


def dist(a, b):
    return (abs(ORD_TX[a[1]] - ORD_TX[b[1]]) + abs(ORD_NW[a[2]] - ORD_NW[b[2]]) + abs(ORD_TZ[a[3]] - ORD_TZ[b[3]]) +
            abs(ORD_RY[a[4]] - ORD_RY[b[4]]) + ((a[1] == 68) != (b[1] == 68)))


def bowl(center, slope=0.05, other_variant=2.0):
    c = CANDS[center]
    return [1.0 + slope * dist(c, d) if d[0] == c[0] else other_variant for d in CANDS]


def test_candidate_table_matches_library():
    tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, [1.0] * len(CANDS), ncalls=3)
    assert all(0 <= t < len(CANDS) for t in tr)
    first = {v: min(k for k, c in enumerate(CANDS) if c[0] == v) for v in (2, 3, 1, 5)}
    rk4_only = set(range(first[3], first[5]))
    tr = S.s4_online_simulate(S.S4_OP_WAVE_RHS, BOX, list(np.linspace(1, 2, len(CANDS))), ncalls=400,
                              restart_prob=0.2)
    assert not rk4_only & set(tr)  # stage pairs and whole steps only for RK4
    assert any(t >= first[5] for t in tr)  # the RHS reaches its pair-lane tiles
    tr = S.s4_online_simulate(S.S4_OP_ADJOINT_STEP, BOX, list(np.linspace(1, 2, len(CANDS))), ncalls=400,
                              restart_prob=0.2)
    assert max(tr) < first[2]  # row kernels only for the RHS and RK4
    tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, list(np.linspace(1, 2, len(CANDS))), ncalls=400, restart_prob=0.2)
    assert max(tr) < first[5]  # pair-lane tiles only for the RHS
    tr = S.s4_online_simulate(S.S4_OP_RK4, [BOX, BOX], list(np.linspace(1, 2, len(CANDS))), ncalls=400,
                              restart_prob=0.2)
    assert max(tr) < first[1]  # widened stage pairs only on one box


def test_converges_on_a_smooth_landscape():
    target = CANDS.index((0, 16, 4, 32, 0))
    cost = bowl(target)
    tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=0.0, ncalls=120)
    assert tr[0] != target
    assert all(t == target for t in tr[-30:])
    # hill climbing: it walks, it does not enumerate all candidates
    assert len(set(tr)) < 30


def test_restarts_escape_a_local_optimum():
    start = S.s4_online_simulate(S.S4_OP_RK4, BOX, [1.0] * len(CANDS), ncalls=1)[0]
    glob = CANDS.index((1, 32, 16, 16, 0))
    cost = [1.5] * len(CANDS)
    cost[start] = 1.0  # an isolated local optimum at the starting setting
    for i, d in enumerate(CANDS):  # a good basin around the global optimum
        if d[0] == 1 and dist(d, CANDS[glob]) <= 1:
            cost[i] = 0.75
    cost[glob] = 0.7
    stuck = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=0.0, ncalls=500)
    assert all(t == start for t in stuck[-100:])
    tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=0.05, seed=3, ncalls=3000)
    assert np.mean([t == glob for t in tr[-300:]]) > 0.85


def test_excursions_are_cheap():
    # An excursion starts with probability restart_prob per call and is
    # abandoned at its first trial slower than 1.5x the best, so on average
    # it costs about two calls at the worst setting's price: the steady
    # overhead stays below 2 * restart_prob * (worst / best - 1), 8 % here.
    target = CANDS.index((1, 64, 16, 64, 0))
    cost = bowl(target, slope=0.3, other_variant=3.0)
    p = 0.02
    bound = 1.0 + 2 * p * (max(cost) / cost[target] - 1.0)
    for seed in (5, 6, 7):
        tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=p, seed=seed, ncalls=4000)
        steady = np.mean([cost[t] for t in tr[-2000:]])
        assert steady <= bound * cost[target], (seed, steady)


def test_noise_tolerance_and_determinism():
    target = CANDS.index((0, 32, 8, 16, 0))
    cost = bowl(target, slope=0.1)
    a = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, noise=0.03, restart_prob=0.01, seed=7, ncalls=600)
    b = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, noise=0.03, restart_prob=0.01, seed=7, ncalls=600)
    assert a == b
    final = max(set(a[-100:]), key=a[-100:].count)
    assert cost[final] <= 1.05 * cost[target]


def test_simulation_rejects_bad_arguments():
    import pytest
    with pytest.raises(S.Sten4Error):
        S.s4_online_simulate(S.S4_OP_RK4, BOX, [1.0] * 5, ncalls=3)
    with pytest.raises(S.Sten4Error):
        S.s4_online_simulate(S.S4_OP_RK4, BOX, [1.0] * len(CANDS), noise=2.0, ncalls=3)


def test_moves_between_kernel_sets():
    """A per-stage basin whose best z chunk (8) has no fused-pair counterpart
    must still lead to a better fused-pair setting without random restarts,
    past two kernel sets that are worse everywhere."""
    stage_best, pair_best = (0, 32, 8, 8, 0), (1, 32, 16, 16, 0)
    cost = [(1.0 + 0.05 * dist(d, stage_best)) if d[0] == 0 else (0.85 + 0.05 * dist(d, pair_best)) if d[0] == 1
            else 2.0 for d in CANDS]
    tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=0.0, ncalls=200)
    assert all(CANDS[t] == pair_best for t in tr[-30:])


def test_reaches_every_kernel_set():
    """From the per-stage start the neighbourhood reaches the best setting of
    whichever kernel set holds it, without random restarts."""
    for best in ((3, 64, 4, 32, 0), (2, 256, 4, 32, 4), (1, 64, 16, 64, 0), (4, 64, 16, 32, 0)):
        cost = [0.6 + 0.05 * dist(d, best) if d[0] == best[0] else 1.0 + 0.01 * dist(d, (0, 64, 8, 32, 0))
                for d in CANDS]
        tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=0.0, ncalls=300)
        assert all(CANDS[t] == best for t in tr[-30:]), best


def test_whole_steps_skipped_for_huge_planes():
    """Boxes whose z planes reach 2 GiB never get a whole-step setting (those
    kernels address one plane with 31-bit byte offsets), even when it would be
    the fastest; ordinary boxes reach it."""
    huge = S.make_box((16384, 16384, 4), 2, (1, 16400, 16400 * 16388), 1.0)
    cost = [0.5 if d[0] == 4 else 1.0 + 0.01 * i for i, d in enumerate(CANDS)]
    tr = S.s4_online_simulate(S.S4_OP_RK4, huge, cost, restart_prob=0.3, ncalls=400)
    assert all(CANDS[t][0] != 4 for t in tr)
    tr = S.s4_online_simulate(S.S4_OP_RK4, BOX, cost, restart_prob=0.3, ncalls=400)
    # (restarts take 30 % of the calls here: the search's home is what counts)
    assert sum(CANDS[t][0] == 4 for t in tr[-100:]) > 50


def cube(n):
    return S.make_box((n, n, n), 2, (1, n + 4, (n + 4) * (n + 4)), 1.0 / n)


def start_of(op, box):
    return CANDS[S.s4_online_simulate(op, box, [1.0] * len(CANDS), restart_prob=0.0, ncalls=1)[0]]


def test_whole_step_start_follows_the_cost_model():
    """The untuned whole-step setting of one periodic box (the search's start):
    equal 8-plane runs on 32 x 16 lanes for boxes too small to fill the GPU,
    else the shape and work order the cost model rates cheapest -- 28 x 28
    output tiles in equal runs where the box divides into them (224^3,
    448^3), 64 x 11 tiles of 68-point rows where 64 divides the side (256^3,
    320^3, 384^3, 512^3), 60 x 12 tiles in equal runs on 192^3 and 272^3 (on
    the cubes of side 128, 192, 224, 256, 320, 384, 448 and 512 these are the
    fastest measured settings)."""
    want = {64: (4, 32, 8, 0, 0), 128: (4, 32, 8, 16, 0), 160: (4, 32, 8, 32, 0), 192: (4, 64, 16, 0, 0),
            224: (4, 32, 16, 0, 0), 256: (4, 68, 16, 32, 0), 272: (4, 64, 16, 0, 0), 320: (4, 68, 16, 64, 0),
            384: (4, 68, 16, 64, 0), 448: (4, 32, 16, 0, 0), 512: (4, 68, 16, 64, 0)}
    for n, w in want.items():
        assert start_of(S.S4_OP_RK4, cube(n)) == w, n
    # a set of boxes keeps 32-plane chunks on 32 x 16 lanes
    assert CANDS[S.s4_online_simulate(S.S4_OP_RK4, [cube(64), cube(96)], [1.0] * len(CANDS), restart_prob=0.0,
                                      ncalls=1)[0]] == (4, 32, 8, 32, 0)


def test_mixed_kernel_start():
    """The multi-field kernel starts on 32 x 8 lanes (16 x 16 for boxes narrower
    than 24) with the longest z chunk giving every CU one item per field, and
    8-plane chunks where none does."""
    assert start_of(S.S4_OP_DERIV_MIXED, cube(192)) == (0, 32, 4, 64, 0)
    assert start_of(S.S4_OP_DERIV_MIXED, cube(128)) == (0, 32, 4, 32, 0)
    assert start_of(S.S4_OP_DERIV_MIXED, cube(112)) == (0, 32, 4, 16, 0)
    assert start_of(S.S4_OP_DERIV_MIXED, cube(64)) == (0, 32, 4, 8, 0)
    assert start_of(S.S4_OP_DERIV_MIXED, cube(20)) == (0, 16, 4, 8, 0)


def test_search_skips_settings_that_starve_the_device():
    """On a 128^3 box the search never visits a setting whose launch hands
    fewer work items than a quarter of the CUs (e.g. per-stage kernels with
    whole-box z chunks of 64 x 8 tiles: 32 items) while other settings give
    every CU one, even where it would be the cheapest and restarts are
    frequent; such settings stay reachable on boxes that no setting fills."""
    b = cube(128)
    starving = CANDS.index((0, 64, 8, 0, 0))
    cost = [0.5 if i == starving else 1.0 + 0.001 * i for i in range(len(CANDS))]
    tr = S.s4_online_simulate(S.S4_OP_RK4, b, cost, restart_prob=0.5, ncalls=600)
    assert starving not in tr
    tiny = cube(16)  # 1 tile: no setting fills the device
    tr = S.s4_online_simulate(S.S4_OP_RK4, tiny, cost, restart_prob=0.5, ncalls=600)
    assert starving in tr
