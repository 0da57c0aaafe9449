#!/usr/bin/env python3
"""Benchmark of the FP64 4th-order stencil hot path on one MI355X.

Headline: classical RK4 of the 3-D scalar wave equation (first-order form)
on one 256^3 periodic box with 2 ghost zones, h = 1/256, dt = h/4, inputs
u = U + Gaussian pulse (sigma 0.1), rho = U with U uniform in [-1, 1)
(seeded splitmix64).  A step is one RK4 step, captured once in a hipGraph
and replayed, with the kernel set the tuner picks: one whole-step kernel,
two fused stage-pair kernels, or four stage kernels (Laplacian + stage
update + running sum, periodic addressing).  value = interior points x RK4
steps / s.

The same JSON line also reports, each on its own workload:
  tuning   the RK4 tile choice from the heuristic, from the library's on-line
           random-restart hill climber after 60 calls, and from the sweep
  rhs      one 4th-order Laplacian RHS on the 256^3 box (ghosts read), with
           four rotating buffer sets so no pass finds its data in the
           256 MB last-level cache
  latency32  microseconds per RHS and per RK4 step on the cache-resident
           32^3 box
  copy     a streaming copy of 1 GiB (achievable HBM bandwidth: one 16-byte
           vector per lane in a single pass)
  batched  one RK4 step over a 60-box, 3-level bboxset (sides 16..96, 3
           ghosts) in per-box launches, one persistent batched launch per
           stage, and the batched step replayed as a hipGraph
  level    60 boxes (sides 16..96, 3 ghosts) tiling a 280 x 224 x 168
           periodic domain as one refinement level: the host build of the
           ghost-exchange schedule with derivative bboxsets, one exchange,
           and RK4 steps with an exchange before every stage in the three
           launch modes, beside one box spanning the same domain
  adjoint  loss and gradient through 50 RK4 steps on a 128^3 box with
           variable c^2, checkpoint every 10 steps
and, on rank 0 at N=1, the CPU oracle: it runs the headline's warm-up and
timed steps from the same inputs, its final state is compared with the timed
GPU outputs (max_rel_err, max-norm relative error over interior points of u
and rho; the run fails above 1e-12), and its time, continued to about 20 s
of CPU work, is the cpu_baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpoint-updates/s + % HBM peak, 4th-order 3D stencil RHS; batched & adjoint"
HBM_PEAK_GBS = 8000.0
# FP64 operations per field point issued by the mixed kernel (fma counted as 2):
# D1_x, D1_y, D1_z 5 each; the x, y, z tap sums of D2 4 each and their
# weighting with the centre tap 7; D1_x on halo rows 5 * 4/TY (2.5 at TY = 8);
# D_xy 5; D1_x f + D1_y f 1 and its z derivative (D_xz + D_yz) 5; quadratic
# form 14; sums 3
MIXED_FLOPS_PER_FIELD_POINT = 64.5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("s4_kernels.hip", "s4_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1308_1343_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def kernel_set(ch):
    """Name of the kernel set behind a tile choice (s4_get_choice's kernel op)."""
    k = ch["kernel_op"]
    return ("stage pairs" if k == 100 else "stage pairs per tap" if k == 101 else "whole steps" if k == 102
            else "pair-lane tiles" if k >= 300 else "rows" if k >= 200 else "tiles")


def kernels_per_step(ch, nbox, level=False):
    """Kernel launches of one RK4 step on nbox boxes, per launch mode, for the
    kernel set of tile choice ch: whole steps 1 per box (1 batched), stage
    pairs 2, per-stage sets 4; on a level every pass is preceded by one
    exchange launch (all boxes).  A graph replays the batched launches as one
    graph launch per step."""
    k = ch["kernel_op"]
    per = 1 if k == 102 else 2 if k in (100, 101) else 4
    sync = per if level else 0
    return {"perbox": per * nbox + sync, "batched": per + sync, "graph_kernels": per + sync, "graph_launches": 1}


def traffic_from_profile(kernel_key, tile):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source with the same tile choice; else None.  An
    entry is one record, or a list of records (one per tile the sweep
    ran)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    entries = t.get(kernel_key)
    if isinstance(entries, dict):
        entries = [entries]
    for e in entries or []:
        if e.get("source_hash") == kernel_source_hash() and list(e.get("tile") or []) == list(tile):
            return e.get("bytes_per_launch")
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sections", default="rk4,tuning,rhs,latency32,rk4c2,copy,mixed,batched,level,adjoint,cpu")
    ap.add_argument("--no-tune", action="store_true", help="skip the tile sweep (heuristic or cached choice)")
    ap.add_argument("--tune-cache", default=None, help="JSON file of tuned tile choices to load and update")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    sections = set(args.sections.split(","))

    import numpy as np
    import torch

    import paper_1308_1343_amd as S
    import workload as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.tune_cache:
        os.environ["S4_TUNE_CACHE"] = args.tune_cache
    ctx = S.Context(0)
    K, WU = args.steps, args.warmup
    out = {}

    # ------------------------------------------------------------------ RK4 256^3 (headline)
    d = W.wave256()
    g = d["ghost"]
    n = d["n"]
    npts = n[0] * n[1] * n[2]

    def to_dev(a):
        t = S.alloc_field(n, g, fill=0.0)
        S.interior(t, g).copy_(torch.from_numpy(a))
        return t

    # the timed state and its workspace are allocated (and touched) before
    # the tile sweep, so the timed steps run on memory already in use
    u, rho = to_dev(d["u"]), to_dev(d["rho"])
    box = S.box_of(u, g, d["dx"])
    ws = S.workspace(S.s4_workspace_size(box, S.S4_OP_RK4, S.S4_GRAPH))
    ws.zero_()
    tuned = {}
    if not args.no_tune:
        # the library's tile sweep for each loop setup timed below (run before any timing)
        t0 = time.perf_counter()
        for op in (S.S4_OP_RK4, S.S4_OP_WAVE_RHS):
            S.s4_tune(ctx, op, box, flags=1)
        tuned["wave256_s"] = round(time.perf_counter() - t0, 3)
    choice = S.s4_get_choice(ctx, S.S4_OP_RK4, box)
    stream = torch.cuda.current_stream()
    log(f"[bench] rk4 256^3: warmup {WU} steps, tile {choice}")
    S.s4_rk4(ctx, box, [u], [rho], None, d["dt"], WU, "graph", ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    S.s4_rk4(ctx, box, [u], [rho], None, d["dt"], K, "graph", ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    # the timed outputs (after WU + K steps), checked against the oracle in the CPU leg
    timed_u, timed_rho = u.cpu().numpy(), rho.cpu().numpy()
    finite = bool(np.isfinite(timed_u).all() and np.isfinite(timed_rho).all())
    log(f"[bench] rk4 256^3: {K} steps in {wall * 1e3:.2f} ms wall, {ev_ms:.2f} ms events, finite={finite}")
    value = npts * K / wall / 1e9
    # dominant kernel: the only kernel in the timed region.  Per-stage kernel set:
    # 4 launches per step moving 4, 8, 10, 6 accesses per point; fused stage
    # pairs: 2 launches per step moving 6 (stages 1-2) and 8 (stages 3-4);
    # whole steps: 1 launch reading u_n, rho_n and writing u_{n+1}, rho_{n+1}.
    kop = choice["kernel_op"]
    launch_bytes = [4] if kop == 102 else [6, 8] if kop in (100, 101) else [4, 8, 10, 6]  # 8-byte accesses
    nlaunch = len(launch_bytes)
    bytes_per_launch = npts * 8 * sum(launch_bytes) / nlaunch
    launch_s = ev_ms / 1e3 / (nlaunch * K)
    achieved = bytes_per_launch / launch_s / 1e9
    if kop == 102:
        kname = f"k_rk4_step4<{choice['tile_x']},{choice['threads'] // 64}>"
        tkey = "step4_wave256"
    elif kop == 100:
        kname = f"k_rk4_pair<{choice['tile_x']},{choice['threads'] // 64},pair 0|1>"
        tkey = "pair_wave256"
    elif kop == 101:
        kname = f"k_pair2<{choice['tile_x']},{choice['threads'] // 64},pair 0|1>"
        tkey = "pair2_wave256"
    elif kop >= 200:
        wx = choice["tile_x"] // 64
        kname = f"k_rows_single<{wx},{4 // wx},{choice['tile_y'] // (4 // wx)},periodic,stage 1..4>"
        tkey = "rows_stage_wave256"
    else:
        kname = f"k_tiles_single<{choice['tile_x']},{choice['threads'] // 64},periodic,stage 1..4>"
        tkey = "stage_wave256"
    tile_rk4 = [choice["tile_x"], choice["tile_y"], choice["z_chunk"], choice["threads"]]
    traffic = traffic_from_profile(tkey, tile_rk4)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kname, "avg_launch_us": round(launch_s * 1e6, 2),
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            "bytes_per_point_step": 8 * sum(launch_bytes), "launches_per_step": nlaunch,
            "kernel_set": kernel_set(choice)}
    del u, rho, ws

    # ------------------------------------------------------------------ tile choice: heuristic, on-line, sweep
    if "tuning" in sections:
        # the paper's LoopControl comparison on this loop: the heuristic start,
        # the on-line random-restart hill climber after a fixed number of calls,
        # and the offline sweep, each timed afterwards on the same data
        uu, rr = to_dev(d["u"]), to_dev(d["rho"])
        wst = S.workspace(S.s4_workspace_size(box, S.S4_OP_RK4, S.S4_GRAPH))
        # fresh contexts that do not load the tuned choices: the heuristic start
        # and the on-line search from that start
        saved = os.environ.pop("S4_TUNE_CACHE", None)
        try:
            heur = S.s4_get_choice(S.Context(0), S.S4_OP_RK4, box)["candidate"]
            on = S.Context(0)
        finally:
            if saved is not None:
                os.environ["S4_TUNE_CACHE"] = saved
        S.s4_set_online_tuning(on, True, 0.02, 1)
        ncalls, spc = 60, 4
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(ncalls):
            S.s4_rk4(on, box, [uu], [rr], None, d["dt"], spc, "graph", ws=wst)
        torch.cuda.synchronize()
        online_total = time.perf_counter() - t0
        onc = S.s4_get_choice(on, S.S4_OP_RK4, box)["candidate"]

        def per_step(cand):
            S.s4_set_choice(ctx, S.S4_OP_RK4, box, cand)
            S.s4_rk4(ctx, box, [uu], [rr], None, d["dt"], 4, "graph", ws=wst)
            ts = []
            for _ in range(5):
                e0.record(stream)
                S.s4_rk4(ctx, box, [uu], [rr], None, d["dt"], 10, "graph", ws=wst)
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) / 10)
            S.s4_set_choice(ctx, S.S4_OP_RK4, box, -1)
            return sorted(ts)[2]

        sweep = choice["candidate"] if choice["tuned"] else None
        out["tuning"] = {"workload": "wave256 RK4 step", "heuristic": {"candidate": heur, "ms_per_step": round(per_step(heur), 4)},
                         "online": {"candidate": onc, "ms_per_step": round(per_step(onc), 4), "calls": ncalls,
                                    "steps_per_call": spc,
                                    "ms_per_step_during_search": round(online_total * 1e3 / (ncalls * spc), 4)}}
        if sweep is not None:
            out["tuning"]["sweep"] = {"candidate": sweep, "ms_per_step": round(per_step(sweep), 4)}
        log(f"[bench] tuning: {out['tuning']}")
        del uu, rr, wst

    # ------------------------------------------------------------------ RHS 256^3, rotating buffers
    if "rhs" in sections:
        nset = 4
        us = [to_dev(d["u"]) for _ in range(nset)]
        for t in us:
            S.s4_fill_ghosts_periodic(ctx, box, [t])
        outs = [S.alloc_field(n, g, fill=0.0) for _ in range(nset)]
        reps = max(20, K // 2)
        for i in range(8):
            S.s4_wave_rhs(ctx, box, [us[i % nset]], None, [outs[i % nset]])
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            S.s4_wave_rhs(ctx, box, [us[i % nset]], None, [outs[i % nset]])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = npts * 16 / (ms / 1e3) / 1e9
        ch = S.s4_get_choice(ctx, S.S4_OP_WAVE_RHS, box)
        out["rhs"] = {"workload": "wave256 single RHS (ghosts read, c=1)", "us_per_rhs": round(ms * 1e3, 2),
                      "gpoint_per_s": round(npts / (ms / 1e3) / 1e9, 1), "achieved_GBs": round(gbs, 1),
                      "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_point": 16,
                      "tile": [ch["tile_x"], ch["tile_y"], ch["z_chunk"], ch["threads"]], "kernel_set": kernel_set(ch),
                      "traffic": traffic_from_profile("rhs_wave256", [ch["tile_x"], ch["tile_y"], ch["z_chunk"],
                                                                      ch["threads"]])}
        log(f"[bench] rhs: {out['rhs']}")
        del us, outs

    # ------------------------------------------------------------------ 32^3 latency
    if "latency32" in sections:
        # the cache-resident 32^3 box: microseconds per RHS and per RK4 step
        # (no HBM fraction: 0.5 MB per field stays in cache)
        d32 = W.wave32()
        g32, n32 = d32["ghost"], d32["n"]
        u32 = S.alloc_field(n32, g32, fill=0.0)
        r32 = S.alloc_field(n32, g32, fill=0.0)
        S.interior(u32, g32).copy_(torch.from_numpy(d32["u"]))
        S.interior(r32, g32).copy_(torch.from_numpy(d32["rho"]))
        b32 = S.box_of(u32, g32, d32["dx"])
        S.s4_fill_ghosts_periodic(ctx, b32, [u32])
        o32 = S.alloc_field(n32, g32, fill=0.0)
        ws32 = S.workspace(S.s4_workspace_size(b32, S.S4_OP_RK4, S.S4_GRAPH))
        for _ in range(20):
            S.s4_wave_rhs(ctx, b32, [u32], None, [o32])
        S.s4_rk4(ctx, b32, [u32], [r32], None, d32["dt"], 20, "graph", ws=ws32)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(200):
            S.s4_wave_rhs(ctx, b32, [u32], None, [o32])
        e1.record(stream)
        torch.cuda.synchronize()
        rhs_us = e0.elapsed_time(e1) / 200 * 1e3
        e0.record(stream)
        S.s4_rk4(ctx, b32, [u32], [r32], None, d32["dt"], 200, "graph", ws=ws32)
        e1.record(stream)
        torch.cuda.synchronize()
        step_us = e0.elapsed_time(e1) / 200 * 1e3
        out["latency32"] = {"workload": "wave32: 32^3 + 2 ghosts, periodic, cache-resident",
                            "us_per_rhs": round(rhs_us, 2), "us_per_rk4_step": round(step_us, 2),
                            "rk4_kernel_set": kernel_set(S.s4_get_choice(ctx, S.S4_OP_RK4, b32))}
        log(f"[bench] latency32: {out['latency32']}")
        del u32, r32, o32, ws32

    # ------------------------------------------------------------------ 256^3 RK4 with variable c^2
    if "rk4c2" in sections:
        # the headline box with a variable wave speed (c^2 = 1 + 0.5 U[-1,1), the
        # adjoint workload's form): its own loop setup, tuned apart; 40 B per point-step
        rk4c2 = S.S4_OP_RK4 | S.S4_WITH_C2
        if not args.no_tune:
            S.s4_tune(ctx, rk4c2, box, flags=1)
            torch.cuda.empty_cache()
        uc, rc = to_dev(d["u"]), to_dev(d["rho"])
        cc = to_dev(1.0 + 0.5 * W.uniform_pm1(d["seed"], 99, tuple(n[::-1])))  # c^2 is read at interior points only
        wsc = S.workspace(S.s4_workspace_size(box, S.S4_OP_RK4, S.S4_GRAPH))
        S.s4_rk4(ctx, box, [uc], [rc], [cc], d["dt"], 20, "graph", ws=wsc)
        torch.cuda.synchronize()
        e0.record(stream)
        S.s4_rk4(ctx, box, [uc], [rc], [cc], d["dt"], 100, "graph", ws=wsc)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 100
        chc = S.s4_get_choice(ctx, rk4c2, box)
        out["rk4_c2"] = {"workload": "wave256 RK4 step with variable c^2", "ms_per_step": round(ms, 4),
                         "gpoint_steps_per_s": round(npts / (ms / 1e3) / 1e9, 2),
                         "achieved_GBs": round(npts * 40 / (ms / 1e3) / 1e9, 1), "bytes_per_point_step": 40,
                         "tile": [chc["tile_x"], chc["tile_y"], chc["z_chunk"], chc["threads"]],
                         "kernel_set": kernel_set(chc), "tuned": bool(chc["tuned"]),
                         "finite": bool(torch.isfinite(uc).all().item())}
        log(f"[bench] rk4_c2: {out['rk4_c2']}")
        del uc, rc, cc, wsc

    # ------------------------------------------------------------------ copy probe
    if "copy" in sections:
        nb = 1 << 30
        a = torch.empty(nb // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            S.s4_copy(ctx, b, a)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(10):
            S.s4_copy(ctx, b, a)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out["copy"] = {"bytes": 2 * nb, "us": round(ms * 1e3, 1), "GBs": round(2 * nb / (ms / 1e3) / 1e9, 1)}
        log(f"[bench] copy: {out['copy']}")
        del a, b

    # ------------------------------------------------------------------ multi-field mixed derivatives
    if "mixed" in sections:
        md = W.mixed_fields()
        gm = md["ghost"]
        nm = md["n"]
        mpts = nm[0] * nm[1] * nm[2]
        gfs = []
        for f in md["fields"]:
            t = S.alloc_field(nm, gm, fill=0.0)
            S.interior(t, gm).copy_(torch.from_numpy(f))
            gfs.append(t)
        mbox = S.box_of(gfs[0], gm, md["dx"])
        if not args.no_tune:
            S.s4_tune(ctx, S.S4_OP_DERIV_MIXED, mbox, flags=1)
            torch.cuda.empty_cache()
        S.s4_fill_ghosts_periodic(ctx, [mbox] * len(gfs), gfs)
        mouts = [S.alloc_field(nm, gm, fill=0.0) for _ in gfs]
        for _ in range(3):
            S.s4_deriv_mixed(ctx, mbox, gfs, md["A"], mouts)
        reps = 10
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            S.s4_deriv_mixed(ctx, mbox, gfs, md["A"], mouts)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nf = len(gfs)
        gbs = mpts * nf * 16 / (ms / 1e3) / 1e9
        ch = S.s4_get_choice(ctx, S.S4_OP_DERIV_MIXED, mbox)
        out["mixed"] = {"workload": "mixed192: 6 fields, 192^3 + 2 ghosts, sine-mode fields, symmetric A",
                        "us_per_call": round(ms * 1e3, 1), "gpoint_per_s": round(mpts / (ms / 1e3) / 1e9, 2),
                        "field_gpoint_per_s": round(mpts * nf / (ms / 1e3) / 1e9, 1),
                        "achieved_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                        "bytes_per_point": 16 * nf,
                        "fp64_tflops_est": round(mpts * nf * MIXED_FLOPS_PER_FIELD_POINT / (ms / 1e3) / 1e12, 2),
                        "tile": [ch["tile_x"], ch["tile_y"], ch["z_chunk"], ch["threads"]], "kernel_set": kernel_set(ch)}
        log(f"[bench] mixed: {out['mixed']}")
        del gfs, mouts

    # ------------------------------------------------------------------ batched bboxset
    if "batched" in sections:
        bd = W.bboxset()
        gb = bd["ghost"]
        fields, boxes = [], []
        for i, bx in enumerate(bd["boxes"]):
            fu = S.alloc_field(bx["n"], gb, fill=0.0)
            fr = S.alloc_field(bx["n"], gb, fill=0.0)
            S.interior(fu, gb).copy_(torch.from_numpy(bd["u"][i]))
            S.interior(fr, gb).copy_(torch.from_numpy(bd["rho"][i]))
            fields.append((fu, fr))
            boxes.append(S.box_of(fu, gb, bx["dx"], bx["level"]))
        bpts = sum(int(np.prod(bx["n"])) for bx in bd["boxes"])
        if not args.no_tune:
            S.s4_tune(ctx, S.S4_OP_RK4, boxes, flags=1)
            torch.cuda.empty_cache()
        wsb = S.workspace(S.s4_workspace_size(boxes, S.S4_OP_RK4, S.S4_GRAPH))
        us_ = [f[0] for f in fields]
        rs_ = [f[1] for f in fields]
        res = {}
        kb = max(10, K // 5)
        for mode in ("perbox", "batched", "graph"):
            S.s4_rk4(ctx, boxes, us_, rs_, None, bd["dt"], 3, mode, ws=wsb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            S.s4_rk4(ctx, boxes, us_, rs_, None, bd["dt"], kb, mode, ws=wsb)
            e1.record(stream)
            torch.cuda.synchronize()
            w_ = time.perf_counter() - t0
            res[mode] = {"ms_per_step": round(w_ * 1e3 / kb, 4), "gpoint_steps_per_s": round(bpts * kb / w_ / 1e9, 2),
                         "event_ms_per_step": round(e0.elapsed_time(e1) / kb, 4)}
        ch = S.s4_get_choice(ctx, S.S4_OP_RK4, boxes)
        out["batched"] = {"workload": "bboxset60: 3 levels x 20 boxes, sides U[16,96], g=3, 1 RK4 step",
                          "interior_points": bpts, "steps": kb, "modes": res,
                          "speedup_batched_vs_perbox": round(res["perbox"]["ms_per_step"] / res["batched"]["ms_per_step"], 3),
                          "speedup_graph_vs_perbox": round(res["perbox"]["ms_per_step"] / res["graph"]["ms_per_step"], 3),
                          "tile": [ch["tile_x"], ch["tile_y"], ch["z_chunk"], ch["threads"]], "kernel_set": kernel_set(ch),
                          "launches_per_step": kernels_per_step(ch, len(boxes))}
        log(f"[bench] batched: {out['batched']}")
        del fields, us_, rs_, wsb

    # ------------------------------------------------------------------ level with ghost exchange
    if "level" in sections:
        ld = W.level_tiling()
        gl = ld["ghost"]
        lus, lrs, lboxes = [], [], []
        for bx in ld["boxes"]:
            sl = W.box_slice(bx)
            fu = S.alloc_field(bx["n"], gl, fill=0.0)
            fr = S.alloc_field(bx["n"], gl, fill=0.0)
            S.interior(fu, gl).copy_(torch.from_numpy(np.ascontiguousarray(ld["u"][sl])))
            S.interior(fr, gl).copy_(torch.from_numpy(np.ascontiguousarray(ld["rho"][sl])))
            lus.append(fu)
            lrs.append(fr)
            lboxes.append(S.box_of(fu, gl, ld["dx"]))
        llo = [bx["lo"] for bx in ld["boxes"]]
        t0 = time.perf_counter()
        lev = S.s4_level_create(lboxes, llo, ld["domain"], 2, "faces")
        plan_ms = (time.perf_counter() - t0) * 1e3
        info = S.s4_level_info(lev)
        lpts = info["points"]
        if not args.no_tune:
            S.s4_tune(ctx, S.S4_OP_RK4, lboxes, flags=1)
            torch.cuda.empty_cache()
        wsl = S.workspace(S.s4_level_workspace_size(lev, S.S4_OP_RK4))
        kl = max(10, K // 5)
        res = {}
        for mode in ("perbox", "batched", "graph"):
            S.s4_level_rk4(ctx, lev, lus, lrs, None, ld["dt"], 3, mode, ws=wsl)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            S.s4_level_rk4(ctx, lev, lus, lrs, None, ld["dt"], kl, mode, ws=wsl)
            e1.record(stream)
            torch.cuda.synchronize()
            w_ = time.perf_counter() - t0
            res[mode] = {"ms_per_step": round(w_ * 1e3 / kl, 4), "gpoint_steps_per_s": round(lpts * kl / w_ / 1e9, 2),
                         "event_ms_per_step": round(e0.elapsed_time(e1) / kl, 4)}
        # one exchange per call (the call uploads its schedule and synchronises first)
        wss = S.workspace(S.s4_level_workspace_size(lev, S.S4_OP_LEVEL_SYNC))
        S.s4_level_sync(ctx, lev, lus, ws=wss)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            S.s4_level_sync(ctx, lev, lus, ws=wss)
        torch.cuda.synchronize()
        sync_ms = (time.perf_counter() - t0) * 1e3 / 20
        del wsl, wss, lus, lrs
        torch.cuda.empty_cache()
        # the same domain as one periodic box (no exchange: wrapped addressing)
        one_u = S.alloc_field(ld["domain"], 2, fill=0.0)
        one_r = S.alloc_field(ld["domain"], 2, fill=0.0)
        S.interior(one_u, 2).copy_(torch.from_numpy(ld["u"]))
        S.interior(one_r, 2).copy_(torch.from_numpy(ld["rho"]))
        ob = S.box_of(one_u, 2, ld["dx"])
        wso = S.s4_rk4(ctx, ob, [one_u], [one_r], None, ld["dt"], 4, "graph")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.s4_rk4(ctx, ob, [one_u], [one_r], None, ld["dt"], kl, "graph", ws=wso)
        torch.cuda.synchronize()
        one_ms = (time.perf_counter() - t0) * 1e3 / kl
        del one_u, one_r, wso
        ch = S.s4_level_choice(ctx, lev)
        # the same level with 4 ghost layers and a full exchange of width 4:
        # whole RK4 steps, one exchange of (u, rho) per step
        lw = W.level_tiling(ghost=4)
        wus, wrs, wboxes = [], [], []
        for bx in lw["boxes"]:
            sl = W.box_slice(bx)
            fu = S.alloc_field(bx["n"], 4, fill=0.0)
            fr = S.alloc_field(bx["n"], 4, fill=0.0)
            S.interior(fu, 4).copy_(torch.from_numpy(np.ascontiguousarray(lw["u"][sl])))
            S.interior(fr, 4).copy_(torch.from_numpy(np.ascontiguousarray(lw["rho"][sl])))
            wus.append(fu)
            wrs.append(fr)
            wboxes.append(S.box_of(fu, 4, lw["dx"]))
        levw = S.s4_level_create(wboxes, [bx["lo"] for bx in lw["boxes"]], lw["domain"], 4, "full")
        infow = S.s4_level_info(levw)
        if not args.no_tune:
            S.s4_tune(ctx, S.S4_OP_RK4, wboxes, flags=1)
        wsw = S.workspace(S.s4_level_workspace_size(levw, S.S4_OP_RK4))
        resw = {}
        for mode in ("perbox", "batched", "graph"):
            S.s4_level_rk4(ctx, levw, wus, wrs, None, lw["dt"], 4, mode, ws=wsw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            S.s4_level_rk4(ctx, levw, wus, wrs, None, lw["dt"], kl, mode, ws=wsw)
            e1.record(stream)
            torch.cuda.synchronize()
            w_ = time.perf_counter() - t0
            resw[mode] = {"ms_per_step": round(w_ * 1e3 / kl, 4),
                          "gpoint_steps_per_s": round(lpts * kl / w_ / 1e9, 2),
                          "event_ms_per_step": round(e0.elapsed_time(e1) / kl, 4)}
        chw = S.s4_level_choice(ctx, levw)
        wide = {"workload": "level60 with 4 ghost layers, full exchange of width 4 before every RK4 step",
                "modes": resw, "schedule_pieces": infow["pieces"],
                "ghost_points_per_exchange": infow["filled"], "exchange_bytes": 2 * 16 * infow["filled"],
                "level_graph_over_single_box": round(resw["graph"]["ms_per_step"] / one_ms, 3),
                "tile": [chw["tile_x"], chw["tile_y"], chw["z_chunk"], chw["threads"]],
                "kernel_set": kernel_set(chw), "launches_per_step": kernels_per_step(chw, len(wboxes), level=True)}
        del wus, wrs, wsw
        out["level"] = {"workload": "level60: 60 boxes, sides U[16,96], g=3, tiling a 280x224x168 periodic domain, "
                                    "face exchange of width 2 before every RK4 stage",
                        "interior_points": lpts, "steps": kl, "modes": res,
                        "schedule_build_ms": round(plan_ms, 2), "schedule_pieces": info["pieces"],
                        "ghost_points_per_exchange": info["filled"],
                        "exchange_call_ms": round(sync_ms, 4),
                        "exchange_bytes": 16 * info["filled"],
                        "single_box_same_domain_ms_per_step": round(one_ms, 4),
                        "level_graph_over_single_box": round(res["graph"]["ms_per_step"] / one_ms, 3),
                        "tile": [ch["tile_x"], ch["tile_y"], ch["z_chunk"], ch["threads"]], "kernel_set": kernel_set(ch),
                        "launches_per_step": kernels_per_step(ch, len(lboxes), level=True),
                        "wide": wide}
        log(f"[bench] level: {out['level']}")

    # ------------------------------------------------------------------ adjoint
    if "adjoint" in sections:
        from paper_1308_1343_amd.autograd import wave_rk4
        ad = W.adjoint_case()
        ga = ad["ghost"]
        na = ad["n"]
        apts = na[0] * na[1] * na[2]

        def compact(a, fill=0.0):
            t = torch.full((na[2] + 2 * ga, na[1] + 2 * ga, na[0] + 2 * ga), fill, dtype=torch.float64, device=dev)
            S.interior(t, ga).copy_(torch.from_numpy(a))
            return t

        u0, r0, c2, ut = compact(ad["u0"]), compact(ad["rho0"]), compact(ad["c2"], 1.0), compact(ad["u_target"])
        if not args.no_tune:
            abox = S.box_of(u0, ga, ad["dx"])
            # the forward steps and their replays pass c^2: that loop setup is tuned
            for op in (S.S4_OP_RK4 | S.S4_WITH_C2, S.S4_OP_ADJOINT_STEP):
                S.s4_tune(ctx, op, abox, flags=1)
            torch.cuda.empty_cache()
        times = []
        for rep in range(2):
            u0.requires_grad_(True)
            r0.requires_grad_(True)
            c2.requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uT, rT = wave_rk4(u0, r0, c2, ga, ad["dx"], ad["dt"], ad["nsteps"], ad["checkpoint"], ctx)
            diff = S.interior(uT, ga) - S.interior(ut, ga)
            J = 0.5 * (diff * diff).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            J.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append((t1 - t0, t2 - t1))
            gu = u0.grad
            u0.grad = r0.grad = c2.grad = None
            u0, r0, c2 = u0.detach(), r0.detach(), c2.detach()
        tf, tb = times[-1]
        out["adjoint"] = {"workload": "adjoint128: 128^3, variable c^2, 50 RK4 steps, checkpoint every 10",
                          "forward_s": round(tf, 4), "backward_s": round(tb, 4),
                          "forward_gpoint_steps_per_s": round(apts * ad["nsteps"] / tf / 1e9, 2),
                          "backward_gpoint_steps_per_s": round(apts * ad["nsteps"] / tb / 1e9, 2),
                          "backward_over_forward": round(tb / tf, 2), "loss": float(J.item()),
                          "grad_finite": bool(torch.isfinite(gu).all().item())}
        log(f"[bench] adjoint: {out['adjoint']}")

    # ------------------------------------------------------------------ CPU oracle baseline
    # The oracle runs the headline's WU + K steps from the same inputs: its
    # final state is the parity reference for the timed outputs, and its time
    # (continued by more steps up to about 20 s of CPU work) is the baseline.
    cpu = None
    parity = None
    if "cpu" in sections:
        import oracle as O
        u0 = O.embed(d["u"], g)
        r0 = O.embed(d["rho"], g)
        nrun = WU + K
        t0 = time.perf_counter()
        ou, orr = O.rk4(u0, r0, g, d["dx"], d["dt"], nrun)
        el = time.perf_counter() - t0
        sl = (slice(g, -g),) * 3

        def rel_err(got, want):
            return float(np.max(np.abs(got[sl] - want[sl])) / np.max(np.abs(want[sl])))

        parity = {"u": rel_err(timed_u, ou), "rho": rel_err(timed_rho, orr), "steps": nrun,
                  "reference": "FP64 oracle from the same inputs", "tolerance": 1e-12}
        parity["max"] = max(parity["u"], parity["rho"])
        log(f"[bench] parity of the timed 256^3 outputs: {parity}")
        m = nrun
        if el < 10.0:  # continue to about 20 s of CPU work
            more = int(min(300, max(1, math.ceil((20.0 - el) / max(el / nrun, 1e-3)))))
            t0 = time.perf_counter()
            O.rk4(ou, orr, g, d["dx"], d["dt"], more)
            el += time.perf_counter() - t0
            m += more
        model = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as f:
                model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
        except OSError:
            pass
        cpu = {"value": round(npts * m / el / 1e9, 5), "unit": "Gpoint-updates/s", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": f"{m} RK4 steps of the 256^3 wave workload ({nrun} from the inputs of the timed GPU run, "
                         f"the parity reference, then {m - nrun} more), plain C FP64 oracle with OpenMP on {model}, "
                         f"{el:.1f} s"}
        log(f"[bench] cpu: {cpu}")
        # the same oracle on one thread, a few steps (about 5 s)
        nthr = O.num_threads()
        O.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            O.rk4(u0, r0, g, d["dx"], d["dt"], 1)
            one1 = time.perf_counter() - t0
            m1 = int(min(20, max(1, math.ceil(4.0 / max(one1, 1e-3)))))
            t0 = time.perf_counter()
            O.rk4(u0, r0, g, d["dx"], d["dt"], m1)
            el1 = time.perf_counter() - t0
        finally:
            O.set_num_threads(nthr)
        out["cpu_single_thread"] = {"value": round(npts * m1 / el1 / 1e9, 5), "unit": "Gpoint-updates/s",
                                    "cores": 1, "kind": "oracle",
                                    "sample": f"{m1} RK4 steps of the 256^3 wave workload on one thread, "
                                              f"{model}, {el1:.1f} s"}
        log(f"[bench] cpu single thread: {out['cpu_single_thread']}")

    # the single-box RHS against the copy probe of the same run (SURVEY's "% of a STREAM-copy probe")
    if "rhs" in out and "copy" in out:
        out["rhs"]["frac_of_copy"] = round(out["rhs"]["achieved_GBs"] / out["copy"]["GBs"], 4)
        if out["rhs"].get("traffic"):
            out["rhs"]["traffic_GBs"] = round(out["rhs"]["traffic"] / (out["rhs"]["us_per_rhs"] * 1e3), 1)
    rec = {"metric": METRIC, "value": round(value, 3), "unit": "Gpoint-updates/s", "n_gpus": 1, "steps": K,
           "warmup": WU, "ms_per_step": round(wall * 1e3 / K, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "wave256_rk4: 256^3 interior + 2 ghosts, periodic, FP64, h=1/256, dt=h/4, "
                                  "u=U+Gaussian(0.1), rho=U, RK4 steps replayed as a hipGraph",
                      "points": npts, "seed": d["seed"], "tile": [choice["tile_x"], choice["tile_y"],
                                                                   choice["z_chunk"], choice["threads"]],
                      "tile_from_tuner": bool(choice["tuned"])},
           "roofline": roof, "cpu_baseline": cpu, "max_rel_err": None if parity is None else parity["max"],
           "parity": parity}
    rec.update(out)
    print(json.dumps(rec), flush=True)
    if parity is not None and not parity["max"] <= parity["tolerance"]:
        log(f"[bench] PARITY FAILURE: timed outputs differ from the oracle by {parity['max']:.3e} "
            f"(> {parity['tolerance']:.0e})")
        sys.exit(1)


if __name__ == "__main__":
    main()
