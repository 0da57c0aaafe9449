"""Shared helpers of the GPU tests: moving oracle-layout numpy arrays (compact,
(nz+2g, ny+2g, nx+2g)) to and from device box views, and the parity metric."""
import numpy as np
import torch

import paper_1308_1343_amd as S

NAN = float("nan")


def dev(a, g, pad=True, ghost_value=NAN):
    """Device box view holding numpy ghosted array `a`; ghosts set to ghost_value
    (NaN canaries by default) unless keep_ghosts."""
    nz, ny, nx = a.shape
    t = S.alloc_field((nx - 2 * g, ny - 2 * g, nz - 2 * g), g, pad=pad, fill=ghost_value)
    t[g:nz - g, g:ny - g, g:nx - g].copy_(torch.from_numpy(np.ascontiguousarray(a[g:nz - g, g:ny - g, g:nx - g])))
    return t


def dev_full(a, g, pad=True):
    """Device box view holding all of `a`, ghosts included."""
    nz, ny, nx = a.shape
    t = S.alloc_field((nx - 2 * g, ny - 2 * g, nz - 2 * g), g, pad=pad, fill=NAN)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return t


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def inner(a, g):
    return a[g:a.shape[0] - g, g:a.shape[1] - g, g:a.shape[2] - g]


def rel(x, y, g):
    """max-norm relative error over interior points: max|x - y| / max|y|."""
    xi, yi = inner(x, g), inner(y, g)
    return float(np.max(np.abs(xi - yi)) / max(np.max(np.abs(yi)), 1e-300))


def ghosts_untouched(a, g):
    m = np.ones(a.shape, bool)
    m[g:-g, g:-g, g:-g] = False
    return bool(np.all(np.isnan(a[m])))


def cands_by_kind(ctx, op, boxes):
    """Candidate indices this op may use on these boxes, by kernel set:
    "tiles" (LDS tile traversal), "rows" (row-register traversal), "pairs"
    (pair-lane tiles of the RHS), "fused" (both RK4 stage-pair sets and the
    whole-step kernels)."""
    nc = S.s4_get_choice(ctx, op, boxes)["ncandidates"]
    out = {"tiles": [], "rows": [], "pairs": [], "fused": []}
    for c in range(nc):
        try:
            S.s4_set_choice(ctx, op, boxes, c)
        except S.Sten4Error as e:  # a candidate these boxes do not fit
            assert e.code == S.S4_ENOTSUP
            continue
        k = S.s4_get_choice(ctx, op, boxes)["kernel_op"]
        out["fused" if k in (100, 101, 102) else "pairs" if k >= 300 else "rows" if k >= 200
            else "tiles"].append(c)
    S.s4_set_choice(ctx, op, boxes, -1)
    return out
