"""s4_rk4_noalloc (the library's static scratch array instead of a caller
workspace) against s4_rk4 with a workspace, bit for bit, on two calls in a
row with the second on smaller boxes, in both launch modes it accepts; plus
the oracle on one case and the host-side rejections."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1308_1343_amd as S
import workload as W
from _gpu import host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return S.Context(0)


def fields(n, g, seed):
    u = S.alloc_field(n, g, fill=0.0)
    r = S.alloc_field(n, g, fill=0.0)
    ua = W.uniform_pm1(seed, 1, tuple(n[::-1]))
    ra = W.uniform_pm1(seed, 2, tuple(n[::-1]))
    S.interior(u, g).copy_(torch.from_numpy(ua))
    S.interior(r, g).copy_(torch.from_numpy(ra))
    return u, r, ua, ra


def run_pair(ctx, shapes, g, mode, nsteps, seed):
    """(noalloc result, workspace result) on the boxes `shapes`."""
    dt = 0.25 / max(max(n) for n in shapes)
    A = [fields(n, g, seed + i) for i, n in enumerate(shapes)]
    B = [fields(n, g, seed + i) for i, n in enumerate(shapes)]
    boxes = [S.box_of(a[0], g, 1.0 / n[0]) for a, n in zip(A, shapes)]
    S.s4_rk4_noalloc(ctx, boxes, [a[0] for a in A], [a[1] for a in A], None, dt, nsteps, mode)
    S.s4_rk4(ctx, boxes, [b[0] for b in B], [b[1] for b in B], None, dt, nsteps, mode)
    return A, B, boxes, dt


@pytest.mark.parametrize("mode", ["perbox", "batched"])
@pytest.mark.parametrize("nsteps", [4, 3])
def test_noalloc_matches_workspace_call_twice(ctx, mode, nsteps):
    g = 2
    for shapes in ([(48, 40, 36)], [(20, 16, 12)]):  # the second call on a smaller box
        A, B, boxes, dt = run_pair(ctx, shapes, g, mode, nsteps, 11)
        for a, b in zip(A, B):
            np.testing.assert_array_equal(host(a[0]), host(b[0]))
            np.testing.assert_array_equal(host(a[1]), host(b[1]))
    # the last call against the oracle
    (u, r, ua, ra), = A
    n = shapes[0]
    wu, wr = O.rk4(O.embed(ua, g), O.embed(ra, g), g, 1.0 / n[0], dt, nsteps)
    assert rel(host(u), wu, g) <= 1e-12 and rel(host(r), wr, g) <= 1e-12


@pytest.mark.parametrize("mode", ["perbox", "batched"])
def test_noalloc_box_sets_twice(ctx, mode):
    g = 3
    for shapes in ([(24, 20, 16), (33, 17, 21), (16, 16, 16)], [(18, 16, 16), (16, 20, 17)]):
        A, B, boxes, dt = run_pair(ctx, shapes, g, mode, 2, 21)
        for i, (a, b) in enumerate(zip(A, B)):
            np.testing.assert_array_equal(host(a[0]), host(b[0]), err_msg=f"box {i}")
            np.testing.assert_array_equal(host(a[1]), host(b[1]), err_msg=f"box {i}")


def test_noalloc_rejections(ctx):
    u = S.alloc_field((16, 16, 16), 2, fill=0.0)
    r = S.alloc_field((16, 16, 16), 2, fill=0.0)
    b = S.box_of(u, 2, 1 / 16)
    with pytest.raises(S.Sten4Error) as e:
        S.s4_rk4_noalloc(ctx, b, [u], [r], None, 0.01, 1, "graph")
    assert e.value.code == S.S4_ENOTSUP
    # a box whose workspace exceeds the scratch array: rejected before any launch
    big = S.make_box((256, 256, 256), 2, (1, 272, 272 * 260), 1 / 256)
    assert S.s4_workspace_size(big, S.S4_OP_RK4, S.S4_BATCHED) > S.S4_NOALLOC_SCRATCH_BYTES
    with pytest.raises(S.Sten4Error) as e:
        S.s4_rk4_noalloc(ctx, big, [u], [r], None, 0.01, 1, "batched")
    assert e.value.code == S.S4_ENOMEM
    # nothing to do: accepted
    S.s4_rk4_noalloc(ctx, b, [u], [r], None, 0.01, 0, "batched")
