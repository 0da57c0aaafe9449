"""The tensor-level surface (wave_rhs, rk4, deriv_mixed, BoxSet) against the
FP64 oracle: each call only builds descriptors and workspaces around the C
ABI, so results must match the oracle as the C-ABI calls do."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1308_1343_amd as S
import workload as W
from _gpu import NAN, dev, dev_full, host, rel

pytestmark = pytest.mark.gpu
TOL = 1e-12


def rand(n, g, seed, stream):
    return O.embed(W.uniform_pm1(seed, stream, tuple(n[::-1])), g)


def test_wave_rhs_and_fill():
    n, g, dx = (40, 24, 18), 2, (1 / 40, 1 / 24, 1 / 18)
    a = rand(n, g, 5, 1)
    u = dev(a, g)
    S.fill_ghosts(u, g)
    af = O.fill_ghosts_periodic(a.copy(), g)
    np.testing.assert_array_equal(host(u), af)
    c2h = O.embed(1.0 + 0.5 * W.uniform_pm1(5, 2, n[::-1]), g)
    for c2 in (None, dev(c2h, g)):
        out = S.wave_rhs(u, g, dx, c2=c2)
        want = O.wave_rhs(af, g, dx, None if c2 is None else c2h)
        assert rel(host(out), want, g) <= TOL


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
def test_rk4(mode):
    n, g = (36, 20, 28), 2
    dx, dt = 1 / 36, 0.25 / 36
    a, r = rand(n, g, 6, 1), rand(n, g, 6, 2)
    u, rho = dev(a, g, ghost_value=0.0), dev(r, g, ghost_value=0.0)
    S.rk4(u, rho, g, dx, dt, 5, mode=mode)
    wu, wr = O.rk4(a, r, g, dx, dt, 5)
    assert rel(host(u), wu, g) <= TOL and rel(host(rho), wr, g) <= TOL


def test_deriv_mixed():
    n, g, dx = (24, 20, 16), 2, (1 / 24, 1 / 20, 1 / 16)
    A = np.array([[0.5, -0.25, 0.75], [-0.25, 1.0, 0.1], [0.75, 0.1, -0.6]])
    fs = [O.fill_ghosts_periodic(rand(n, g, 7, k), g) for k in range(3)]
    gs = [dev_full(f, g) for f in fs]
    outs = S.deriv_mixed(gs, A, g, dx)
    for f, o in zip(fs, outs):
        assert rel(host(o), O.deriv_mixed(f, g, dx, A), g) <= TOL


@pytest.mark.parametrize("mode", ["perbox", "batched", "graph"])
def test_boxset_rk4_and_rhs(mode):
    spec = [{"n": (16, 20, 24), "ghost": 3, "dx": 1 / 16, "level": 0},
            ((33, 17, 9), 3, (1 / 32, 1 / 34, 1 / 18), 1),
            ((20, 20, 20), 2, 1 / 20)]
    bs = S.BoxSet(spec)
    assert len(bs) == 3
    u, rho = bs.alloc(0.0), bs.alloc(0.0)
    host_u, host_r = [], []
    for i, (t, q, sp) in enumerate(zip(u, rho, bs.spec)):
        n, g = sp[0], sp[1]
        a, r = rand(n, g, 8, 2 * i), rand(n, g, 8, 2 * i + 1)
        S.interior(t, g).copy_(torch.from_numpy(S_interior(a, g)))
        S.interior(q, g).copy_(torch.from_numpy(S_interior(r, g)))
        host_u.append(a)
        host_r.append(r)
    dt = 0.25 / 34
    bs.rk4(u, rho, dt, 3, mode=mode)
    for i, sp in enumerate(bs.spec):
        n, g, dx = sp[0], sp[1], sp[2]
        wu, wr = O.rk4(host_u[i], host_r[i], g, dx, dt, 3)
        assert rel(host(u[i]), wu, g) <= TOL and rel(host(rho[i]), wr, g) <= TOL, f"box {i}"
    bs.fill_ghosts(u)
    outs = bs.wave_rhs(u)
    for i, sp in enumerate(bs.spec):
        n, g, dx = sp[0], sp[1], sp[2]
        uf = host(u[i])
        assert rel(host(outs[i]), O.wave_rhs(uf, g, dx), g) <= TOL, f"box {i}"


def S_interior(a, g):
    return np.ascontiguousarray(a[g:-g, g:-g, g:-g])


def test_boxset_rejects_mismatched_fields():
    bs = S.BoxSet([((8, 8, 8), 2, 0.125), ((9, 8, 8), 2, 0.125)])
    u = bs.alloc()
    with pytest.raises(ValueError):
        bs.boxes(u[::-1])
    with pytest.raises(ValueError):
        bs.boxes(u[:1])
