"""Tensor-level calls: wave_rhs, rk4, deriv_mixed and BoxSet.

Each call derives the s4_box descriptors from the tensor views, takes the
device's default context and a workspace, and calls the C ABI; nothing here
computes field values.  A field is a ghosted (z, y, x) float64 view of
device memory whose [0, 0, 0] element is the ghost corner (alloc_field makes
one with aligned, padded rows).

Workspaces: rk4 keeps one per device, grown on demand and reused, so that
the graph captured for a loop setup (keyed on the workspace address) is
replayed by later calls.  Calls that may overlap on different streams must
pass their own `ws`.
"""

from __future__ import annotations

import threading

import torch

from . import (S4_OP_RK4, Context, S4Box, alloc_field, box_of, s4_deriv_mixed, s4_fill_ghosts_periodic,
               s4_rk4, s4_wave_rhs, s4_workspace_size, workspace)

_lock = threading.Lock()
_ctx: dict = {}
_ws: dict = {}


def _device_index(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise TypeError("fields must be device tensors")
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def default_context(device: int | None = None) -> Context:
    """The context this module uses on `device` (created on first use)."""
    dev = torch.cuda.current_device() if device is None else int(device)
    with _lock:
        if dev not in _ctx:
            _ctx[dev] = Context(dev)
        return _ctx[dev]


def _workspace(dev: int, nbytes: int) -> torch.Tensor:
    with _lock:
        w = _ws.get(dev)
        if w is None or w.numel() < nbytes:
            w = workspace(nbytes, f"cuda:{dev}")
            _ws[dev] = w
        return w


def _like(u: torch.Tensor, ghost: int, fill=None) -> torch.Tensor:
    n = tuple(s - 2 * ghost for s in reversed(u.shape))
    return alloc_field(n, ghost, device=u.device, fill=fill)


def wave_rhs(u, ghost, dx, c2=None, out=None, ctx=None, stream=None):
    """rho_t = c^2 L u at the interior points of one box (u's ghosts filled;
    c2 None means c = 1).  Returns `out` (a new field like u if None); its
    ghosts are not written."""
    ctx = ctx or default_context(_device_index(u))
    out = _like(u, ghost, 0.0) if out is None else out
    b = box_of(u, ghost, dx)
    s4_wave_rhs(ctx, b, [u], None if c2 is None else [c2], [out], stream)
    return out


def rk4(u, rho, ghost, dx, dt, nsteps, c2=None, mode="graph", ctx=None, ws=None, stream=None):
    """nsteps classical RK4 steps of the wave equation on one periodic box,
    in place at interior points.  Returns (u, rho)."""
    dev = _device_index(u)
    ctx = ctx or default_context(dev)
    b = box_of(u, ghost, dx)
    if ws is None:
        ws = _workspace(dev, s4_workspace_size(b, S4_OP_RK4, 2))
    s4_rk4(ctx, b, [u], [rho], None if c2 is None else [c2], dt, nsteps, mode, ws=ws, stream=stream)
    return u, rho


def deriv_mixed(gs, A, ghost, dx, out=None, ctx=None, stream=None):
    """For every field g of gs (ghosts filled, edges included):
    sum_a D2_a g + sum_{a<b} D_ab g + sum_ab A_ab D1_a g D1_b g at interior
    points.  All fields share one box layout.  Returns the list of outputs."""
    gs = list(gs)
    ctx = ctx or default_context(_device_index(gs[0]))
    b = box_of(gs[0], ghost, dx)
    out = [_like(gs[0], ghost, 0.0) for _ in gs] if out is None else list(out)
    s4_deriv_mixed(ctx, b, gs, A, out, stream)
    return out


def fill_ghosts(f, ghost, ctx=None, stream=None):
    """Periodic ghost fill of one box field (each box its own neighbour)."""
    ctx = ctx or default_context(_device_index(f))
    s4_fill_ghosts_periodic(ctx, box_of(f, ghost, 1.0), [f], stream)
    return f


class BoxSet:
    """The boxes of one bboxset, each with its own interior size, ghost width,
    grid spacing and refinement level; operations run over all boxes in one
    call (in S4_BATCHED or S4_GRAPH mode, one persistent launch per pass).

    boxes: iterable of dicts {"n": (nx, ny, nz), "ghost": g, "dx": h or
    (hx, hy, hz), "level": l} or of (n, ghost, dx[, level]) tuples."""

    def __init__(self, boxes, device=None):
        self.spec = []
        for bx in boxes:
            if isinstance(bx, dict):
                n, g, dx, lev = bx["n"], bx["ghost"], bx["dx"], bx.get("level", 0)
            else:
                n, g, dx = bx[0], bx[1], bx[2]
                lev = bx[3] if len(bx) > 3 else 0
            self.spec.append((tuple(int(v) for v in n), int(g), dx, int(lev)))
        if not self.spec:
            raise ValueError("a BoxSet needs at least one box")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.ctx = default_context(self.device)
        self._ws = None

    def __len__(self):
        return len(self.spec)

    def alloc(self, fill=0.0):
        """One field per box, in the padded layout."""
        return [alloc_field(n, g, device=f"cuda:{self.device}", fill=fill) for n, g, _, _ in self.spec]

    def boxes(self, fields) -> list[S4Box]:
        """Descriptors of the boxes laid out as `fields` (one per box)."""
        fields = list(fields)
        if len(fields) != len(self.spec):
            raise ValueError(f"{len(fields)} fields for {len(self.spec)} boxes")
        out = []
        for t, (n, g, dx, lev) in zip(fields, self.spec):
            b = box_of(t, g, dx, lev)
            if tuple(b.n) != n:
                raise ValueError(f"field of interior {tuple(b.n)} for a box of {n}")
            out.append(b)
        return out

    def fill_ghosts(self, f, stream=None):
        s4_fill_ghosts_periodic(self.ctx, self.boxes(f), list(f), stream)
        return f

    def wave_rhs(self, u, c2=None, out=None, stream=None):
        out = [_like(t, g, 0.0) for t, (_, g, _, _) in zip(u, self.spec)] if out is None else list(out)
        s4_wave_rhs(self.ctx, self.boxes(u), list(u), None if c2 is None else list(c2), out, stream)
        return out

    def rk4(self, u, rho, dt, nsteps, c2=None, mode="graph", ws=None, stream=None):
        """nsteps RK4 steps of every box (each box its own periodic neighbour)."""
        b = self.boxes(u)
        if ws is None:
            need = s4_workspace_size(b, S4_OP_RK4, 2)
            if self._ws is None or self._ws.numel() < need:
                self._ws = workspace(need, f"cuda:{self.device}")
            ws = self._ws
        s4_rk4(self.ctx, b, list(u), list(rho), None if c2 is None else list(c2), dt, nsteps, mode, ws=ws,
               stream=stream)
        return u, rho
