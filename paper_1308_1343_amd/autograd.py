"""Backpropagation through RK4 steps of the wave equation with the library's
hand-written adjoint kernels (s4_rk4_adjoint_step), checkpointing every k
steps.

WaveRK4.apply(u0, rho0, c2, ghost, dx, dt, nsteps, k, ctx) returns
(u_T, rho_T) after nsteps classical RK4 steps on one periodic box.  Fields
are ghosted (z, y, x) float64 device tensors in one shared layout (compact
or padded views both work); only interior points carry values, and the
gradients it returns are zero on ghost points.  Forward keeps the state at
steps 0, k, 2k, ...; backward walks the segments in reverse, recomputes each
segment's step states from its checkpoint (one out-of-place step each) and
applies one adjoint step per forward step, accumulating dJ/dc2.  With c2 the
recomputing steps also keep their third stage state y_3, which the adjoint
step of dJ/dc2 reads, so that step need not form it again.  Every arithmetic
step runs in libsten4.
"""

from __future__ import annotations

import torch

from . import (S4_GRAPH, S4_OP_ADJOINT_STEP, S4_OP_RK4, S4_PERBOX, box_of, interior,
               s4_rk4, s4_rk4_adjoint_step, s4_rk4_adjoint_step_y3, s4_rk4_step_to, s4_rk4_step_to_y3,
               s4_workspace_size, workspace)


def _like(t: torch.Tensor, ghost: int, fill=0.0) -> torch.Tensor:
    """A fresh field with t's shape and strides (same layout, same box descriptor)."""
    out = torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)
    # empty_strided on a non-compact stride pattern allocates the full span
    out.fill_(fill)
    return out


def _copy_field(t: torch.Tensor) -> torch.Tensor:
    out = torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)
    out.copy_(t)
    return out


class WaveRK4(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u0, rho0, c2, ghost, dx, dt, nsteps, k, s4ctx):
        box = box_of(u0, ghost, dx)
        for t in (rho0,) + ((c2,) if c2 is not None else ()):
            if t.shape != u0.shape or t.stride() != u0.stride():
                raise ValueError("u0, rho0 and c2 must share one layout")
        ws = workspace(s4_workspace_size(box, S4_OP_RK4, S4_GRAPH), u0.device)
        # outputs carry interior values only; their ghosts are zero constants
        u, rho = _like(u0, ghost), _like(rho0, ghost)
        interior(u, ghost).copy_(interior(u0.detach(), ghost))
        interior(rho, ghost).copy_(interior(rho0.detach(), ghost))
        c2d = None if c2 is None else [c2.detach()]
        ckpts = []
        step = 0
        while step < nsteps:
            m = min(k, nsteps - step)
            ckpts.append((_copy_field(u), _copy_field(rho)))
            s4_rk4(s4ctx, box, [u], [rho], c2d, dt, m, S4_GRAPH, ws=ws)
            step += m
        fctx.meta = (ghost, dx, dt, nsteps, k, s4ctx, c2 is not None)
        fctx.ckpts = ckpts
        fctx.c2 = None if c2 is None else c2.detach()
        return u, rho

    @staticmethod
    def backward(fctx, gu, grho):
        ghost, dx, dt, nsteps, k, s4ctx, has_c2 = fctx.meta
        ckpts, c2 = fctx.ckpts, fctx.c2
        ref = ckpts[0][0] if ckpts else None
        if ref is None:
            return gu, grho, (None if not has_c2 else torch.zeros_like(c2)), None, None, None, None, None, None
        box = box_of(ref, ghost, dx)
        lam_u = _like(ref, ghost)
        lam_r = _like(ref, ghost)
        if gu is not None:
            interior(lam_u, ghost).copy_(interior(gu, ghost))
        if grho is not None:
            interior(lam_r, ghost).copy_(interior(grho, ghost))
        c2bar = _like(ref, ghost) if has_c2 else None
        ws_f = workspace(s4_workspace_size(box, S4_OP_RK4, S4_PERBOX), ref.device)
        ws_a = workspace(s4_workspace_size(box, S4_OP_ADJOINT_STEP), ref.device)
        def field():
            # only interior points are ever read
            return torch.empty_strided(ref.shape, ref.stride(), dtype=ref.dtype, device=ref.device)

        for si in reversed(range(len(ckpts))):
            s0 = si * k
            m = min(k, nsteps - s0)
            states, y3 = [ckpts[si]], []
            for _ in range(m - 1):
                # the next state, out of place (with c2: and this step's y_3)
                nu, nr = field(), field()
                if has_c2:
                    u3, r3 = field(), field()
                    s4_rk4_step_to_y3(s4ctx, box, states[-1][0], states[-1][1], c2, dt, nu, nr, u3, r3, ws=ws_f)
                    y3.append((u3, r3))
                else:
                    s4_rk4_step_to(s4ctx, box, states[-1][0], states[-1][1], c2, dt, nu, nr, ws=ws_f)
                states.append((nu, nr))
            for j in reversed(range(m)):
                un, rn = states.pop()
                if j < len(y3):
                    u3, r3 = y3.pop()
                    s4_rk4_adjoint_step_y3(s4ctx, box, un, rn, u3, r3, c2, dt, lam_u, lam_r, c2bar, ws=ws_a)
                else:
                    s4_rk4_adjoint_step(s4ctx, box, un, rn, c2, dt, lam_u, lam_r, c2bar, ws=ws_a)
        return lam_u, lam_r, c2bar, None, None, None, None, None, None


def wave_rk4(u0, rho0, c2, ghost, dx, dt, nsteps, k, s4ctx):
    return WaveRK4.apply(u0, rho0, c2, ghost, dx, dt, nsteps, k, s4ctx)
