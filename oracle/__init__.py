"""numpy access to the plain-C FP64 oracle (liboracle4.so, built from oracle4.c).

TEST INFRASTRUCTURE ONLY.  Imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the HIP library or its binding.

Every field is a float64 numpy array of shape (nz+2g, ny+2g, nx+2g), C order,
x fastest: one box with its ghost zones, interior at [g:-g, g:-g, g:-g].
Axis numbers follow the grid: 0 = x (last array dimension), 1 = y, 2 = z.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        # ORACLE4_LIB lets the mutation test load a deliberately broken build
        path = os.environ.get("ORACLE4_LIB") or os.path.join(_HERE, "liboracle4.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.o4_num_threads.restype = i
        L.o4_set_num_threads.argtypes = [i]
        L.o4_fill_ghosts_periodic.argtypes = [i, i, i, i, P]
        L.o4_d1.argtypes = [i, i, i, i, i, d, P, P]
        L.o4_d2.argtypes = [i, i, i, i, i, d, P, P]
        L.o4_dmix.argtypes = [i, i, i, i, i, i, d, d, P, P]
        L.o4_laplacian.argtypes = [i, i, i, i, P, P, P]
        L.o4_wave_rhs.argtypes = [i, i, i, i, P, P, P, P]
        L.o4_rk4.argtypes = [i, i, i, i, P, P, d, i, P, P]
        L.o4_deriv_mixed.argtypes = [i, i, i, i, P, P, P, P]
        L.o4_wave_adjoint_rhs.argtypes = [i, i, i, i, P, P, P, P, P, P]
        L.o4_rk4_adjoint_step.argtypes = [i, i, i, i, P, P, d, P, P, P, P, P]
        L.o4_wave_loss_grad.argtypes = [i, i, i, i, P, P, d, i, P, P, P, P, P, P]
        L.o4_wave_loss_grad.restype = d
        _LIB = L
    return _LIB


def num_threads() -> int:
    return lib().o4_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (timing only; results are independent of it)."""
    lib().o4_set_num_threads(int(n))


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dx(dx):
    if np.isscalar(dx):
        dx = (dx, dx, dx)
    return (ctypes.c_double * 3)(*[float(v) for v in dx])


def dims(a, g):
    """(nx, ny, nz) interior sizes of a ghosted array."""
    nz, ny, nx = a.shape
    return nx - 2 * g, ny - 2 * g, nz - 2 * g


def embed(inner, g, value=0.0):
    """Ghosted array holding `inner` in its interior and `value` in its ghosts."""
    nz, ny, nx = inner.shape
    a = np.full((nz + 2 * g, ny + 2 * g, nx + 2 * g), value, dtype=np.float64)
    a[g:g + nz, g:g + ny, g:g + nx] = inner
    return a


def interior(a, g):
    return a[g:a.shape[0] - g, g:a.shape[1] - g, g:a.shape[2] - g]


def fill_ghosts_periodic(a, g):
    """Periodic ghost fill in place (axes x, then y, then z)."""
    lib().o4_fill_ghosts_periodic(*dims(a, g), g, _p(a))
    return a


def d1(f, g, axis, h):
    out = np.zeros_like(f)
    lib().o4_d1(*dims(f, g), g, axis, h, _p(f), _p(out))
    return out


def d2(f, g, axis, h):
    out = np.zeros_like(f)
    lib().o4_d2(*dims(f, g), g, axis, h, _p(f), _p(out))
    return out


def dmix(f, g, a, b, ha, hb):
    out = np.zeros_like(f)
    lib().o4_dmix(*dims(f, g), g, a, b, ha, hb, _p(f), _p(out))
    return out


def laplacian(f, g, dx):
    out = np.zeros_like(f)
    lib().o4_laplacian(*dims(f, g), g, _dx(dx), _p(f), _p(out))
    return out


def wave_rhs(u, g, dx, c2=None):
    """rho_t = c^2 L u on interior points (u's ghosts must be filled)."""
    out = np.zeros_like(u)
    lib().o4_wave_rhs(*dims(u, g), g, _dx(dx), _p(u), _p(c2), _p(out))
    return out


def rk4(u, rho, g, dx, dt, nsteps, c2=None):
    """nsteps classical RK4 steps of the wave equation with periodic ghost fills.
    Returns new arrays (u ghosts filled as of the last stage fill)."""
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    rho = np.array(rho, dtype=np.float64, copy=True, order="C")
    lib().o4_rk4(*dims(u, g), g, _dx(dx), _p(c2), float(dt), int(nsteps), _p(u), _p(rho))
    return u, rho


def deriv_mixed(f, g, dx, A):
    """out = sum_a D2_a f + sum_{a<b} D_ab f + sum_ab A_ab D1_a f D1_b f (ghosts of f filled)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(9))
    out = np.zeros_like(f)
    lib().o4_deriv_mixed(*dims(f, g), g, _dx(dx), _p(A), _p(f), _p(out))
    return out


def wave_adjoint_rhs(lu, lrho, g, dx, c2=None):
    """F^T(lu, lrho) = (L_p(c^2 lrho), lu) for periodic boxes."""
    ou = np.zeros_like(lu)
    orr = np.zeros_like(lu)
    lib().o4_wave_adjoint_rhs(*dims(lu, g), g, _dx(dx), _p(lu), _p(lrho), _p(c2), _p(ou), _p(orr))
    return ou, orr


def rk4_adjoint_step(u_n, rho_n, lam_u, lam_rho, g, dx, dt, c2=None, c2bar=None):
    """One backward RK4 step: returns (lam_u_n, lam_rho_n, c2bar) (new arrays)."""
    lu = np.array(lam_u, dtype=np.float64, copy=True, order="C")
    lr = np.array(lam_rho, dtype=np.float64, copy=True, order="C")
    if c2 is not None:
        c2bar = np.zeros_like(lu) if c2bar is None else np.array(c2bar, dtype=np.float64, copy=True, order="C")
    else:
        c2bar = None
    lib().o4_rk4_adjoint_step(*dims(lu, g), g, _dx(dx), _p(c2), float(dt),
                              _p(np.ascontiguousarray(u_n)), _p(np.ascontiguousarray(rho_n)),
                              _p(lu), _p(lr), _p(c2bar))
    return lu, lr, c2bar


def wave_loss_grad(u0, rho0, c2, u_target, g, dx, dt, nsteps):
    """J = 1/2 sum (u_N - u_target)^2 and its gradient (store-all backward).
    Returns (J, dJ/du0, dJ/drho0, dJ/dc2)."""
    ub = np.zeros_like(u0)
    rb = np.zeros_like(u0)
    cb = np.zeros_like(u0) if c2 is not None else None
    J = lib().o4_wave_loss_grad(*dims(u0, g), g, _dx(dx), _p(c2), float(dt), int(nsteps),
                                _p(u0), _p(rho0), _p(u_target), _p(ub), _p(rb), _p(cb))
    return J, ub, rb, cb
