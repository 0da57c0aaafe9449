"""Python binding of libsten4 (include/sten4.h): FP64 4th-order stencils, RK4
and its adjoint over the boxes of an AMR level, as HIP kernels for gfx950.

The functions named s4_* mirror the C ABI one to one and only marshal
arguments (torch tensors become device pointers, the current torch stream
becomes the hipStream_t).  Every arithmetic step runs in libsten4's kernels;
there is no fallback: importing this package fails loudly when the library
is not built.

A field of a box is a 3-D torch view (z, y, x) of float64 device memory
whose [0, 0, 0] element is the ghost corner (-g, -g, -g); `box_of` derives
the s4_box descriptor from such a view and `alloc_field` makes one with the
rows padded so that every interior row starts on a 128-byte boundary.
"""

from __future__ import annotations

import ctypes
import os

import torch  # loaded first: libsten4 then binds to the HIP runtime torch already loaded

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsten4.so")

S4_OK, S4_EINVAL, S4_EGHOST, S4_ELAYOUT, S4_EALIAS, S4_EDEVICE, S4_ENOMEM, S4_ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
S4_PERBOX, S4_BATCHED, S4_GRAPH = 0, 1, 2
S4_OP_FILL, S4_OP_WAVE_RHS, S4_OP_RK4, S4_OP_DERIV_MIXED, S4_OP_ADJOINT_RHS, S4_OP_ADJOINT_STEP = 1, 2, 3, 4, 5, 6
S4_OP_LEVEL_SYNC = 7
S4_WITH_C2 = 0x100  # ORed into S4_OP_RK4: the loop setup of RK4 calls that pass c^2
S4_SET_UNION, S4_SET_INTERSECTION, S4_SET_DIFFERENCE, S4_SET_SYMDIFF = 0, 1, 2, 3
SET_OPS = {"union": S4_SET_UNION, "intersection": S4_SET_INTERSECTION, "difference": S4_SET_DIFFERENCE,
           "symmetric_difference": S4_SET_SYMDIFF}
S4_SYNC_FULL, S4_SYNC_FACES = 0, 1
SYNC_SHAPES = {"full": S4_SYNC_FULL, "faces": S4_SYNC_FACES}
MODES = {"perbox": S4_PERBOX, "batched": S4_BATCHED, "graph": S4_GRAPH}

# the entry points include/sten4.h declares
EXPORTS = ("s4_create", "s4_destroy", "s4_last_error", "s4_check_boxes", "s4_workspace_size",
           "s4_fill_ghosts_periodic", "s4_wave_rhs", "s4_deriv_mixed", "s4_rk4", "s4_rk4_noalloc", "s4_wave_adjoint_rhs",
           "s4_rk4_step_to", "s4_rk4_step_to_y3", "s4_rk4_adjoint_step", "s4_rk4_adjoint_step_y3", "s4_tune", "s4_tune_scratch_size", "s4_get_choice", "s4_set_choice",
           "s4_tune_cache_lookup", "s4_set_online_tuning", "s4_online_simulate", "s4_copy",
           "s4_bset_from_boxes", "s4_bset_free", "s4_bset_op", "s4_bset_shift", "s4_bset_expand",
           "s4_bset_derivative", "s4_bset_info", "s4_bset_keys", "s4_bset_boxes", "s4_bset_contains",
           "s4_bset_equal", "s4_level_create", "s4_level_destroy", "s4_level_info", "s4_level_pieces",
           "s4_level_workspace_size", "s4_level_sync", "s4_level_rk4", "s4_level_choice")


class S4Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32), ("stride", ctypes.c_int64 * 3),
                ("dx", ctypes.c_double * 3), ("level", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def __repr__(self):
        return (f"S4Box(n={tuple(self.n)}, ghost={self.ghost}, stride={tuple(self.stride)}, "
                f"dx={tuple(self.dx)}, level={self.level})")


class Sten4Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sten4 error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_1308_1343_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    BP = ctypes.POINTER(S4Box)
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.s4_create.argtypes = [i, ctypes.POINTER(vp)]
    L.s4_destroy.argtypes = [vp]
    L.s4_destroy.restype = None
    L.s4_last_error.restype = ctypes.c_char_p
    L.s4_check_boxes.argtypes = [BP, i, i]
    L.s4_workspace_size.argtypes = [BP, i, i, i, ctypes.POINTER(sz)]
    L.s4_tune_scratch_size.argtypes = [BP, i, i, ctypes.POINTER(sz)]
    L.s4_fill_ghosts_periodic.argtypes = [vp, BP, i, PP, vp]
    L.s4_wave_rhs.argtypes = [vp, BP, i, PP, PP, PP, vp]
    L.s4_deriv_mixed.argtypes = [vp, BP, i, PP, ctypes.POINTER(d), PP, vp]
    L.s4_rk4.argtypes = [vp, BP, i, PP, PP, PP, d, i, i, vp, sz, vp]
    L.s4_rk4_noalloc.argtypes = [vp, BP, i, PP, PP, PP, d, i, i, vp]
    L.s4_wave_adjoint_rhs.argtypes = [vp, BP, i, PP, PP, PP, PP, PP, vp]
    L.s4_rk4_adjoint_step.argtypes = [vp, BP, vp, vp, vp, d, vp, vp, vp, vp, sz, vp]
    L.s4_rk4_step_to.argtypes = [vp, BP, vp, vp, vp, d, vp, vp, vp, sz, vp]
    L.s4_rk4_step_to_y3.argtypes = [vp, BP, vp, vp, vp, d, vp, vp, vp, vp, vp, sz, vp]
    L.s4_rk4_adjoint_step_y3.argtypes = [vp, BP, vp, vp, vp, vp, vp, d, vp, vp, vp, vp, sz, vp]
    L.s4_tune.argtypes = [vp, i, BP, i, i, vp, sz, vp]
    L.s4_get_choice.argtypes = [vp, i, BP, i, ctypes.POINTER(i)]
    L.s4_set_choice.argtypes = [vp, i, BP, i, i]
    L.s4_tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i, BP, i, i, ctypes.POINTER(i)]
    L.s4_copy.argtypes = [vp, vp, vp, sz, vp]
    L.s4_set_online_tuning.argtypes = [vp, i, d, ctypes.c_uint64]
    L.s4_online_simulate.argtypes = [i, BP, i, ctypes.POINTER(d), i, d, d, ctypes.c_uint64, i, i,
                                     ctypes.POINTER(i)]
    I64P = ctypes.POINTER(ctypes.c_int64)
    L.s4_bset_from_boxes.argtypes = [i, I64P, I64P, ctypes.c_int64, ctypes.POINTER(vp)]
    L.s4_bset_free.argtypes = [vp]
    L.s4_bset_free.restype = None
    L.s4_bset_op.argtypes = [i, vp, vp, ctypes.POINTER(vp)]
    L.s4_bset_shift.argtypes = [vp, I64P, ctypes.POINTER(vp)]
    L.s4_bset_expand.argtypes = [vp, I64P, I64P, ctypes.POINTER(vp)]
    L.s4_bset_derivative.argtypes = [vp, i, ctypes.POINTER(vp)]
    L.s4_bset_info.argtypes = [vp, I64P]
    L.s4_bset_keys.argtypes = [vp, I64P, ctypes.c_int64, I64P]
    L.s4_bset_boxes.argtypes = [vp, I64P, I64P, ctypes.c_int64, I64P]
    L.s4_bset_contains.argtypes = [vp, I64P, ctypes.POINTER(i)]
    L.s4_bset_equal.argtypes = [vp, vp, ctypes.POINTER(i)]
    L.s4_level_create.argtypes = [BP, I64P, i, I64P, i, i, ctypes.POINTER(vp)]
    L.s4_level_destroy.argtypes = [vp]
    L.s4_level_destroy.restype = None
    L.s4_level_info.argtypes = [vp, I64P]
    L.s4_level_pieces.argtypes = [vp, I64P, ctypes.c_int64, I64P]
    L.s4_level_workspace_size.argtypes = [vp, i, ctypes.POINTER(sz)]
    L.s4_level_sync.argtypes = [vp, vp, PP, vp, sz, vp]
    L.s4_level_rk4.argtypes = [vp, vp, PP, PP, PP, d, i, i, vp, sz, vp]
    L.s4_level_choice.argtypes = [vp, vp, ctypes.POINTER(i)]
    for name in EXPORTS:
        if name not in ("s4_destroy", "s4_last_error", "s4_bset_free", "s4_level_destroy"):
            getattr(L, name).restype = i
    _lib = L
    return L


def s4_last_error() -> str:
    return lib().s4_last_error().decode()


def _check(rc):
    if rc != S4_OK:
        raise Sten4Error(rc, s4_last_error())
    return rc


# --------------------------------------------------------------------------- layout helpers

def make_box(n, ghost, stride, dx, level=0) -> S4Box:
    b = S4Box()
    b.n[:] = [int(v) for v in n]
    b.ghost = int(ghost)
    b.stride[:] = [int(v) for v in stride]
    dx = (dx, dx, dx) if isinstance(dx, (int, float)) else dx
    b.dx[:] = [float(v) for v in dx]
    b.level = int(level)
    b.reserved = 0
    return b


def box_of(t: torch.Tensor, ghost: int, dx, level: int = 0) -> S4Box:
    """Descriptor of a (z, y, x) view whose [0,0,0] element is the ghost corner."""
    if t.dim() != 3:
        raise ValueError("a box field is a 3-D (z, y, x) view")
    nz, ny, nx = (s - 2 * ghost for s in t.shape)
    sz, sy, sx = t.stride()
    return make_box((nx, ny, nz), ghost, (sx, sy, sz), dx, level)


def alloc_field(n, ghost, device="cuda", pad=True, fill=None) -> torch.Tensor:
    """Ghosted (z, y, x) float64 view of fresh device memory.  With pad=True the
    row stride is a multiple of 16 elements and the buffer is offset so that
    (i=0, j, k) starts a 128-byte line for every row (the aligned, padded
    layout of the paper's LoopControl, Sec. III-A)."""
    nx, ny, nz = (int(v) for v in n)
    g = int(ghost)
    sy = nx + 2 * g
    off = 0
    if pad:
        sy = (sy + 15) // 16 * 16
        off = (16 - g % 16) % 16
    sz = sy * (ny + 2 * g)
    buf = torch.empty(off + sz * (nz + 2 * g), dtype=torch.float64, device=device)
    if fill is not None:
        buf.fill_(fill)
    return buf[off:].as_strided((nz + 2 * g, ny + 2 * g, nx + 2 * g), (sz, sy, 1))


def interior(t: torch.Tensor, ghost: int) -> torch.Tensor:
    g = ghost
    return t[g:t.shape[0] - g, g:t.shape[1] - g, g:t.shape[2] - g]


def _boxes(boxes):
    if isinstance(boxes, S4Box):
        boxes = [boxes]
    arr = (S4Box * len(boxes))(*boxes)
    return arr, len(boxes)


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[0 if t is None else _ptr(t) for t in ts])


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if t.dtype != torch.float64 and t.dtype != torch.uint8:
        raise TypeError("fields must be float64")
    if not t.is_cuda:
        raise TypeError("fields must be device tensors")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# --------------------------------------------------------------------------- context

class Context:
    """An s4_ctx bound to one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().s4_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            lib().s4_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def s4_create(device: int = 0) -> Context:
    return Context(device)


def s4_destroy(ctx: Context):
    ctx.close()


# --------------------------------------------------------------------------- entry points

def s4_check_boxes(boxes, op) -> int:
    arr, n = _boxes(boxes)
    return lib().s4_check_boxes(arr, n, op)


def s4_workspace_size(boxes, op, mode=S4_GRAPH) -> int:
    arr, n = _boxes(boxes)
    out = ctypes.c_size_t()
    _check(lib().s4_workspace_size(arr, n, op, mode, ctypes.byref(out)))
    return out.value


def s4_tune_scratch_size(boxes, op) -> int:
    arr, n = _boxes(boxes)
    out = ctypes.c_size_t()
    _check(lib().s4_tune_scratch_size(arr, n, op, ctypes.byref(out)))
    return out.value


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """A 256-byte aligned device buffer (torch's allocator aligns blocks to 512 bytes)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def s4_fill_ghosts_periodic(ctx, boxes, f, stream=None):
    arr, n = _boxes(boxes)
    _check(lib().s4_fill_ghosts_periodic(ctx.handle, arr, n, _ptrs(f), _stream(stream)))


def s4_wave_rhs(ctx, boxes, u, c2, rho_t, stream=None):
    arr, n = _boxes(boxes)
    _check(lib().s4_wave_rhs(ctx.handle, arr, n, _ptrs(u), None if c2 is None else _ptrs(c2),
                             _ptrs(rho_t), _stream(stream)))


def s4_deriv_mixed(ctx, box, g, A, out, stream=None):
    arr, _ = _boxes(box)
    A9 = (ctypes.c_double * 9)(*[float(v) for v in torch.as_tensor(A, dtype=torch.float64).reshape(9).tolist()])
    _check(lib().s4_deriv_mixed(ctx.handle, arr, len(g), _ptrs(g), A9, _ptrs(out), _stream(stream)))


def s4_rk4(ctx, boxes, u, rho, c2, dt, nsteps, mode=S4_GRAPH, ws=None, stream=None):
    arr, n = _boxes(boxes)
    mode = MODES.get(mode, mode)
    if ws is None:
        ws = workspace(s4_workspace_size(boxes, S4_OP_RK4, mode), u[0].device)
    _check(lib().s4_rk4(ctx.handle, arr, n, _ptrs(u), _ptrs(rho), None if c2 is None else _ptrs(c2),
                        float(dt), int(nsteps), int(mode), _ptr(ws), ws.numel(), _stream(stream)))
    return ws


S4_NOALLOC_SCRATCH_BYTES = 128 << 20


def s4_rk4_noalloc(ctx, boxes, u, rho, c2, dt, nsteps, mode=S4_BATCHED, stream=None):
    """s4_rk4 on the library's own scratch array (no workspace, no allocation)."""
    arr, n = _boxes(boxes)
    mode = MODES.get(mode, mode)
    _check(lib().s4_rk4_noalloc(ctx.handle, arr, n, _ptrs(u), _ptrs(rho), None if c2 is None else _ptrs(c2),
                                float(dt), int(nsteps), int(mode), _stream(stream)))


def s4_rk4_step_to(ctx, box, u_in, rho_in, c2, dt, u_out, rho_out, ws=None, stream=None):
    arr, _ = _boxes(box)
    if ws is None:
        ws = workspace(s4_workspace_size(box, S4_OP_RK4, S4_PERBOX), u_in.device)
    _check(lib().s4_rk4_step_to(ctx.handle, arr, _ptr(u_in), _ptr(rho_in), _ptr(c2), float(dt), _ptr(u_out),
                                _ptr(rho_out), _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def s4_rk4_step_to_y3(ctx, box, u_in, rho_in, c2, dt, u_out, rho_out, u3_out, rho3_out, ws=None, stream=None):
    arr, _ = _boxes(box)
    if ws is None:
        ws = workspace(s4_workspace_size(box, S4_OP_RK4, S4_PERBOX), u_in.device)
    _check(lib().s4_rk4_step_to_y3(ctx.handle, arr, _ptr(u_in), _ptr(rho_in), _ptr(c2), float(dt), _ptr(u_out),
                                   _ptr(rho_out), _ptr(u3_out), _ptr(rho3_out), _ptr(ws), ws.numel(),
                                   _stream(stream)))
    return ws


def s4_wave_adjoint_rhs(ctx, boxes, lu, lrho, c2, out_u, out_rho, stream=None):
    arr, n = _boxes(boxes)
    _check(lib().s4_wave_adjoint_rhs(ctx.handle, arr, n, _ptrs(lu), _ptrs(lrho),
                                     None if c2 is None else _ptrs(c2), _ptrs(out_u), _ptrs(out_rho),
                                     _stream(stream)))


def s4_rk4_adjoint_step(ctx, box, u_n, rho_n, c2, dt, lam_u, lam_rho, c2_bar, ws=None, stream=None):
    arr, _ = _boxes(box)
    if ws is None:
        ws = workspace(s4_workspace_size(box, S4_OP_ADJOINT_STEP), u_n.device)
    _check(lib().s4_rk4_adjoint_step(ctx.handle, arr, _ptr(u_n), _ptr(rho_n), _ptr(c2), float(dt), _ptr(lam_u),
                                     _ptr(lam_rho), _ptr(c2_bar), _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def s4_rk4_adjoint_step_y3(ctx, box, u_n, rho_n, u3, rho3, c2, dt, lam_u, lam_rho, c2_bar, ws=None, stream=None):
    arr, _ = _boxes(box)
    if ws is None:
        ws = workspace(s4_workspace_size(box, S4_OP_ADJOINT_STEP), u_n.device)
    _check(lib().s4_rk4_adjoint_step_y3(ctx.handle, arr, _ptr(u_n), _ptr(rho_n), _ptr(u3), _ptr(rho3), _ptr(c2),
                                        float(dt), _ptr(lam_u), _ptr(lam_rho), _ptr(c2_bar), _ptr(ws), ws.numel(),
                                        _stream(stream)))
    return ws


def s4_tune(ctx, op, boxes, flags=0, scratch=None, stream=None):
    arr, n = _boxes(boxes)
    if scratch is None:
        scratch = workspace(s4_tune_scratch_size(boxes, op))
    _check(lib().s4_tune(ctx.handle, op, arr, n, int(flags), _ptr(scratch), scratch.numel(), _stream(stream)))


CHOICE_KEYS = ("kernel_op", "tile_x", "tile_y", "z_chunk", "threads", "tuned", "candidate", "ncandidates")


def s4_get_choice(ctx, op, boxes) -> dict:
    arr, n = _boxes(boxes)
    out = (ctypes.c_int * 8)()
    _check(lib().s4_get_choice(ctx.handle, op, arr, n, out))
    return dict(zip(CHOICE_KEYS, list(out)))


def s4_level_choice(ctx, level) -> dict:
    """The tile choice s4_level_rk4 uses on this level (keys as s4_get_choice)."""
    out = (ctypes.c_int * 8)()
    _check(lib().s4_level_choice(ctx.handle, level.handle, out))
    return dict(zip(CHOICE_KEYS, list(out)))


def s4_set_choice(ctx, op, boxes, candidate):
    arr, n = _boxes(boxes)
    _check(lib().s4_set_choice(ctx.handle, op, arr, n, int(candidate)))


def s4_tune_cache_lookup(path, device, op, boxes, level=0) -> int:
    """Candidate a context on `device` would take from the cache file at
    `path` for this loop setup (level 0: the boxes, 1: a level, 2: a wide
    level), or -1 (host only)."""
    arr, n = _boxes(boxes)
    out = ctypes.c_int()
    _check(lib().s4_tune_cache_lookup(os.fsencode(path), device.encode(), int(op), arr, n, int(level),
                                      ctypes.byref(out)))
    return out.value


def s4_set_online_tuning(ctx, enable=True, restart_prob=0.02, seed=1):
    _check(lib().s4_set_online_tuning(ctx.handle, int(bool(enable)), float(restart_prob), int(seed)))


def s4_online_simulate(op, boxes, cost, noise=0.0, restart_prob=0.02, seed=1, lag=1, ncalls=100):
    """Trace of candidates the on-line tuner picks against synthetic costs (host only)."""
    arr, n = _boxes(boxes)
    c = (ctypes.c_double * len(cost))(*[float(v) for v in cost])
    trace = (ctypes.c_int * ncalls)()
    _check(lib().s4_online_simulate(op, arr, n, c, len(cost), float(noise), float(restart_prob), int(seed),
                                    int(lag), int(ncalls), trace))
    return list(trace)


def s4_copy(ctx, dst, src, nbytes=None, stream=None):
    nb = dst.numel() * dst.element_size() if nbytes is None else int(nbytes)
    _check(lib().s4_copy(ctx.handle, _ptr(dst), _ptr(src), nb, _stream(stream)))


# --------------------------------------------------------------------------- bboxsets and levels

def _i64(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * max(1, len(vals)))(*vals)


class BSet:
    """Owner of an s4_bset handle (freed with the object)."""

    def __init__(self, handle, dim):
        self.handle = handle
        self.dim = dim
        self._free = lib().s4_bset_free  # kept: module globals may be gone at interpreter exit

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._free(h)
            self.handle = None


def _new_bset(fn, dim, *args):
    h = ctypes.c_void_p()
    _check(fn(*args, ctypes.byref(h)))
    return BSet(h, dim)


def s4_bset_from_boxes(dim, boxes) -> BSet:
    """boxes: iterable of (lo, hi) half-open integer boxes of `dim` coordinates."""
    boxes = list(boxes)
    lo = _i64([c for b in boxes for c in b[0]])
    hi = _i64([c for b in boxes for c in b[1]])
    return _new_bset(lib().s4_bset_from_boxes, dim, int(dim), lo, hi, len(boxes))


def s4_bset_op(op, a: BSet, b: BSet) -> BSet:
    return _new_bset(lib().s4_bset_op, a.dim, int(SET_OPS.get(op, op)), a.handle, b.handle)


def s4_bset_shift(a: BSet, v) -> BSet:
    return _new_bset(lib().s4_bset_shift, a.dim, a.handle, _i64(v))


def s4_bset_expand(a: BSet, lo, hi) -> BSet:
    return _new_bset(lib().s4_bset_expand, a.dim, a.handle, _i64(lo), _i64(hi))


def s4_bset_derivative(a: BSet, axis) -> BSet:
    return _new_bset(lib().s4_bset_derivative, a.dim, a.handle, int(axis))


def s4_bset_info(a: BSet) -> dict:
    out = (ctypes.c_int64 * 4)()
    _check(lib().s4_bset_info(a.handle, out))
    return dict(zip(("dim", "points", "keys", "boxes"), list(out)))


def s4_bset_keys(a: BSet) -> list:
    cnt = ctypes.c_int64()
    _check(lib().s4_bset_keys(a.handle, None, 0, ctypes.byref(cnt)))
    out = (ctypes.c_int64 * max(1, cnt.value * a.dim))()
    _check(lib().s4_bset_keys(a.handle, out, cnt.value, ctypes.byref(cnt)))
    return [tuple(out[k * a.dim:(k + 1) * a.dim]) for k in range(cnt.value)]


def s4_bset_boxes(a: BSet) -> list:
    cnt = ctypes.c_int64()
    _check(lib().s4_bset_boxes(a.handle, None, None, 0, ctypes.byref(cnt)))
    lo = (ctypes.c_int64 * max(1, cnt.value * a.dim))()
    hi = (ctypes.c_int64 * max(1, cnt.value * a.dim))()
    _check(lib().s4_bset_boxes(a.handle, lo, hi, cnt.value, ctypes.byref(cnt)))
    d = a.dim
    return [(tuple(lo[k * d:(k + 1) * d]), tuple(hi[k * d:(k + 1) * d])) for k in range(cnt.value)]


def s4_bset_contains(a: BSet, p) -> bool:
    out = ctypes.c_int()
    _check(lib().s4_bset_contains(a.handle, _i64(p), ctypes.byref(out)))
    return bool(out.value)


def s4_bset_equal(a: BSet, b: BSet) -> bool:
    out = ctypes.c_int()
    _check(lib().s4_bset_equal(a.handle, b.handle, ctypes.byref(out)))
    return bool(out.value)


class Level:
    """Owner of an s4_level handle (freed with the object) and the boxes it was built for."""

    def __init__(self, handle, boxes):
        self.handle = handle
        self.boxes = boxes
        self._free = lib().s4_level_destroy

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._free(h)
            self.handle = None


def s4_level_create(boxes, lo, domain, width, shape="faces") -> Level:
    """boxes: s4_box descriptors; lo: global (x, y, z) origin of each interior;
    domain: periodic extents (0 = open axis)."""
    arr, n = _boxes(boxes)
    h = ctypes.c_void_p()
    _check(lib().s4_level_create(arr, _i64([c for l in lo for c in l]), n, _i64(domain), int(width),
                                 int(SYNC_SHAPES.get(shape, shape)), ctypes.byref(h)))
    return Level(h, list(boxes) if not isinstance(boxes, S4Box) else [boxes])


def s4_level_destroy(level: Level):
    level.__del__()


def s4_level_info(level: Level) -> dict:
    out = (ctypes.c_int64 * 7)()
    _check(lib().s4_level_info(level.handle, out))
    return dict(zip(("boxes", "pieces", "filled", "uncovered", "points", "width", "shape"), list(out)))


def s4_level_pieces(level: Level) -> list:
    """[(dst, src, dst start xyz, src start xyz, extent xyz)] in box-local interior coordinates."""
    cnt = ctypes.c_int64()
    _check(lib().s4_level_pieces(level.handle, None, 0, ctypes.byref(cnt)))
    out = (ctypes.c_int64 * max(1, 11 * cnt.value))()
    _check(lib().s4_level_pieces(level.handle, out, cnt.value, ctypes.byref(cnt)))
    res = []
    for k in range(cnt.value):
        o = out[11 * k:11 * k + 11]
        res.append((o[0], o[1], tuple(o[2:5]), tuple(o[5:8]), tuple(o[8:11])))
    return res


def s4_level_workspace_size(level: Level, op) -> int:
    out = ctypes.c_size_t()
    _check(lib().s4_level_workspace_size(level.handle, int(op), ctypes.byref(out)))
    return out.value


def s4_level_sync(ctx, level: Level, f, ws=None, stream=None):
    if ws is None:
        ws = workspace(s4_level_workspace_size(level, S4_OP_LEVEL_SYNC), f[0].device)
    _check(lib().s4_level_sync(ctx.handle, level.handle, _ptrs(f), _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def s4_level_rk4(ctx, level: Level, u, rho, c2, dt, nsteps, mode=S4_GRAPH, ws=None, stream=None):
    mode = MODES.get(mode, mode)
    if ws is None:
        ws = workspace(s4_level_workspace_size(level, S4_OP_RK4), u[0].device)
    _check(lib().s4_level_rk4(ctx.handle, level.handle, _ptrs(u), _ptrs(rho), None if c2 is None else _ptrs(c2),
                              float(dt), int(nsteps), int(mode), _ptr(ws), ws.numel(), _stream(stream)))
    return ws


lib()  # fail at import when the HIP library is missing: there is no other implementation

from .tensors import BoxSet, default_context, deriv_mixed, fill_ghosts, rk4, wave_rhs  # noqa: E402
