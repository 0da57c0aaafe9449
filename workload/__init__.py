"""Seeded synthetic inputs for the stencil workloads.

Both the CPU oracle (in tests) and the HIP path receive their inputs from
this module as identical host float64 bytes; the HIP side copies them to
the device.  The module holds none of the method's arithmetic (no finite
differences, no time stepping, no adjoint): only random draws and the
closed-form initial fields (sine modes, a Gaussian pulse) that the method is
applied to.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014; the form
popularised by Vigna).  Its state advances by the odd constant GAMMA and
each output is a fixed bijective mix of the state, so the i-th output of a
stream is mix(key + (i + 1) * GAMMA): the generator is counter based and can
be evaluated for a whole array at once.  A double in [0, 1) takes the top 53
bits: (z >> 11) * 2**-53.

Grid convention: a box of n interior points per axis on the unit periodic
cube has spacing h = 1/n and interior point i at x_i = i * h.  Interior
arrays are float64, C order (z, y, x), x fastest.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM_MUL = np.uint64(0xD1342543DE82EF95)

# fixed seeds of the five workloads; written into every bench record
SEEDS = {
    "wave32": 1308_0,
    "wave256": 1308_1,
    "mixed192": 1308_2,
    "bboxset60": 1308_3,
    "adjoint128": 1308_4,
    "level60": 1308_5,
}


def _mix(z: np.ndarray) -> np.ndarray:
    """splitmix64 output function (a bijection on 64-bit words)."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    """Key of an independent stream: the mixed (seed, stream) pair."""
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(stream) * _STREAM_MUL)
    return _mix(np.array([s], dtype=np.uint64))[0]


def splitmix64(key: np.uint64, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the splitmix64 stream with state `key`."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + i * GAMMA)


def uniform01(seed: int, stream: int, shape) -> np.ndarray:
    shape = tuple(int(v) for v in np.atleast_1d(shape))
    count = int(np.prod(shape))
    z = splitmix64(stream_key(seed, stream), count)
    return ((z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)).reshape(shape)


def uniform_pm1(seed: int, stream: int, shape) -> np.ndarray:
    """Uniform draws in [-1, 1): 2r - 1 with r in [0, 1)."""
    return 2.0 * uniform01(seed, stream, shape) - 1.0


class Sequence:
    """Sequential reader of one splitmix64 stream (for small discrete draws)."""

    def __init__(self, seed: int, stream: int):
        self.key = stream_key(seed, stream)
        self.pos = 0

    def u64(self) -> int:
        v = int(splitmix64(self.key, 1, self.pos)[0])
        self.pos += 1
        return v

    def real(self) -> float:
        return (self.u64() >> 11) * (2.0 ** -53)

    def integer(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive), by scaling a [0,1) draw."""
        return lo + min(int(self.real() * (hi - lo + 1)), hi - lo)


# ----------------------------------------------------------------------------
# closed-form fields on the unit periodic cube


def coords(n: int):
    """Interior coordinates x_i = i/n along one axis."""
    return np.arange(n, dtype=np.float64) / n


def sine_mode_111(n) -> np.ndarray:
    """sin(2 pi x) sin(2 pi y) sin(2 pi z) sampled at interior points."""
    nx, ny, nz = _n3(n)
    sx = np.sin(2.0 * np.pi * coords(nx))
    sy = np.sin(2.0 * np.pi * coords(ny))
    sz = np.sin(2.0 * np.pi * coords(nz))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def gaussian_pulse(n, sigma: float = 0.1, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """exp(-|x - c|^2 / (2 sigma^2)) with the minimum-image distance on the unit cube."""
    nx, ny, nz = _n3(n)

    def d2(m, c):
        d = coords(m) - c
        d -= np.round(d)
        return d * d

    r2 = d2(nz, center[2])[:, None, None] + d2(ny, center[1])[None, :, None] + d2(nx, center[0])[None, None, :]
    return np.exp(-r2 / (2.0 * sigma * sigma))


def sine_modes(seed: int, stream: int, nmodes: int = 8, kmax: int = 4):
    """Random modes: amplitudes a in [-1,1), wave vectors in {-kmax..kmax}^3 minus 0,
    phases in [0, 2 pi).  Returned as (a[m], kappa[m,3] (x,y,z), phi[m])."""
    seq = Sequence(seed, stream)
    a = np.empty(nmodes)
    kap = np.empty((nmodes, 3), dtype=np.int64)
    phi = np.empty(nmodes)
    for m in range(nmodes):
        while True:
            k = [seq.integer(-kmax, kmax) for _ in range(3)]
            if any(k):
                break
        kap[m] = k
        phi[m] = 2.0 * np.pi * seq.real()
        a[m] = 2.0 * seq.real() - 1.0
    return a, kap, phi


def sine_sum(n, modes) -> np.ndarray:
    """g(x) = sum_m a_m sin(2 pi kappa_m . x + phi_m) at interior points."""
    nx, ny, nz = _n3(n)
    a, kap, phi = modes
    X = coords(nx)[None, None, :]
    Y = coords(ny)[None, :, None]
    Z = coords(nz)[:, None, None]
    out = np.zeros((nz, ny, nx))
    for m in range(len(a)):
        out += a[m] * np.sin(2.0 * np.pi * (kap[m, 0] * X + kap[m, 1] * Y + kap[m, 2] * Z) + phi[m])
    return out


def random_symmetric3(seed: int, stream: int) -> np.ndarray:
    """Symmetric 3x3 matrix with entries uniform in [-1, 1)."""
    r = uniform_pm1(seed, stream, (6,))
    A = np.empty((3, 3))
    A[0, 0], A[1, 1], A[2, 2] = r[0], r[1], r[2]
    A[0, 1] = A[1, 0] = r[3]
    A[0, 2] = A[2, 0] = r[4]
    A[1, 2] = A[2, 1] = r[5]
    return A


def _n3(n):
    if np.isscalar(n):
        return int(n), int(n), int(n)
    nx, ny, nz = (int(v) for v in n)
    return nx, ny, nz


# ----------------------------------------------------------------------------
# the five workloads


def wave_cube(n: int, seed: int, pulse: str, sigma: float = 0.1):
    """Wave equation in first-order form on one periodic n^3 box, h = 1/n, c = 1.

    u = U + P, rho = U' with U, U' uniform in [-1, 1) and P the smooth part:
    pulse "mode111" (sin sin sin) or "gauss" (Gaussian of width sigma at the centre).
    """
    u = uniform_pm1(seed, 1, (n, n, n))
    rho = uniform_pm1(seed, 2, (n, n, n))
    if pulse == "mode111":
        u += sine_mode_111(n)
    elif pulse == "gauss":
        u += gaussian_pulse(n, sigma)
    elif pulse != "none":
        raise ValueError(pulse)
    h = 1.0 / n
    return dict(n=(n, n, n), ghost=2, dx=(h, h, h), dt=0.25 * h, u=u, rho=rho, seed=seed)


def wave32(seed: int = SEEDS["wave32"]):
    """32^3 box + 2 ghosts, u = U + sin sin sin, rho = U, one RHS and 10 RK4 steps."""
    d = wave_cube(32, seed, "mode111")
    d["nsteps"] = 10
    return d


def wave256(seed: int = SEEDS["wave256"]):
    """256^3 box + 2 ghosts, u = U + Gaussian(sigma 0.1), rho = U, 100 RK4 steps."""
    d = wave_cube(256, seed, "gauss")
    d["nsteps"] = 100
    return d


def mixed_fields(n: int = 192, nfield: int = 6, seed: int = SEEDS["mixed192"]):
    """Multi-field workload: nfield smooth fields (8 random-phase sine modes, |k_i| <= 4)
    on an n^3 box + 2 ghosts, h = 1/n, and a symmetric 3x3 coefficient matrix A."""
    modes = [sine_modes(seed, 10 + f) for f in range(nfield)]
    fields = [sine_sum(n, m) for m in modes]
    A = random_symmetric3(seed, 3)
    h = 1.0 / n
    return dict(n=(n, n, n), ghost=2, dx=(h, h, h), fields=fields, modes=modes, A=A, seed=seed)


def bboxset(seed: int = SEEDS["bboxset60"], nlevels: int = 3, per_level: int = 20,
            smin: int = 16, smax: int = 96, ghost: int = 3, h0: float = 1.0 / 32):
    """Boxes of a block-structured refinement hierarchy.

    Per level l: spacing h0 / 2**l and `per_level` non-overlapping boxes, each side
    uniform in [smin, smax], placed by rejection sampling inside a level domain of
    4*smax points per axis.  Every box is treated as self-periodic.  Returns the box
    list (lo, n, level, dx) and seeded u, rho interior arrays per box.
    """
    seq = Sequence(seed, 5)
    dom = 4 * smax
    boxes = []
    for lev in range(nlevels):
        placed = []
        while len(placed) < per_level:
            n = [seq.integer(smin, smax) for _ in range(3)]
            for _ in range(1000):
                lo = [seq.integer(0, dom - n[a]) for a in range(3)]
                if all(not _overlap(lo, n, b["lo"], b["n"]) for b in placed):
                    break
            else:
                raise RuntimeError("box placement failed")
            h = h0 / 2 ** lev
            placed.append(dict(lo=tuple(lo), n=tuple(n), level=lev, dx=(h, h, h)))
        boxes.extend(placed)
    hmin = min(b["dx"][0] for b in boxes)
    us, rhos = [], []
    for i, b in enumerate(boxes):
        nx, ny, nz = b["n"]
        us.append(uniform_pm1(seed, 100 + 2 * i, (nz, ny, nx)))
        rhos.append(uniform_pm1(seed, 101 + 2 * i, (nz, ny, nx)))
    return dict(boxes=boxes, ghost=ghost, dt=0.25 * hmin, u=us, rho=rhos, seed=seed, nsteps=1)


def _partition(seq: Sequence, total: int, parts: int, smin: int, smax: int):
    """`parts` integer lengths in [smin, smax] that sum to `total`: the first
    parts - 1 uniform, the last the remainder, all redrawn until it fits."""
    for _ in range(100000):
        lens = [seq.integer(smin, smax) for _ in range(parts - 1)]
        last = total - sum(lens)
        if smin <= last <= smax:
            return lens + [last]
    raise RuntimeError("no partition found")


def level_tiling(seed: int = SEEDS["level60"], counts=(5, 4, 3), smin: int = 16, smax: int = 96,
                 ghost: int = 3, domain=None, h: float = 1.0 / 256):
    """One refinement level tiling a periodic domain with counts[0]*counts[1]*counts[2] boxes.

    z is cut into counts[2] slabs, every slab's y extent into counts[1] rows
    and every row's x extent into counts[0] boxes, each cut at seeded
    positions with box sides in [smin, smax].  Cuts differ between slabs and
    rows, so box faces meet in T-junctions and a ghost zone spans several
    neighbours.  The domain defaults to counts * (smin + smax) / 2 points.
    Spacing h on every axis, dt = h / 4.  u = U + S and rho = U' on the whole
    domain, with U, U' uniform in [-1, 1) and S a sine mode of one period
    along every axis of the domain; each box's interior is its slice.
    Returns boxes (dicts with lo (x, y, z) and n), domain (x, y, z), ghost,
    dx, dt and the global (z, y, x) arrays u, rho.
    """
    if domain is None:
        domain = tuple(c * (smin + smax) // 2 for c in counts)
    Nx, Ny, Nz = (int(v) for v in domain)
    seq = Sequence(seed, 7)
    boxes = []
    z0 = 0
    for lz in _partition(seq, Nz, counts[2], smin, smax):
        y0 = 0
        for ly in _partition(seq, Ny, counts[1], smin, smax):
            x0 = 0
            for lx in _partition(seq, Nx, counts[0], smin, smax):
                boxes.append(dict(lo=(x0, y0, z0), n=(lx, ly, lz)))
                x0 += lx
            y0 += ly
        z0 += lz
    u = uniform_pm1(seed, 1, (Nz, Ny, Nx)) + sine_mode_111((Nx, Ny, Nz))
    rho = uniform_pm1(seed, 2, (Nz, Ny, Nx))
    return dict(boxes=boxes, domain=(Nx, Ny, Nz), ghost=ghost, dx=(h, h, h), dt=0.25 * h, u=u, rho=rho,
                seed=seed)


def box_slice(b):
    """(z, y, x) slice of a global array holding box b's interior."""
    (x, y, z), (nx, ny, nz) = b["lo"], b["n"]
    return np.s_[z:z + nz, y:y + ny, x:x + nx]


def _overlap(lo1, n1, lo2, n2):
    return all(lo1[a] < lo2[a] + n2[a] and lo2[a] < lo1[a] + n1[a] for a in range(3))


def adjoint_case(n: int = 128, seed: int = SEEDS["adjoint128"], nsteps: int = 50, checkpoint: int = 10):
    """Variable-speed wave problem for the gradient: c^2 = 1 + 0.5 f / max|f| with f a
    sum of 8 random sine modes; u0, rho0, u_target uniform in [-1, 1); h = 1/n,
    dt = h/4, loss 0.5 * sum over interior points of (u(T) - u_target)^2."""
    f = sine_sum(n, sine_modes(seed, 20))
    c2 = 1.0 + 0.5 * f / np.max(np.abs(f))
    u0 = uniform_pm1(seed, 21, (n, n, n))
    rho0 = uniform_pm1(seed, 22, (n, n, n))
    ut = uniform_pm1(seed, 23, (n, n, n))
    h = 1.0 / n
    return dict(n=(n, n, n), ghost=2, dx=(h, h, h), dt=0.25 * h, c2=c2, u0=u0, rho0=rho0,
                u_target=ut, nsteps=nsteps, checkpoint=checkpoint, seed=seed)
