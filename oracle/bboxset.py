"""Brute-force boolean-grid model of bboxsets and of same-level ghost exchange.

TEST INFRASTRUCTURE ONLY.  Imported by the tests; never by the HIP library or
its binding, and it shares no code with the library's bboxset algebra.

A bboxset (Sec. II) is a set of points of the integer grid Z^d, d = 1..3.  Here
a set is the plain definition: a boolean array `chi` over a window
[wlo, wlo + chi.shape) with chi[p - wlo] true exactly for the members p.
Array axis a is coordinate a (axis 0 = x).  A bbox is a half-open integer
box (lo, hi): the points p with lo[a] <= p[a] < hi[a] on every axis; it is
empty when hi[a] <= lo[a] on some axis.

The discrete derivative (Sec. II-B) is taken with the paper's leftward
difference in mod-2 arithmetic:
    (d_a R)(p) = R(p) xor R(p - e_a),
so the anti-derivative is a running xor that scans each axis from low to
high coordinates.  (The shift operator of the paper's formula is read as
"move the set by +e_a", the only reading under which the difference is
leftward and the recovery scans left to right, as the section states.)
For a bbox [lo, hi) the full derivative d_0 d_1 .. R is its 2^d corners
{lo_a, hi_a} per axis; an L-shaped region in 2D has 6 such points.

The window must hold one spare layer above every member on each axis, so
that d_a of the members sitting at the window's top still lands inside it;
`window_of` adds that layer.
"""

from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------- sets on a window

def window_of(boxes, dim, margin=1):
    """Smallest window holding every box, with `margin` spare layers on both sides."""
    boxes = [b for b in boxes if not box_empty(b)]
    if not boxes:
        return tuple([0] * dim), tuple([2 * margin + 1] * dim)
    lo = [min(b[0][a] for b in boxes) - margin for a in range(dim)]
    hi = [max(b[1][a] for b in boxes) + margin for a in range(dim)]
    return tuple(lo), tuple(h - l for h, l in zip(hi, lo))


def box_empty(b):
    lo, hi = b
    return any(h <= l for l, h in zip(lo, hi))


def rasterize(boxes, wlo, shape):
    """The union of the boxes as a boolean grid over the window."""
    chi = np.zeros(shape, dtype=bool)
    for lo, hi in boxes:
        if box_empty((lo, hi)):
            continue
        sl = []
        for a in range(len(shape)):
            l, h = lo[a] - wlo[a], hi[a] - wlo[a]
            assert 0 <= l and h <= shape[a], "box outside the window"
            sl.append(slice(l, h))
        chi[tuple(sl)] = True
    return chi


def members(chi, wlo):
    """Sorted list of member points (tuples of window-free coordinates)."""
    idx = np.argwhere(chi)
    return sorted(tuple(int(v) + int(o) for v, o in zip(row, wlo)) for row in idx)


def contains_brute(boxes, p):
    """Membership straight from the box list: p lies in at least one box."""
    return any(all(lo[a] <= p[a] < hi[a] for a in range(len(p))) for lo, hi in boxes)


def translate(chi, v):
    """The set moved by the integer vector v: result(p) = chi(p - v).  Members
    must not leave the window."""
    out = np.zeros_like(chi)
    src, dst = [], []
    for a, s in enumerate(v):
        n = chi.shape[a]
        if s >= 0:
            src.append(slice(0, n - s))
            dst.append(slice(s, n))
        else:
            src.append(slice(-s, n))
            dst.append(slice(0, n + s))
    out[tuple(dst)] = chi[tuple(src)]
    assert out.sum() == chi.sum(), "translation left the window"
    return out


def derivative(chi, axis):
    """d_axis R: R xor (R moved by +e_axis)."""
    e = [0] * chi.ndim
    e[axis] = 1
    return chi ^ translate(chi, e)


def antiderivative(d, axis):
    """Running xor from low to high coordinates along `axis` (inverse of derivative)."""
    return np.bitwise_xor.accumulate(d, axis=axis)


def full_derivative(chi):
    """d_0 d_1 ... d_{dim-1} R."""
    out = chi
    for a in range(chi.ndim):
        out = derivative(out, a)
    return out


def key_points(chi, wlo):
    """Members of the full derivative: the points a derivative bboxset stores."""
    return members(full_derivative(chi), wlo)


def expand(chi, lo, hi):
    """Minkowski sum with the box [-lo, hi] per axis: every member grows by
    lo[a] points downward and hi[a] points upward along axis a."""
    out = chi.copy()
    for a in range(chi.ndim):
        acc = np.zeros_like(out)
        for s in range(-lo[a], hi[a] + 1):
            e = [0] * chi.ndim
            e[a] = s
            acc |= translate(out, e)
        out = acc
    return out


SET_OPS = {
    "union": lambda r, s: r | s,
    "intersection": lambda r, s: r & s,
    "difference": lambda r, s: r & ~s,
    "symmetric_difference": lambda r, s: r ^ s,
}


def disjoint_cover(boxes, chi, wlo):
    """True when the boxes are pairwise disjoint, non-empty and their union is chi."""
    cover = np.zeros(chi.shape, dtype=np.int32)
    for lo, hi in boxes:
        if box_empty((lo, hi)):
            return False
        sl = tuple(slice(l - o, h - o) for l, h, o in zip(lo, hi, wlo))
        if any(s.start < 0 or s.stop > n for s, n in zip(sl, chi.shape)):
            return False
        cover[sl] += 1
    return bool(cover.max(initial=0) <= 1 and np.array_equal(cover == 1, chi))


# --------------------------------------------------------------------------- one level of boxes

def level_extent(lo, n, domain):
    """Extent of the owner map: the periodic extent on periodic axes
    (domain[a] > 0), the level's upper bound on open axes (domain[a] == 0)."""
    return tuple(int(domain[a]) if domain[a] > 0 else max(l[a] + m[a] for l, m in zip(lo, n)) for a in range(3))


def level_owner(lo, n, domain):
    """Owner map of a level over [0, level_extent): owner[x, y, z] = index of
    the box whose interior holds the point, -1 where none does.  Boxes must
    lie inside [0, extent) and must not overlap (AssertionError)."""
    ext = level_extent(lo, n, domain)
    own = np.full(ext, -1, dtype=np.int64)
    for b, (l, m) in enumerate(zip(lo, n)):
        assert all(0 <= l[a] and l[a] + m[a] <= ext[a] for a in range(3)), "box outside the domain"
        sl = tuple(slice(l[a], l[a] + m[a]) for a in range(3))
        assert (own[sl] < 0).all(), "boxes overlap"
        own[sl] = b
    return own


def sync_mask(n, g, width, shape):
    """Ghost points of a box (local coordinates in [-g, n+g) per axis, array
    index = coordinate + g, axis 0 = x) that a same-level ghost exchange of
    `width` layers fills.  shape "full": every point outside the interior
    that lies within `width` of it on every axis (faces, edges and corners);
    "faces": only points outside the interior along exactly one axis, within
    `width` of it (what an axis-aligned stencil of radius `width` reads)."""
    ext = [np.arange(-g, m + g) for m in n]
    inside = [(e >= 0) & (e < m) for e, m in zip(ext, n)]
    near = [(e >= -width) & (e < m + width) for e, m in zip(ext, n)]
    I = [np.asarray(v).reshape([-1 if a == b else 1 for b in range(3)]) for a, v in enumerate(inside)]
    N = [np.asarray(v).reshape([-1 if a == b else 1 for b in range(3)]) for a, v in enumerate(near)]
    interior = I[0] & I[1] & I[2]
    if shape == "full":
        m = N[0] & N[1] & N[2] & ~interior
    elif shape == "faces":
        m = np.zeros((n[0] + 2 * g, n[1] + 2 * g, n[2] + 2 * g), dtype=bool)
        for a in range(3):
            b, c = [x for x in range(3) if x != a]
            m |= N[a] & ~I[a] & I[b] & I[c]
    else:
        raise ValueError(shape)
    return np.broadcast_to(m, (n[0] + 2 * g, n[1] + 2 * g, n[2] + 2 * g))


def sync_sources(lo, n, g, domain, width, shape):
    """For every box b, the map of its ghost points to their sources under a
    same-level exchange: arrays (ghost point local coords, owner box or -1,
    owner-local coords).  A ghost point p of box b is the grid point
    lo_b + p, taken modulo domain[a] on periodic axes (domain[a] > 0); on an
    open axis (domain[a] == 0) a point outside the level's extent has no
    owner."""
    own = level_owner(lo, n, domain)
    ext = np.asarray(own.shape)
    per = np.asarray([d > 0 for d in domain])
    out = []
    for b in range(len(lo)):
        m = sync_mask(n[b], g, width, shape)
        pts = np.argwhere(m) - g                      # local coords
        glob = pts + np.asarray(lo[b])
        glob = np.where(per, glob % np.where(per, ext, 1), glob)
        inside = ((glob >= 0) & (glob < ext)).all(axis=1)
        safe = np.where(inside[:, None], glob, 0)
        who = np.where(inside, own[safe[:, 0], safe[:, 1], safe[:, 2]], -1)
        src = glob - np.asarray(lo)[np.maximum(who, 0)]
        out.append((pts, who, src))
    return out


def check_pieces(pieces, lo, n, g, domain, width, shape):
    """Check a list of copy pieces (dst box, src box, dst start[3], src start[3],
    extent[3], all in box-local interior coordinates) against sync_sources
    point by point: every coverable ghost point is written by exactly one
    piece, from the right box and point, and nothing else is written.
    Returns (filled, uncovered) point counts."""
    nb = len(lo)
    sh = [tuple(m + 2 * g for m in n[b]) for b in range(nb)]
    want_box = [np.full(s, -2, dtype=np.int64) for s in sh]
    want_src = [np.zeros(s + (3,), dtype=np.int64) for s in sh]
    for b, (pts, who, src) in enumerate(sync_sources(lo, n, g, domain, width, shape)):
        ix = tuple((pts + g).T)
        want_box[b][ix] = who
        want_src[b][ix] = src
    count = [np.zeros(s, dtype=np.int64) for s in sh]
    got_box = [np.full(s, -2, dtype=np.int64) for s in sh]
    got_src = [np.zeros(s + (3,), dtype=np.int64) for s in sh]
    for dst, srcb, d0, s0, ext in pieces:
        assert all(e > 0 for e in ext), "empty piece"
        sl = tuple(slice(d0[a] + g, d0[a] + g + ext[a]) for a in range(3))
        assert all(s.start >= 0 and s.stop <= m for s, m in zip(sl, sh[dst])), "piece outside the box"
        count[dst][sl] += 1
        got_box[dst][sl] = srcb
        grid = np.stack(np.meshgrid(*[s0[a] + np.arange(ext[a]) for a in range(3)], indexing="ij"), axis=-1)
        got_src[dst][sl] = grid
    filled = uncovered = 0
    for b in range(nb):
        assert count[b].max(initial=0) <= 1, f"box {b}: a ghost point is written twice"
        w = count[b] == 1
        assert np.array_equal(w, want_box[b] >= 0), f"box {b}: written points differ from the coverable ghosts"
        assert np.array_equal(got_box[b][w], want_box[b][w]), f"box {b}: wrong source box"
        assert np.array_equal(got_src[b][w], want_src[b][w]), f"box {b}: wrong source point"
        filled += int(w.sum())
        uncovered += int((want_box[b] == -1).sum())
    return filled, uncovered
