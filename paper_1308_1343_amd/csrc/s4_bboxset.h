// s4_bboxset.h -- bboxsets stored as discrete derivatives, and the ghost
// exchange schedule of one refinement level built from them (host only).
//
// A bboxset is a set of points of Z^D.  It is stored by dimensional
// recursion (Sec. II-C): a D-dimensional set keeps, for every coordinate n
// along its last axis where its (D-1)-dimensional cross-section changes, the
// change itself,
//     d[n] = section(n) xor section(n - 1),
// the leftward mod-2 derivative of Sec. II-B taken along that axis, as a
// (D-1)-dimensional bboxset of the same kind.  A 0-dimensional set is one
// boolean.  Only non-empty changes are kept, so the representation of a set
// is unique and two sets are equal exactly when their trees are.  The
// section at n is the xor of all changes at coordinates <= n: the
// anti-derivative, a scan from low to high coordinates.  Fully unrolled, the
// leaves are the points of d_0 d_1 ... R: the 2^D corners of a bbox, 6 points
// for an L-shape.
//
// Set operations follow the sweep of Sec. II-C (Fig. 2): walk the union of
// the two operands' change coordinates in order, keep the current sections
// R' and S' of both operands and T' of the result, and at each coordinate
// update R' and S' by their changes, form T' := R' (op) S' one dimension
// down, and store T's change T'_new xor T'_old where it is non-empty.  The
// symmetric difference needs no sweep: it is the xor of the two stored
// derivatives, change by change.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <array>
#include <map>
#include <utility>
#include <vector>

#include "sten4.h"

namespace s4 {

// Error reporting shared with the rest of the C ABI (message for s4_last_error).
int set_error(int code, const char *fmt, ...);

namespace bs {

using coord = int64_t;

enum SetOp : int { UNION = 0, INTERSECTION = 1, DIFFERENCE = 2, SYMDIFF = 3 };

inline bool apply(SetOp op, bool r, bool s)
{
    switch (op) {
    case UNION:
        return r || s;
    case INTERSECTION:
        return r && s;
    case DIFFERENCE:
        return r && !s;
    default:
        return r != s;
    }
}

template <int D>
struct Set {
    std::map<coord, Set<D - 1>> d; // change of the section along axis D-1, non-empty entries only
};

template <>
struct Set<0> {
    bool on = false;
};

template <int D>
bool empty(const Set<D> &a)
{
    if constexpr (D == 0)
        return !a.on;
    else
        return a.d.empty();
}

template <int D>
bool equal(const Set<D> &a, const Set<D> &b)
{
    if constexpr (D == 0) {
        return a.on == b.on;
    } else {
        if (a.d.size() != b.d.size())
            return false;
        for (auto i = a.d.begin(), j = b.d.begin(); i != a.d.end(); ++i, ++j)
            if (i->first != j->first || !equal<D - 1>(i->second, j->second))
                return false;
        return true;
    }
}

// R xor S, change by change (the xor of two sets is the xor of their derivatives)
template <int D>
Set<D> sym(const Set<D> &a, const Set<D> &b)
{
    Set<D> r;
    if constexpr (D == 0) {
        r.on = a.on != b.on;
    } else {
        auto i = a.d.begin(), j = b.d.begin();
        while (i != a.d.end() || j != b.d.end()) {
            if (j == b.d.end() || (i != a.d.end() && i->first < j->first)) {
                r.d.emplace_hint(r.d.end(), *i++);
            } else if (i == a.d.end() || j->first < i->first) {
                r.d.emplace_hint(r.d.end(), *j++);
            } else {
                Set<D - 1> x = sym<D - 1>(i->second, j->second);
                if (!empty<D - 1>(x))
                    r.d.emplace_hint(r.d.end(), i->first, std::move(x));
                ++i;
                ++j;
            }
        }
    }
    return r;
}

// T := R (op) S by the sweep over the last axis
template <int D>
Set<D> combine(SetOp op, const Set<D> &R, const Set<D> &S)
{
    if constexpr (D == 0) {
        Set<0> t;
        t.on = apply(op, R.on, S.on);
        return t;
    } else {
        if (op == SYMDIFF)
            return sym<D>(R, S);
        if (empty<D>(S))
            return op == INTERSECTION ? Set<D>{} : R;
        if (empty<D>(R))
            return op == UNION ? S : Set<D>{};
        Set<D> T;
        Set<D - 1> r, s, t; // sections of R, S and T on the sweep line
        auto i = R.d.begin(), j = S.d.begin();
        while (i != R.d.end() || j != S.d.end()) {
            const coord n = (j == S.d.end() || (i != R.d.end() && i->first <= j->first)) ? i->first : j->first;
            if (i != R.d.end() && i->first == n)
                r = sym<D - 1>(r, (i++)->second);
            if (j != S.d.end() && j->first == n)
                s = sym<D - 1>(s, (j++)->second);
            Set<D - 1> tn = combine<D - 1>(op, r, s);
            Set<D - 1> dt = sym<D - 1>(tn, t);
            if (!empty<D - 1>(dt))
                T.d.emplace_hint(T.d.end(), n, std::move(dt));
            t = std::move(tn);
        }
        return T;
    }
}

// the bbox [lo, hi) (empty if hi <= lo on any axis); lo, hi have D entries
template <int D>
Set<D> box(const coord *lo, const coord *hi)
{
    Set<D> s;
    if constexpr (D == 0) {
        s.on = true;
    } else {
        for (int a = 0; a < D; ++a)
            if (hi[a] <= lo[a])
                return s;
        Set<D - 1> c = box<D - 1>(lo, hi);
        s.d.emplace(lo[D - 1], c);
        s.d.emplace(hi[D - 1], std::move(c));
    }
    return s;
}

// the set moved by v: p is a member of the result iff p - v is one of a
template <int D>
Set<D> shift(const Set<D> &a, const coord *v)
{
    if constexpr (D == 0) {
        return a;
    } else {
        Set<D> r;
        for (const auto &e : a.d)
            r.d.emplace_hint(r.d.end(), e.first + v[D - 1], shift<D - 1>(e.second, v));
        return r;
    }
}

// d_axis R = R xor (R moved by +e_axis)
template <int D>
Set<D> derivative(const Set<D> &a, int axis)
{
    coord v[3] = {0, 0, 0};
    v[axis] = 1;
    return sym<D>(a, shift<D>(a, v));
}

// number of points
template <int D>
__int128 size(const Set<D> &a)
{
    if constexpr (D == 0) {
        return a.on ? 1 : 0;
    } else {
        __int128 tot = 0, secsize = 0;
        Set<D - 1> sec;
        coord prev = 0;
        for (const auto &e : a.d) {
            tot += (__int128)(e.first - prev) * secsize;
            sec = sym<D - 1>(sec, e.second);
            secsize = size<D - 1>(sec);
            prev = e.first;
        }
        return tot;
    }
}

// number of points of the full derivative (what the representation stores)
template <int D>
int64_t nkeys(const Set<D> &a)
{
    if constexpr (D == 0) {
        return a.on ? 1 : 0;
    } else {
        int64_t k = 0;
        for (const auto &e : a.d)
            k += nkeys<D - 1>(e.second);
        return k;
    }
}

template <int D, int DT>
void keys(const Set<D> &a, std::array<coord, DT> &p, std::vector<std::array<coord, DT>> &out)
{
    if constexpr (D == 0) {
        if (a.on)
            out.push_back(p);
    } else {
        for (const auto &e : a.d) {
            p[D - 1] = e.first;
            keys<D - 1, DT>(e.second, p, out);
        }
    }
}

template <int DT>
using BoxList = std::vector<std::pair<std::array<coord, DT>, std::array<coord, DT>>>;

// disjoint bboxes whose union is the set: one run of boxes per interval of
// constant section along the last axis, recursively
template <int D, int DT>
void boxes(const Set<D> &a, std::array<coord, DT> &lo, std::array<coord, DT> &hi, BoxList<DT> &out)
{
    if constexpr (D == 0) {
        if (a.on)
            out.emplace_back(lo, hi);
    } else {
        Set<D - 1> sec;
        for (auto it = a.d.begin(); it != a.d.end();) {
            sec = sym<D - 1>(sec, it->second);
            const coord n0 = it->first;
            if (++it == a.d.end())
                break;
            if (!empty<D - 1>(sec)) {
                lo[D - 1] = n0;
                hi[D - 1] = it->first;
                boxes<D - 1, DT>(sec, lo, hi, out);
            }
        }
    }
}

template <int D>
bool contains(const Set<D> &a, const coord *p)
{
    if constexpr (D == 0) {
        return a.on;
    } else {
        bool r = false;
        for (const auto &e : a.d) {
            if (e.first > p[D - 1])
                break;
            r ^= contains<D - 1>(e.second, p);
        }
        return r;
    }
}

// a u (a moved by +1) u ... u (a moved by +up) along one axis, by doubling
template <int D>
Set<D> grow_up(const Set<D> &a, int axis, coord up)
{
    Set<D> s = a;
    coord covered = 0; // s = union of the moves by 0 .. covered
    while (covered < up) {
        const coord step = std::min(covered + 1, up - covered);
        coord v[3] = {0, 0, 0};
        v[axis] = step;
        s = combine<D>(UNION, s, shift<D>(s, v));
        covered += step;
    }
    return s;
}

// Minkowski sum with the box [-lo, hi] per axis (lo, hi >= 0)
template <int D>
Set<D> expand(const Set<D> &a, const coord *lo, const coord *hi)
{
    Set<D> s = a;
    for (int ax = 0; ax < D; ++ax) {
        coord v[3] = {0, 0, 0};
        v[ax] = -lo[ax];
        s = grow_up<D>(shift<D>(s, v), ax, lo[ax] + hi[ax]);
    }
    return s;
}

// union of many sets by a balanced pairwise reduction
template <int D>
Set<D> union_all(std::vector<Set<D>> parts)
{
    if (parts.empty())
        return Set<D>{};
    while (parts.size() > 1) {
        std::vector<Set<D>> next;
        next.reserve((parts.size() + 1) / 2);
        for (size_t i = 0; i + 1 < parts.size(); i += 2)
            next.push_back(combine<D>(UNION, parts[i], parts[i + 1]));
        if (parts.size() % 2)
            next.push_back(std::move(parts.back()));
        parts.swap(next);
    }
    return std::move(parts[0]);
}

} // namespace bs

// ---------------------------------------------------------------------------
// Ghost exchange of one refinement level (Sec. II: boxes of a level fill
// each other's ghost zones).  A piece copies an extent of points from the
// interior of box `src` into the ghost zone of box `dst`; starts are in
// box-local interior coordinates (0 = first interior point, negative =
// ghost).

struct LevelPiece {
    int32_t dst, src;
    int64_t d0[3], s0[3];
    int64_t n[3];
};

} // namespace s4

struct s4_level {
    std::vector<s4_box> boxes;
    std::vector<std::array<int64_t, 3>> lo; // global origin of each interior
    int64_t domain[3];                      // periodic extent per axis, 0 = not periodic
    int width, shape;
    std::vector<s4::LevelPiece> pieces;
    int64_t filled = 0, uncovered = 0, points = 0;
    uint64_t serial = 0; // unique per schedule (graph cache key)
};
