// s4_bboxset.cpp -- the C ABI of bboxsets (s4_bset_*) and of the level
// ghost-exchange schedule (s4_level_create and its queries).  Host code only:
// the schedule is executed by s4_level_sync / s4_level_rk4 in s4_api.cpp.

#include <atomic>
#include <climits>
#include <cstring>
#include <new>

#include "s4_bboxset.h"

using namespace s4;
using bs::coord;
using bs::Set;

struct s4_bset {
    int dim = 3;
    Set<1> s1;
    Set<2> s2;
    Set<3> s3;
};

namespace {

const coord COORD_MAX = (coord)1 << 40;

template <int D>
Set<D> &part(s4_bset &h)
{
    if constexpr (D == 1)
        return h.s1;
    else if constexpr (D == 2)
        return h.s2;
    else
        return h.s3;
}

template <int D>
const Set<D> &part(const s4_bset &h)
{
    return part<D>(const_cast<s4_bset &>(h));
}

// call f.template operator()<D>() for the handle's dimension
template <class F>
int by_dim(int dim, F &&f)
{
    switch (dim) {
    case 1:
        return f(std::integral_constant<int, 1>{});
    case 2:
        return f(std::integral_constant<int, 2>{});
    case 3:
        return f(std::integral_constant<int, 3>{});
    default:
        return set_error(S4_EINVAL, "bboxset dim %d not in 1..3", dim);
    }
}

bool coord_ok(coord c)
{
    return c >= -COORD_MAX && c <= COORD_MAX;
}

// a new handle holding `s`; nullptr on allocation failure
template <int D>
int give(Set<D> &&s, s4_bset **out)
{
    s4_bset *h = new (std::nothrow) s4_bset;
    if (!h)
        return set_error(S4_EINVAL, "out of host memory");
    h->dim = D;
    part<D>(*h) = std::move(s);
    *out = h;
    return S4_OK;
}

// every key coordinate must stay in range after an operation that moves sets
template <int D>
bool in_range(const Set<D> &a)
{
    if constexpr (D == 0) {
        return true;
    } else {
        for (const auto &e : a.d)
            if (!coord_ok(e.first) || !in_range<D - 1>(e.second))
                return false;
        return true;
    }
}

} // namespace

extern "C" {

int s4_bset_from_boxes(int dim, const int64_t *lo, const int64_t *hi, int64_t nbox, s4_bset **out)
{
    if (!out)
        return set_error(S4_EINVAL, "NULL argument");
    *out = nullptr;
    if (nbox < 0 || (nbox > 0 && (!lo || !hi)))
        return set_error(S4_EINVAL, "bad box array");
    if (nbox > ((int64_t)1 << 32))
        return set_error(S4_EINVAL, "too many boxes");
    return by_dim(dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        std::vector<Set<D>> parts;
        parts.reserve((size_t)nbox);
        for (int64_t k = 0; k < nbox; ++k) {
            const int64_t *l = lo + k * D, *h = hi + k * D;
            for (int a = 0; a < D; ++a)
                if (!coord_ok(l[a]) || !coord_ok(h[a]))
                    return set_error(S4_EINVAL, "box %lld: coordinate beyond 2^40", (long long)k);
            Set<D> b = bs::box<D>(l, h);
            if (!bs::empty<D>(b))
                parts.push_back(std::move(b));
        }
        return give<D>(bs::union_all<D>(std::move(parts)), out);
    });
}

void s4_bset_free(s4_bset *s)
{
    delete s;
}

int s4_bset_op(int op, const s4_bset *a, const s4_bset *b, s4_bset **out)
{
    if (!a || !b || !out)
        return set_error(S4_EINVAL, "NULL argument");
    *out = nullptr;
    if (op < S4_SET_UNION || op > S4_SET_SYMDIFF)
        return set_error(S4_EINVAL, "unknown set operation %d", op);
    if (a->dim != b->dim)
        return set_error(S4_EINVAL, "set dims differ (%d, %d)", a->dim, b->dim);
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        return give<D>(bs::combine<D>((bs::SetOp)op, part<D>(*a), part<D>(*b)), out);
    });
}

int s4_bset_shift(const s4_bset *a, const int64_t *v, s4_bset **out)
{
    if (!a || !v || !out)
        return set_error(S4_EINVAL, "NULL argument");
    *out = nullptr;
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        for (int k = 0; k < D; ++k)
            if (!coord_ok(v[k]))
                return set_error(S4_EINVAL, "shift beyond 2^40");
        Set<D> r = bs::shift<D>(part<D>(*a), v);
        if (!in_range<D>(r))
            return set_error(S4_EINVAL, "shifted set leaves the coordinate range");
        return give<D>(std::move(r), out);
    });
}

int s4_bset_expand(const s4_bset *a, const int64_t *lo, const int64_t *hi, s4_bset **out)
{
    if (!a || !lo || !hi || !out)
        return set_error(S4_EINVAL, "NULL argument");
    *out = nullptr;
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        for (int k = 0; k < D; ++k)
            if (lo[k] < 0 || hi[k] < 0 || lo[k] > (1 << 20) || hi[k] > (1 << 20))
                return set_error(S4_EINVAL, "expand widths must lie in [0, 2^20]");
        Set<D> r = bs::expand<D>(part<D>(*a), lo, hi);
        if (!in_range<D>(r))
            return set_error(S4_EINVAL, "expanded set leaves the coordinate range");
        return give<D>(std::move(r), out);
    });
}

int s4_bset_derivative(const s4_bset *a, int axis, s4_bset **out)
{
    if (!a || !out)
        return set_error(S4_EINVAL, "NULL argument");
    *out = nullptr;
    if (axis < 0 || axis >= a->dim)
        return set_error(S4_EINVAL, "axis %d not in [0, %d)", axis, a->dim);
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        Set<D> r = bs::derivative<D>(part<D>(*a), axis);
        if (!in_range<D>(r))
            return set_error(S4_EINVAL, "derivative leaves the coordinate range");
        return give<D>(std::move(r), out);
    });
}

int s4_bset_info(const s4_bset *a, int64_t info[4])
{
    if (!a || !info)
        return set_error(S4_EINVAL, "NULL argument");
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        const Set<D> &s = part<D>(*a);
        const __int128 n = bs::size<D>(s);
        if (n > (__int128)INT64_MAX)
            return set_error(S4_EINVAL, "point count beyond int64");
        std::array<coord, D> l{}, h{};
        bs::BoxList<D> bl;
        bs::boxes<D, D>(s, l, h, bl);
        info[0] = D;
        info[1] = (int64_t)n;
        info[2] = bs::nkeys<D>(s);
        info[3] = (int64_t)bl.size();
        return S4_OK;
    });
}

int s4_bset_keys(const s4_bset *a, int64_t *out, int64_t max, int64_t *count)
{
    if (!a || !count || (max > 0 && !out))
        return set_error(S4_EINVAL, "NULL argument");
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        std::array<coord, D> p{};
        std::vector<std::array<coord, D>> k;
        bs::keys<D, D>(part<D>(*a), p, k);
        *count = (int64_t)k.size();
        for (int64_t i = 0; i < std::min<int64_t>(max, *count); ++i)
            for (int d = 0; d < D; ++d)
                out[i * D + d] = k[(size_t)i][d];
        return S4_OK;
    });
}

int s4_bset_boxes(const s4_bset *a, int64_t *lo, int64_t *hi, int64_t max, int64_t *count)
{
    if (!a || !count || (max > 0 && (!lo || !hi)))
        return set_error(S4_EINVAL, "NULL argument");
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        std::array<coord, D> l{}, h{};
        bs::BoxList<D> bl;
        bs::boxes<D, D>(part<D>(*a), l, h, bl);
        *count = (int64_t)bl.size();
        for (int64_t i = 0; i < std::min<int64_t>(max, *count); ++i)
            for (int d = 0; d < D; ++d) {
                lo[i * D + d] = bl[(size_t)i].first[d];
                hi[i * D + d] = bl[(size_t)i].second[d];
            }
        return S4_OK;
    });
}

int s4_bset_contains(const s4_bset *a, const int64_t *p, int *out)
{
    if (!a || !p || !out)
        return set_error(S4_EINVAL, "NULL argument");
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        *out = bs::contains<D>(part<D>(*a), p) ? 1 : 0;
        return S4_OK;
    });
}

int s4_bset_equal(const s4_bset *a, const s4_bset *b, int *out)
{
    if (!a || !b || !out)
        return set_error(S4_EINVAL, "NULL argument");
    if (a->dim != b->dim)
        return set_error(S4_EINVAL, "set dims differ (%d, %d)", a->dim, b->dim);
    return by_dim(a->dim, [&](auto dc) -> int {
        constexpr int D = decltype(dc)::value;
        *out = bs::equal<D>(part<D>(*a), part<D>(*b)) ? 1 : 0;
        return S4_OK;
    });
}

// ---------------------------------------------------------------------------
// level schedule

int s4_level_create(const s4_box *b, const int64_t *lo, int nbox, const int64_t domain[3], int width, int shape,
                    s4_level **out)
{
    if (!out)
        return set_error(S4_EINVAL, "NULL argument");
    *out = nullptr;
    if (!lo || !domain)
        return set_error(S4_EINVAL, "NULL argument");
    int r = s4_check_boxes(b, nbox, S4_OP_RK4);
    if (r)
        return r;
    if (shape != S4_SYNC_FULL && shape != S4_SYNC_FACES)
        return set_error(S4_EINVAL, "unknown exchange shape %d", shape);
    for (int i = 0; i < nbox; ++i)
        if (width < 1 || width > b[i].ghost)
            return set_error(S4_EGHOST, "box %d: exchange width %d not in [1, ghost = %d]", i, width, b[i].ghost);
    for (int a = 0; a < 3; ++a) {
        if (domain[a] < 0 || domain[a] > COORD_MAX / 4)
            return set_error(S4_EINVAL, "domain[%d] = %lld out of range", a, (long long)domain[a]);
        if (domain[a] > 0 && width > domain[a])
            return set_error(S4_EINVAL, "width %d exceeds the periodic extent %lld", width, (long long)domain[a]);
    }
    for (int i = 0; i < nbox; ++i)
        for (int a = 0; a < 3; ++a) {
            const int64_t l = lo[3 * i + a], h = l + b[i].n[a];
            if (!coord_ok(l) || !coord_ok(h) || l < -COORD_MAX / 4 || h > COORD_MAX / 4)
                return set_error(S4_EINVAL, "box %d: origin out of range", i);
            if (domain[a] > 0 && (l < 0 || h > domain[a]))
                return set_error(S4_EINVAL, "box %d lies outside the periodic domain along axis %d", i, a);
            if (b[i].dx[a] != b[0].dx[a])
                return set_error(S4_EINVAL, "box %d: grid spacing differs from box 0 (one level, one spacing)", i);
        }

    s4_level *L = new (std::nothrow) s4_level;
    if (!L)
        return set_error(S4_EINVAL, "out of host memory");
    L->boxes.assign(b, b + nbox);
    L->lo.resize((size_t)nbox);
    for (int i = 0; i < nbox; ++i)
        for (int a = 0; a < 3; ++a)
            L->lo[(size_t)i][a] = lo[3 * i + a];
    for (int a = 0; a < 3; ++a)
        L->domain[a] = domain[a];
    L->width = width;
    L->shape = shape;

    // interiors as bboxsets; disjoint iff the union holds all their points
    std::vector<Set<3>> interior((size_t)nbox);
    std::vector<std::array<coord, 3>> ilo((size_t)nbox), ihi((size_t)nbox);
    __int128 total = 0;
    for (int i = 0; i < nbox; ++i) {
        for (int a = 0; a < 3; ++a) {
            ilo[(size_t)i][a] = lo[3 * i + a];
            ihi[(size_t)i][a] = lo[3 * i + a] + b[i].n[a];
        }
        interior[(size_t)i] = bs::box<3>(ilo[(size_t)i].data(), ihi[(size_t)i].data());
        total += bs::size<3>(interior[(size_t)i]);
    }
    if (bs::size<3>(bs::union_all<3>(interior)) != total) {
        delete L;
        return set_error(S4_EINVAL, "box interiors overlap");
    }
    L->points = (int64_t)total;

    // Box interiors and their periodic images that a ghost zone can reach (the
    // images meeting [-width, domain + width) on periodic axes), registered in a
    // coarse grid of cells at least as wide as any ghosted box, so that each box
    // finds its neighbours among the few images sharing its cells instead of
    // among all of them.
    const coord w = width;
    struct Image {
        int box;
        std::array<coord, 3> t, lo, hi;
    };
    std::vector<Image> imgs;
    for (int c = 0; c < nbox; ++c)
        for (int z = -1; z <= 1; ++z)
            for (int y = -1; y <= 1; ++y)
                for (int x = -1; x <= 1; ++x) {
                    const int k[3] = {x, y, z};
                    Image im;
                    im.box = c;
                    bool ok = true;
                    for (int a = 0; a < 3; ++a) {
                        ok = ok && (k[a] == 0 || domain[a] > 0);
                        im.t[a] = k[a] * domain[a];
                        im.lo[a] = ilo[(size_t)c][a] + im.t[a];
                        im.hi[a] = ihi[(size_t)c][a] + im.t[a];
                        if (k[a] != 0)
                            ok = ok && im.lo[a] < domain[a] + w && -w < im.hi[a];
                    }
                    if (ok)
                        imgs.push_back(im);
                }
    std::array<coord, 3> cell{};
    for (int a = 0; a < 3; ++a) {
        coord m = 1;
        for (int c = 0; c < nbox; ++c)
            m = std::max<coord>(m, b[c].n[a]);
        cell[a] = m + 2 * w;
    }
    auto cell_of = [&](coord x, int a) { return x >= 0 ? x / cell[a] : -((-x + cell[a] - 1) / cell[a]); };
    std::map<std::array<coord, 3>, std::vector<int>> grid;
    for (int k = 0; k < (int)imgs.size(); ++k) {
        const Image &im = imgs[(size_t)k];
        for (coord cz = cell_of(im.lo[2], 2); cz <= cell_of(im.hi[2] - 1, 2); ++cz)
            for (coord cy = cell_of(im.lo[1], 1); cy <= cell_of(im.hi[1] - 1, 1); ++cy)
                for (coord cx = cell_of(im.lo[0], 0); cx <= cell_of(im.hi[0] - 1, 0); ++cx)
                    grid[{cx, cy, cz}].push_back(k);
    }

    for (int i = 0; i < nbox; ++i) {
        const auto &bl = ilo[(size_t)i], &bh = ihi[(size_t)i];
        // the ghost region box i needs
        Set<3> grown;
        if (shape == S4_SYNC_FULL) {
            const coord g3[3] = {w, w, w};
            grown = bs::expand<3>(interior[(size_t)i], g3, g3);
        } else {
            std::vector<Set<3>> faces;
            for (int a = 0; a < 3; ++a) {
                std::array<coord, 3> l = bl, h = bh;
                l[a] -= w;
                h[a] += w;
                faces.push_back(bs::box<3>(l.data(), h.data()));
            }
            grown = bs::union_all<3>(std::move(faces));
        }
        const Set<3> need = bs::combine<3>(bs::DIFFERENCE, grown, interior[(size_t)i]);
        std::vector<int> near;
        for (coord cz = cell_of(bl[2] - w, 2); cz <= cell_of(bh[2] + w - 1, 2); ++cz)
            for (coord cy = cell_of(bl[1] - w, 1); cy <= cell_of(bh[1] + w - 1, 1); ++cy)
                for (coord cx = cell_of(bl[0] - w, 0); cx <= cell_of(bh[0] + w - 1, 0); ++cx) {
                    auto it = grid.find({cx, cy, cz});
                    if (it != grid.end())
                        near.insert(near.end(), it->second.begin(), it->second.end());
                }
        std::sort(near.begin(), near.end());
        near.erase(std::unique(near.begin(), near.end()), near.end());
        std::vector<Set<3>> got;
        for (int k : near) {
            const Image &im = imgs[(size_t)k];
            bool touch = true;
            for (int a = 0; a < 3; ++a)
                touch = touch && im.lo[a] < bh[a] + w && bl[a] - w < im.hi[a];
            if (!touch)
                continue;
            Set<3> piece = bs::combine<3>(bs::INTERSECTION, need, bs::box<3>(im.lo.data(), im.hi.data()));
            if (bs::empty<3>(piece))
                continue;
            std::array<coord, 3> pl{}, ph{};
            bs::BoxList<3> boxes;
            bs::boxes<3, 3>(piece, pl, ph, boxes);
            for (const auto &bx : boxes) {
                LevelPiece P;
                P.dst = i;
                P.src = im.box;
                for (int a = 0; a < 3; ++a) {
                    P.d0[a] = bx.first[a] - bl[a];
                    P.s0[a] = bx.first[a] - im.t[a] - ilo[(size_t)im.box][a];
                    P.n[a] = bx.second[a] - bx.first[a];
                }
                L->pieces.push_back(P);
            }
            got.push_back(std::move(piece));
        }
        const Set<3> covered = bs::union_all<3>(std::move(got));
        L->filled += (int64_t)bs::size<3>(covered);
        L->uncovered += (int64_t)bs::size<3>(bs::combine<3>(bs::DIFFERENCE, need, covered));
    }
    static std::atomic<uint64_t> serial{0};
    L->serial = ++serial;
    *out = L;
    return S4_OK;
}

void s4_level_destroy(s4_level *L)
{
    delete L;
}

int s4_level_info(const s4_level *L, int64_t info[7])
{
    if (!L || !info)
        return set_error(S4_EINVAL, "NULL argument");
    info[0] = (int64_t)L->boxes.size();
    info[1] = (int64_t)L->pieces.size();
    info[2] = L->filled;
    info[3] = L->uncovered;
    info[4] = L->points;
    info[5] = L->width;
    info[6] = L->shape;
    return S4_OK;
}

int s4_level_pieces(const s4_level *L, int64_t *out, int64_t max, int64_t *count)
{
    if (!L || !count || (max > 0 && !out))
        return set_error(S4_EINVAL, "NULL argument");
    *count = (int64_t)L->pieces.size();
    for (int64_t k = 0; k < std::min<int64_t>(max, *count); ++k) {
        const LevelPiece &P = L->pieces[(size_t)k];
        int64_t *o = out + 11 * k;
        o[0] = P.dst;
        o[1] = P.src;
        for (int a = 0; a < 3; ++a) {
            o[2 + a] = P.d0[a];
            o[5 + a] = P.s0[a];
            o[8 + a] = P.n[a];
        }
    }
    return S4_OK;
}

} // extern "C"
