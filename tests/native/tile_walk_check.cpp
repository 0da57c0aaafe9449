// Host-side check of the stencil traversal's addressing (s4_internal.h), run
// by tests/test_geometry.py.  For every work item, thread and plane of a
// box it replays the loads, LDS writes and stores the kernels issue -- with
// the same Walker, item_pos and halo_slot code -- tagging each value with the
// element it came from, and checks that
//   * every global read lies inside the box's array (and, with periodic
//     addressing, inside the interior; with ghost addressing, inside the
//     radius-2 shell),
//   * no two threads write different points into one LDS slot of a plane,
//   * each of the 13 stencil taps an active lane uses holds the right point,
//   * every interior point is stored exactly once and nothing else is.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "s4_internal.h"

using namespace s4;

static int fails = 0;
#define CHECK(cond, ...)                                                                               \
    do {                                                                                               \
        if (!(cond)) {                                                                                 \
            if (fails < 20) {                                                                          \
                fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);                                  \
                fprintf(stderr, __VA_ARGS__);                                                          \
                fprintf(stderr, "\n");                                                                 \
            }                                                                                          \
            ++fails;                                                                                   \
        }                                                                                              \
    } while (0)

static int wrapi(int p, int n)
{
    int r = p % n;
    return r < 0 ? r + n : r;
}

template <int TX, int NW, bool WRAP>
static void run(int nx, int ny, int nz, int g, int padx, int pady, int tz_req)
{
    using T = Tile<TX, NW>;
    DevBox B{};
    B.n[0] = nx;
    B.n[1] = ny;
    B.n[2] = nz;
    B.g = g;
    B.sy = nx + 2 * g + padx;
    B.sz = B.sy * (ny + 2 * g + pady);
    B.tz = tz_req > 0 && tz_req < nz ? tz_req : nz;
    B.tiles[0] = (nx + TX - 1) / TX;
    B.tiles[1] = (ny + T::TY - 1) / T::TY;
    B.tiles[2] = (nz + B.tz - 1) / B.tz;
    const int64_t total = B.sz * (nz + 2 * g);
    std::vector<int> written(total, 0);
    const int nitems = B.tiles[0] * B.tiles[1] * B.tiles[2];
    auto expect = [&](int i, int j, int k) -> int64_t {
        if (WRAP)
            return elem(B, wrapi(i, nx), wrapi(j, ny), wrapi(k, nz));
        return elem(B, i, j, k);
    };
    auto check_read = [&](int64_t e, const char *what) {
        CHECK(e >= 0 && e < total, "%s read %lld outside [0,%lld)", what, (long long)e, (long long)total);
        if (e < 0 || e >= total)
            return;
        const int k = (int)(e / B.sz) - g, j = (int)(e % B.sz / B.sy) - g, i = (int)(e % B.sy) - g;
        if (WRAP)
            CHECK(i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz, "%s read a ghost (%d,%d,%d)", what, i, j, k);
        else
            CHECK(i >= -2 && i < nx + 2 && j >= -2 && j < ny + 2 && k >= -2 && k < nz + 2,
                  "%s read beyond the radius-2 shell (%d,%d,%d)", what, i, j, k);
    };
    // also exercise the XCD remap: logical item of every hardware block
    std::vector<int> seen(nitems, 0);
    for (int b = 0; b < nitems; ++b) {
        const int it = xcd_remap(b, nitems, 8);
        CHECK(it >= 0 && it < nitems, "remap out of range");
        if (it >= 0 && it < nitems)
            seen[it]++;
    }
    for (int it = 0; it < nitems; ++it)
        CHECK(seen[it] == 1, "remap not a bijection at %d", it);

    std::vector<Walker<TX, NW, WRAP>> W;
    std::vector<int64_t> lds(2 * T::LY * T::LX);
    for (int item = 0; item < nitems; ++item) {
        const ItemPos P = item_pos(B, item, TX, T::TY);
        CHECK(P.z0 < P.z1 && P.z1 <= nz, "empty or overlong z range");
        W.clear();
        for (int t = 0; t < T::NT; ++t)
            W.emplace_back(B, P, t);
        std::vector<int64_t> q(T::NT * 5);
        for (int t = 0; t < T::NT; ++t)
            for (int d = 0; d < 4; ++d) {
                const int64_t e = W[t].col + W[t].zoff(P.z0 - 2 + d);
                check_read(e, "queue warm-up");
                q[t * 5 + d] = e;
            }
        for (int k = P.z0; k < P.z1; ++k) {
            std::fill(lds.begin(), lds.end(), -1);
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                const int64_t e4 = w.col + w.zoff(k + 2);
                check_read(e4, "queue");
                q[t * 5 + 4] = e4;
                CHECK(w.lc >= 0 && w.lc < T::LY * T::LX, "LDS slot out of range");
                const int64_t own = q[t * 5 + 2];
                CHECK(lds[w.lc] == -1 || lds[w.lc] == own, "LDS own-slot conflict");
                lds[w.lc] = own;
                for (int s = 0; s < T::HS; ++s) {
                    if (w.hl[s] < 0)
                        continue;
                    const int64_t e = w.hcol[s] + w.zoff(k);
                    check_read(e, "halo");
                    CHECK(w.hl[s] >= 0 && w.hl[s] < T::LY * T::LX, "halo LDS slot out of range");
                    CHECK(lds[w.hl[s]] == -1 || lds[w.hl[s]] == e, "halo LDS conflict");
                    lds[w.hl[s]] = e;
                }
            }
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                if (!w.active)
                    continue;
                const int i = w.i, j = w.j;
                CHECK(q[t * 5 + 2] == expect(i, j, k), "centre tag");
                for (int d = -2; d <= 2; ++d) {
                    if (d == 0)
                        continue;
                    CHECK(lds[w.lc + d] == expect(i + d, j, k), "x tap %d at (%d,%d,%d)", d, i, j, k);
                    CHECK(lds[w.lc + d * T::LX] == expect(i, j + d, k), "y tap %d at (%d,%d,%d)", d, i, j, k);
                    CHECK(q[t * 5 + 2 + d] == expect(i, j, k + d), "z tap %d at (%d,%d,%d)", d, i, j, k);
                }
                const int64_t c = w.point(B, k);
                CHECK(c == elem(B, i, j, k), "store offset");
                if (c >= 0 && c < total)
                    written[c]++;
            }
            for (int t = 0; t < T::NT; ++t)
                for (int d = 0; d < 4; ++d)
                    q[t * 5 + d] = q[t * 5 + d + 1];
        }
    }
    for (int k = -g; k < nz + g; ++k)
        for (int j = -g; j < ny + g; ++j)
            for (int i = -g; i < nx + g; ++i) {
                const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                const int c = written[elem(B, i, j, k)];
                CHECK(c == (in ? 1 : 0), "point (%d,%d,%d) stored %d times", i, j, k, c);
            }
}

// the mixed-derivative traversal (ghost addressing, leading-plane LDS with
// corners, second LDS plane of D1_x on the tile rows and the halo rows)
template <int TX, int NW>
static void run_mixed(int nx, int ny, int nz, int g, int padx, int tz_req)
{
    using T = Tile<TX, NW>;
    using M = MixTile<TX, NW>;
    DevBox B{};
    B.n[0] = nx;
    B.n[1] = ny;
    B.n[2] = nz;
    B.g = g;
    B.sy = nx + 2 * g + padx;
    B.sz = B.sy * (ny + 2 * g);
    B.tz = tz_req > 0 && tz_req < nz ? tz_req : nz;
    B.tiles[0] = (nx + TX - 1) / TX;
    B.tiles[1] = (ny + T::TY - 1) / T::TY;
    B.tiles[2] = (nz + B.tz - 1) / B.tz;
    const int64_t total = B.sz * (nz + 2 * g);
    std::vector<int> written(total, 0);
    const int nitems = B.tiles[0] * B.tiles[1] * B.tiles[2];
    std::vector<int64_t> F(M::PF), D(M::PD);
    for (int item = 0; item < nitems; ++item) {
        const ItemPos P = item_pos(B, item, TX, T::TY);
        std::vector<MixWalker<TX, NW>> W;
        for (int t = 0; t < T::NT; ++t)
            W.emplace_back(B, P, t);
        for (int kk = P.z0 - 2; kk <= P.z1 + 1; ++kk) {
            std::fill(F.begin(), F.end(), -1);
            std::fill(D.begin(), D.end(), -1);
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                const int64_t e = w.col + w.zoff(kk);
                CHECK(e >= 0 && e < total, "mixed own read out of range");
                CHECK(F[w.lf] == -1 || F[w.lf] == e, "mixed own LDS conflict");
                F[w.lf] = e;
                for (int s = 0; s < M::HS; ++s) {
                    if (w.hl[s] < 0)
                        continue;
                    const int64_t h = w.hcol[s] + w.zoff(kk);
                    CHECK(h >= 0 && h < total, "mixed halo read out of range");
                    CHECK(w.hl[s] >= 0 && w.hl[s] < M::PF, "mixed halo slot out of range");
                    CHECK(F[w.hl[s]] == -1 || F[w.hl[s]] == h, "mixed halo LDS conflict");
                    F[w.hl[s]] = h;
                }
            }
            // D1_x points: valid when all four x taps hold the x neighbours of the centre
            auto d1x_tag = [&](int e) -> int64_t {
                for (int d = -2; d <= 2; ++d)
                    if (e + d < 0 || e + d >= M::PF || F[e + d] < 0)
                        return -2;
                for (int d = -2; d <= 2; ++d)
                    if (d != 0 && F[e + d] != F[e] + d)
                        return -2;
                return F[e];
            };
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                CHECK(w.ld >= 0 && w.ld < M::PD, "D slot out of range");
                D[w.ld] = d1x_tag(w.lf);
                for (int s = 0; s < M::DS; ++s)
                    if (w.dlf[s] >= 0) {
                        CHECK(w.dld[s] >= 0 && w.dld[s] < M::PD, "D halo slot out of range");
                        CHECK(D[w.dld[s]] == -1, "D halo slot written twice");
                        D[w.dld[s]] = d1x_tag(w.dlf[s]);
                    }
            }
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                if (!w.active)
                    continue;
                const int i = w.i, j = w.j;
                for (int d = -2; d <= 2; ++d) {
                    CHECK(F[w.lf + d] == elem(B, i + d, j, kk), "mixed x tap");
                    CHECK(F[w.lf + d * M::LX] == elem(B, i, j + d, kk), "mixed y tap");
                    CHECK(D[w.ld + d * TX] == elem(B, i, j + d, kk), "D1_x at row %d of (%d,%d,%d)", d, i, j, kk);
                }
                if (kk >= P.z0 + 2) {
                    const int64_t c = w.point(B, kk - 2);
                    CHECK(c == elem(B, i, j, kk - 2), "mixed store offset");
                    written[c]++;
                }
            }
        }
    }
    for (int k = -g; k < nz + g; ++k)
        for (int j = -g; j < ny + g; ++j)
            for (int i = -g; i < nx + g; ++i) {
                const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                CHECK(written[elem(B, i, j, k)] == (in ? 1 : 0), "mixed point (%d,%d,%d) stored %d times", i, j, k,
                      written[elem(B, i, j, k)]);
            }
}

// the fused stage-pair traversal (k_rk4_pair): first stage on the whole
// TXE x TYE region from a 4-plane ring, second stage two planes behind on
// the inner tile from a 3-plane ring, periodic addressing.  Tags encode a
// point (wrapped into the box) and the stage that produced it.  The whole
// RK4 step (k_rk4_step4) walks the same widened tile, also with 68-point
// rows, where the threads past the tile's 15 rows repeat its last point.
static int mod3h(int p)
{
    const int r = p % 3;
    return r < 0 ? r + 3 : r;
}

template <int TXE, int NW>
static void run_pair(int nx, int ny, int nz, int g, int padx, int tz_req)
{
    using T = Tile<TXE, NW>;
    constexpr int TYE = T::TY;
    constexpr int TXO = TXE - 4, TYO = TYE - 4;
    constexpr int P1 = T::LY * T::LX, P2 = TXE * TYE;
    DevBox B{};
    B.n[0] = nx;
    B.n[1] = ny;
    B.n[2] = nz;
    B.g = g;
    B.sy = nx + 2 * g + padx;
    B.sz = B.sy * (ny + 2 * g);
    B.tz = tz_req > 0 && tz_req < nz ? tz_req : nz;
    B.tiles[0] = (nx + TXO - 1) / TXO;
    B.tiles[1] = (ny + TYO - 1) / TYO;
    B.tiles[2] = (nz + B.tz - 1) / B.tz;
    const int64_t total = B.sz * (nz + 2 * g);
    std::vector<int> written(total, 0);
    const int nitems = B.tiles[0] * B.tiles[1] * B.tiles[2];
    auto tag = [&](int i, int j, int k, int stage) -> int64_t {
        return elem(B, wrap_index(i, nx), wrap_index(j, ny), wrap_index(k, nz)) * 4 + stage;
    };
    std::vector<int64_t> ring1(4 * P1), ring2(3 * P2);
    for (int item = 0; item < nitems; ++item) {
        const ItemPos P = item_pos(B, item, TXO, TYO);
        ItemPos Pe = P;
        Pe.x0 -= 2;
        Pe.y0 -= 2;
        std::vector<Walker<TXE, NW, true, false>> W;
        for (int t = 0; t < T::NT; ++t)
            W.emplace_back(B, Pe, tile_thread<TXE, NW>(t));
        std::vector<int64_t> qa(T::NT * 5, -1), qb(T::NT * 5, -1);
        std::fill(ring1.begin(), ring1.end(), -1);
        std::fill(ring2.begin(), ring2.end(), -1);
        for (int f = P.z0 - 4; f <= P.z1 + 3; ++f) {
            // loads and ring-1 writes (before the barrier)
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                const int64_t e = w.col + w.zoff(f);
                CHECK(e >= 0 && e < total, "pair load out of range");
                for (int d = 0; d < 4; ++d)
                    qa[t * 5 + d] = qa[t * 5 + d + 1];
                qa[t * 5 + 4] = tag(w.i, w.j, f, 0);
                CHECK(e * 4 == tag(w.i, w.j, f, 0), "pair own column address");
                int64_t *R1 = &ring1[(f & 3) * P1];
                R1[w.lc] = qa[t * 5 + 4];
                for (int s = 0; s < T::HS; ++s) {
                    if (w.hl[s] < 0)
                        continue;
                    const int64_t h = w.hcol[s] + w.zoff(f);
                    CHECK(h >= 0 && h < total, "pair halo out of range");
                    R1[w.hl[s]] = h * 4;
                }
            }
            const int p1 = f - 2, p2 = f - 4;
            // first stage at p1, every lane
            if (p1 >= P.z0 - 2) {
                for (int t = 0; t < T::NT; ++t) {
                    const auto &w = W[t];
                    const int64_t *L = &ring1[(p1 & 3) * P1];
                    for (int d = -2; d <= 2; ++d) {
                        CHECK(L[w.lc + d] == tag(w.i + d, w.j, p1, 0), "pair stage-1 x tap");
                        CHECK(L[w.lc + d * T::LX] == tag(w.i, w.j + d, p1, 0), "pair stage-1 y tap");
                        CHECK(qa[t * 5 + 2 + d] == tag(w.i, w.j, p1 + d, 0), "pair stage-1 z tap");
                    }
                    const int tl = tile_thread<TXE, NW>(t), lx = tl % TXE, ly = tl / TXE;
                    CHECK(ly * TXE + lx < P2, "pair ring-2 slot out of range");
                    ring2[mod3h(p1) * P2 + ly * TXE + lx] = tag(w.i, w.j, p1, 1);
                    for (int d = 0; d < 4; ++d)
                        qb[t * 5 + d] = qb[t * 5 + d + 1];
                    qb[t * 5 + 4] = tag(w.i, w.j, p1, 1);
                }
            }
            // second stage at p2, output lanes
            for (int t = 0; t < T::NT; ++t) {
                const auto &w = W[t];
                const int tl = tile_thread<TXE, NW>(t), lx = tl % TXE, ly = tl / TXE;
                const bool out = lx >= 2 && lx < TXE - 2 && ly >= 2 && ly < TYE - 2 && w.i < nx && w.j < ny;
                if (!(out && p2 >= P.z0 && p2 < P.z1))
                    continue;
                CHECK(w.i >= 0 && w.j >= 0, "output lane outside the box");
                const int l2 = ly * TXE + lx;
                const int64_t *L = &ring2[mod3h(p2) * P2];
                for (int d = -2; d <= 2; ++d) {
                    CHECK(L[l2 + d] == tag(w.i + d, w.j, p2, 1), "pair stage-2 x tap");
                    CHECK(L[l2 + d * TXE] == tag(w.i, w.j + d, p2, 1), "pair stage-2 y tap");
                    CHECK(qb[t * 5 + 2 + d] == tag(w.i, w.j, p2 + d, 1), "pair stage-2 z tap");
                }
                CHECK(qa[t * 5 + 0] == tag(w.i, w.j, p2, 0), "pair u_n at the output plane");
                const int64_t c = w.point(B, p2);
                CHECK(c == elem(B, w.i, w.j, p2), "pair store offset");
                written[c]++;
            }
        }
    }
    for (int k = -g; k < nz + g; ++k)
        for (int j = -g; j < ny + g; ++j)
            for (int i = -g; i < nx + g; ++i) {
                const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                CHECK(written[elem(B, i, j, k)] == (in ? 1 : 0), "pair point (%d,%d,%d) stored %d times", i, j, k,
                      written[elem(B, i, j, k)]);
            }
}

// the ghost-fill enumeration: every ghost point of the shell exactly once,
// never an interior point, and every source an interior point
static void ghost_shell(int nx, int ny, int nz, int g)
{
    DevBox B{};
    B.n[0] = nx;
    B.n[1] = ny;
    B.n[2] = nz;
    B.g = g;
    B.sy = nx + 2 * g;
    B.sz = B.sy * (ny + 2 * g);
    const int64_t total = B.sz * (nz + 2 * g);
    std::vector<int> hit(total, 0);
    const int64_t cnt = ghost_count(B);
    for (int64_t t = -1; t < cnt + 300; ++t) {
        int i = 0, j = 0, k = 0;
        const bool ok = ghost_point(B, t, i, j, k);
        CHECK(ok == (t >= 0 && t < cnt), "ghost_point validity at %lld", (long long)t);
        if (!ok)
            continue;
        CHECK(i >= -g && i < nx + g && j >= -g && j < ny + g && k >= -g && k < nz + g, "ghost out of the array");
        const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
        CHECK(!in, "interior point (%d,%d,%d) enumerated as ghost", i, j, k);
        hit[elem(B, i, j, k)]++;
        const int si = wrap_index(i, nx), sj = wrap_index(j, ny), sk = wrap_index(k, nz);
        CHECK(si >= 0 && si < nx && sj >= 0 && sj < ny && sk >= 0 && sk < nz, "source not interior");
    }
    for (int k = -g; k < nz + g; ++k)
        for (int j = -g; j < ny + g; ++j)
            for (int i = -g; i < nx + g; ++i) {
                const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                CHECK(hit[elem(B, i, j, k)] == (in ? 0 : 1), "ghost (%d,%d,%d) hit %d times", i, j, k,
                      hit[elem(B, i, j, k)]);
            }
}


// the row-register traversal: per item and wavefront, the loads of every
// plane (RY rows at plane p+2, two rows either side at plane p, the x halo
// on lanes 0..3), the wavefront-wide shifts that hand x taps between lanes,
// the per-row z queues and the stores
template <int WX, int WY, int RY, bool WRAP>
static void run_rows_check(int nx, int ny, int nz, int g, int padx, int pady, int tz_req)
{
    using RW = RowWalker<WX, WY, RY, WRAP>;
    DevBox B{};
    B.n[0] = nx;
    B.n[1] = ny;
    B.n[2] = nz;
    B.g = g;
    B.sy = nx + 2 * g + padx;
    B.sz = B.sy * (ny + 2 * g + pady);
    B.tz = tz_req > 0 && tz_req < nz ? tz_req : nz;
    B.tiles[0] = (nx + RW::TXE - 1) / RW::TXE;
    B.tiles[1] = (ny + RW::TYE - 1) / RW::TYE;
    B.tiles[2] = (nz + B.tz - 1) / B.tz;
    const int64_t total = B.sz * (nz + 2 * g);
    std::vector<int> written(total, 0);
    const int nitems = B.tiles[0] * B.tiles[1] * B.tiles[2];
    auto expect = [&](int i, int j, int k) -> int64_t {
        if (WRAP)
            return elem(B, wrapi(i, nx), wrapi(j, ny), wrapi(k, nz));
        return elem(B, i, j, k);
    };
    auto check_read = [&](int64_t e, const char *what) {
        CHECK(e >= 0 && e < total, "rows: %s read %lld outside [0,%lld)", what, (long long)e, (long long)total);
        if (e < 0 || e >= total)
            return;
        const int k = (int)(e / B.sz) - g, j = (int)(e % B.sz / B.sy) - g, i = (int)(e % B.sy) - g;
        if (WRAP)
            CHECK(i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz, "rows: %s read a ghost (%d,%d,%d)", what, i,
                  j, k);
        else
            CHECK(i >= -2 && i < nx + 2 && j >= -2 && j < ny + 2 && k >= -2 && k < nz + 2,
                  "rows: %s read beyond the radius-2 shell (%d,%d,%d)", what, i, j, k);
    };
    for (int item = 0; item < nitems; ++item) {
        const ItemPos P = item_pos(B, item, RW::TXE, RW::TYE);
        CHECK(P.z0 < P.z1 && P.z1 <= nz, "rows: empty or overlong z range");
        for (int wave = 0; wave < RW::NW; ++wave) {
            std::vector<RW> L;
            for (int lane = 0; lane < 64; ++lane)
                L.emplace_back(B, P, wave, lane);
            bool live = L[0].live;
            for (int lane = 1; lane < 64; ++lane)
                CHECK(L[lane].live == live && L[lane].j0 == L[0].j0, "rows: wavefront-uniform values differ");
            if (!live)
                continue;
            // tags: q[lane][r][0..4], per-plane buffers
            std::vector<int64_t> q(64 * RY * 5, -1);
            auto Q = [&](int lane, int r, int d) -> int64_t & { return q[(lane * RY + r) * 5 + d]; };
            for (int lane = 0; lane < 64; ++lane)
                for (int r = 0; r < RY; ++r)
                    for (int d = 0; d < 4; ++d) {
                        const int64_t e = L[lane].xc + L[lane].roff[r + 2] + L[lane].zoff(P.z0 - 2 + d);
                        check_read(e, "queue warm-up");
                        Q(lane, r, d + 1) = e;
                    }
            for (int k = P.z0; k < P.z1; ++k) {
                // loads of plane k (the kernel issues them two planes ahead; the addresses are these)
                std::vector<int64_t> c(64 * RY), ym(64 * 2), yp(64 * 2), h(64 * RY, -1);
                for (int lane = 0; lane < 64; ++lane) {
                    const RW &w = L[lane];
                    for (int r = 0; r < RY; ++r) {
                        c[lane * RY + r] = w.xc + w.roff[r + 2] + w.zoff(k + 2);
                        check_read(c[lane * RY + r], "row");
                        if (lane < 4) {
                            h[lane * RY + r] = w.hx + w.roff[r + 2] + w.zoff(k);
                            check_read(h[lane * RY + r], "x halo");
                        }
                        if (w.active_x && w.row_in(r)) {
                            const int64_t pt = w.point(B, r, k);
                            CHECK(pt == elem(B, w.i, w.j0 + r, k), "rows: pointwise offset");
                        }
                    }
                    for (int t = 0; t < 2; ++t) {
                        ym[lane * 2 + t] = w.xc + w.roff[t] + w.zoff(k);
                        yp[lane * 2 + t] = w.xc + w.roff[RY + 2 + t] + w.zoff(k);
                        check_read(ym[lane * 2 + t], "y halo");
                        check_read(yp[lane * 2 + t], "y halo");
                    }
                }
                for (int lane = 0; lane < 64; ++lane)
                    for (int r = 0; r < RY; ++r) {
                        for (int d = 0; d < 4; ++d)
                            Q(lane, r, d) = Q(lane, r, d + 1);
                        Q(lane, r, 4) = c[lane * RY + r];
                    }
                for (int r = 0; r < RY; ++r) {
                    // wavefront shifts: lane l reads lane l-1 (shr) or l+1 (shl); edge lanes take the halo
                    std::vector<int64_t> xm1(64), xm2(64), xp1(64), xp2(64);
                    for (int l = 0; l < 64; ++l)
                        xm1[l] = l >= 1 ? Q(l - 1, r, 2) : h[1 * RY + r];
                    for (int l = 0; l < 64; ++l)
                        xm2[l] = l >= 1 ? xm1[l - 1] : h[0 * RY + r];
                    for (int l = 0; l < 64; ++l)
                        xp1[l] = l <= 62 ? Q(l + 1, r, 2) : h[2 * RY + r];
                    for (int l = 0; l < 64; ++l)
                        xp2[l] = l <= 62 ? xp1[l + 1] : h[3 * RY + r];
                    for (int l = 0; l < 64; ++l) {
                        const RW &w = L[l];
                        if (!(w.active_x && w.row_in(r)))
                            continue;
                        const int i = w.i, j = w.j0 + r;
                        const int64_t ym2 = r >= 2 ? Q(l, r - 2, 2) : ym[l * 2 + r];
                        const int64_t ym1 = r >= 1 ? Q(l, r - 1, 2) : ym[l * 2 + 1];
                        const int64_t yp1 = r + 1 < RY ? Q(l, r + 1, 2) : yp[l * 2 + (r + 1 - RY)];
                        const int64_t yp2 = r + 2 < RY ? Q(l, r + 2, 2) : yp[l * 2 + (r + 2 - RY)];
                        CHECK(Q(l, r, 2) == expect(i, j, k), "rows: centre tag at (%d,%d,%d)", i, j, k);
                        CHECK(xm1[l] == expect(i - 1, j, k) && xm2[l] == expect(i - 2, j, k), "rows: x- taps at (%d,%d,%d)",
                              i, j, k);
                        CHECK(xp1[l] == expect(i + 1, j, k) && xp2[l] == expect(i + 2, j, k), "rows: x+ taps at (%d,%d,%d)",
                              i, j, k);
                        CHECK(ym2 == expect(i, j - 2, k) && ym1 == expect(i, j - 1, k), "rows: y- taps at (%d,%d,%d)", i,
                              j, k);
                        CHECK(yp1 == expect(i, j + 1, k) && yp2 == expect(i, j + 2, k), "rows: y+ taps at (%d,%d,%d)", i,
                              j, k);
                        for (int d = -2; d <= 2; ++d)
                            if (d)
                                CHECK(Q(l, r, 2 + d) == expect(i, j, k + d), "rows: z tap %d at (%d,%d,%d)", d, i, j, k);
                        const int64_t pt = w.point(B, r, k);
                        if (pt >= 0 && pt < total)
                            written[pt]++;
                    }
                }
            }
        }
    }
    for (int k = -g; k < nz + g; ++k)
        for (int j = -g; j < ny + g; ++j)
            for (int i = -g; i < nx + g; ++i) {
                const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
                const int cnt = written[elem(B, i, j, k)];
                CHECK(cnt == (in ? 1 : 0), "rows: point (%d,%d,%d) stored %d times", i, j, k, cnt);
            }
}

template <int WX, int RY>
static void row_shapes()
{
    const int S[][7] = {
        // nx ny nz g padx pady tz
        {32, 32, 32, 2, 0, 0, 0},  {37, 19, 23, 2, 3, 1, 16}, {5, 7, 3, 2, 0, 0, 2},  {1, 1, 1, 2, 0, 0, 0},
        {2, 3, 2, 3, 1, 0, 1},     {70, 9, 5, 3, 6, 2, 4},    {130, 9, 7, 2, 14, 0, 5}, {300, 6, 4, 2, 4, 0, 3},
        {64, 8, 9, 4, 0, 0, 32},   {256, 5, 6, 2, 12, 0, 16},
    };
    for (auto &s : S) {
        run_rows_check<WX, 4 / WX, RY, false>(s[0], s[1], s[2], s[3], s[4], s[5], s[6]);
        run_rows_check<WX, 4 / WX, RY, true>(s[0], s[1], s[2], s[3], s[4], s[5], s[6]);
    }
}

template <int TX, int NW>
static void shapes()
{
    const int S[][7] = {
        // nx ny nz g padx pady tz
        {32, 32, 32, 2, 0, 0, 0},   {32, 32, 32, 2, 12, 0, 8},  {37, 19, 23, 2, 3, 1, 16},
        {5, 7, 3, 2, 0, 0, 2},      {1, 1, 1, 2, 0, 0, 0},      {2, 3, 2, 3, 1, 0, 1},
        {70, 9, 5, 3, 6, 2, 4},     {16, 48, 11, 2, 0, 0, 64},  {64, 8, 9, 4, 0, 0, 3},
        {129, 17, 6, 2, 15, 0, 32},
    };
    for (auto &s : S) {
        run<TX, NW, false>(s[0], s[1], s[2], s[3], s[4], s[5], s[6]);
        run<TX, NW, true>(s[0], s[1], s[2], s[3], s[4], s[5], s[6]);
        run_mixed<TX, NW>(s[0], s[1], s[2], s[3], s[4], s[6]);
    }
}

// The per-XCD work queue of the batched kernels, with the workgroups'
// calls interleaved at random: every item is handed out exactly once, every
// workgroup stops within nitems + nq calls, and a workgroup's first item
// comes from its own range while that range lasts.
static void queue_check(int nitems, int nq, int grid, unsigned seed)
{
    std::vector<int> cnt(1 + nq, 0), got(nitems, 0);
    const ItemQueue Q{cnt.data(), nitems, nq};
    std::vector<int> q(grid), left(grid, nq), calls(grid, 0), first(grid, -1);
    std::vector<char> done(grid, 0);
    for (int b = 0; b < grid; ++b)
        q[b] = b % nq;
    int running = grid;
    unsigned x = seed;
    auto add = [](int *p) { return (*p)++; };
    while (running > 0) {
        x = x * 1103515245u + 12345u;
        int b = (int)((x >> 8) % (unsigned)grid);
        while (done[b])
            b = (b + 1) % grid;
        const int start_q = q[b];
        const int lo = queue_lo(start_q, nitems, nq), hi = queue_lo(start_q + 1, nitems, nq);
        const bool own_left = cnt[1 + start_q] < hi - lo;
        const int it = queue_next(Q, q[b], left[b], add);
        ++calls[b];
        CHECK(calls[b] <= nitems + nq + 1, "queue: workgroup %d does not stop", b);
        if (it >= nitems) {
            done[b] = 1;
            --running;
            continue;
        }
        CHECK(it >= 0, "queue: negative item");
        if (it >= 0) {
            got[it]++;
            if (first[b] < 0) {
                first[b] = it;
                if (own_left)
                    CHECK(it >= lo && it < hi, "queue: first item %d of workgroup %d not in its range", it, b);
            }
        }
    }
    for (int i = 0; i < nitems; ++i)
        CHECK(got[i] == 1, "queue: item %d handed out %d times", i, got[i]);
}

// The whole-step kernel's balanced runs: over every workgroup the pieces
// cover each (tile, plane) of the box exactly once, each piece lies in one
// tile and is a non-empty z range inside the box.
static void runs_check(int nx, int ny, int nz, int txo, int tyo, int run)
{
    DevBox B{};
    B.n[0] = nx;
    B.n[1] = ny;
    B.n[2] = nz;
    B.tiles[0] = (nx + txo - 1) / txo;
    B.tiles[1] = (ny + tyo - 1) / tyo;
    const int ntile = B.tiles[0] * B.tiles[1];
    const int64_t total = (int64_t)ntile * nz;
    const int64_t grid = (total + run - 1) / run;
    std::vector<int> seen(total, 0);
    for (int64_t g = 0; g < grid; ++g) {
        int64_t s = g * run;
        const int64_t e = s + run < total ? s + run : total;
        ItemPos P;
        int pieces = 0;
        while (run_piece(B, txo, tyo, s, e, P)) {
            ++pieces;
            CHECK(P.z0 >= 0 && P.z0 < P.z1 && P.z1 <= nz, "run piece z range [%d,%d)", P.z0, P.z1);
            CHECK(P.x0 % txo == 0 && P.x0 < nx && P.y0 % tyo == 0 && P.y0 < ny, "run piece tile origin");
            const int t = P.x0 / txo + (P.y0 / tyo) * B.tiles[0];
            for (int k = P.z0; k < P.z1; ++k)
                if (t >= 0 && t < ntile && k >= 0 && k < nz)
                    seen[(int64_t)t * nz + k]++;
            CHECK(pieces <= run / nz + 2, "run split into too many pieces");
        }
    }
    for (int64_t i = 0; i < total; ++i)
        CHECK(seen[i] == 1, "tile-plane %lld covered %d times", (long long)i, seen[i]);
}

int main()
{
    const int RS[][6] = {{256, 256, 256, 60, 12, 110}, {256, 256, 256, 28, 12, 64}, {5, 7, 3, 60, 12, 2},
                         {70, 9, 5, 28, 28, 1},         {1, 1, 1, 60, 4, 16},       {97, 33, 41, 60, 4, 1000},
                         {32, 32, 32, 28, 12, 1},       {48, 48, 48, 28, 12, 2},    {96, 96, 96, 28, 12, 6},
                         {256, 256, 256, 64, 11, 96},   {70, 33, 17, 64, 11, 5}};
    for (auto &r : RS)
        runs_check(r[0], r[1], r[2], r[3], r[4], r[5]);
    const int QS[][3] = {{1000, 8, 64}, {7, 8, 3}, {0, 8, 4}, {1, 8, 16}, {5000, 8, 1}, {123, 1, 9}, {97, 15, 40}};
    for (auto &s : QS)
        for (unsigned seed = 1; seed <= 3; ++seed)
            queue_check(s[0], s[1], s[2], seed);
    const int G[][4] = {{32, 32, 32, 2}, {5, 7, 6, 3}, {70, 9, 5, 3}, {2, 2, 2, 2}, {3, 17, 4, 3}, {1, 1, 1, 2}};
    for (auto &s : G)
        ghost_shell(s[0], s[1], s[2], s[3]);
    const int PS[][6] = {{32, 32, 32, 2, 0, 16}, {37, 19, 23, 2, 3, 8}, {5, 7, 3, 2, 0, 2}, {1, 2, 1, 2, 0, 0},
                         {70, 9, 5, 3, 6, 64}, {28, 12, 17, 2, 0, 32}};
    for (auto &s : PS) {
        run_pair<32, 8>(s[0], s[1], s[2], s[3], s[4], s[5]);
        run_pair<64, 8>(s[0], s[1], s[2], s[3], s[4], s[5]);
        run_pair<64, 16>(s[0], s[1], s[2], s[3], s[4], s[5]);
        run_pair<32, 16>(s[0], s[1], s[2], s[3], s[4], s[5]);
        run_pair<68, 16>(s[0], s[1], s[2], s[3], s[4], s[5]);
    }
    run_pair<68, 16>(256, 24, 9, 2, 0, 4);
    run_pair<68, 16>(131, 23, 6, 2, 5, 0);
    row_shapes<4, 4>();
    row_shapes<4, 2>();
    row_shapes<2, 4>();
    row_shapes<2, 2>();
    row_shapes<1, 4>();
    row_shapes<1, 2>();
    shapes<64, 4>();
    shapes<64, 8>();
    shapes<32, 4>();
    shapes<32, 8>();
    shapes<16, 4>();
    shapes<16, 8>();
    if (fails) {
        fprintf(stderr, "%d failures\n", fails);
        return 1;
    }
    printf("tile walk OK\n");
    return 0;
}
