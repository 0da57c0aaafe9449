// s4_internal.h -- types and tile geometry shared by the HIP kernels and the
// host side of libsten4 (not installed; the public ABI is include/sten4.h).
//
// Traversal of one box (the GPU form of the paper's LoopControl split of a
// loop's index space, Sec. III-A): the interior is cut into work items, each
// an xy tile of TX x TY points and a chunk of TZ consecutive z planes.  A
// workgroup owns one item at a time; its 64-wide wavefronts cover TX
// consecutive x points (unit stride, so loads coalesce) and 64/TX rows; it
// marches along z keeping the column's five stencil values (z-2..z+2) in
// registers and stages the current plane, with a two-point halo in x and y,
// in LDS.  Lanes outside the box do the loads (at readable addresses) but
// store nothing: the edge mask of Sec. IV-C4.
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define S4_HD __host__ __device__
#else
#define S4_HD
#endif

namespace s4 {

// kinds of per-point work that ride on the tile traversal
enum Op : int {
    OP_RHS = 0,     // rho_t = c2 * L(u)                      (ghosts read)
    OP_STAGE = 1,   // one fused RK4 stage                     (periodic addressing)
    OP_ADJRHS = 2,  // (L(c2*lrho), lu)                        (periodic addressing)
    OP_ADJSTEP = 3, // backward RK4 step (two passes of k_adj2, not a tile-traversal op)
    OP_COUNT = 4
};

// One box as the kernels see it: geometry, stencil coefficients, the tile
// decomposition and the op's field pointers.  All fields of a box share its
// strides.  Passed by value to single-box kernels and stored as a device
// table for the persistent batched kernels.
struct DevBox {
    int32_t n[3];
    int32_t g;
    int64_t sy, sz;        // element strides along y and z (x stride is 1)
    double cx, cy, cz;     // 1 / (12 h_a^2)
    double c0;             // -30 (cx + cy + cz)
    int32_t tiles[3];      // tiles along x and y, z chunks
    int32_t tz;            // z-chunk length
    int32_t item0;         // index of this box's first work item in the launch
    int32_t pad_;
    const double *in;      // stencil input
    const double *inmul;   // optional multiplier of the stencil input (c^2), pointwise
    const double *p[7];    // op inputs (pointwise)
    double *q[5];          // op outputs (pointwise)
};

// Arguments of one multi-field mixed-derivative launch (fields share B's
// layout; work item lin covers field lin / items, tile lin % items).
struct MixArgs {
    DevBox B;
    const double *f[8];
    double *out[8];
    double a[6];  // A_xx, A_yy, A_zz, A_xy + A_yx, A_xz + A_zx, A_yz + A_zy
    double d1[3]; // 1 / (12 h_a)
    double d2[3]; // 1 / (12 h_a^2)
    int32_t nfield;
    int32_t items;
};

// Scalars of one stage launch.  The backward step's passes (k_adj2) use
// a = dt, b = dt/6, a_next = dt/3, b_next = dt/2.
struct StageCoef {
    int stage;      // 1..4
    double a;       // dt * (1/2, 1/2, 1, -)  weight of k_s in the next stage input
    double b;       // dt * (1/6, 1/3, 1/3, 1/6)  weight of k_s in y_{n+1}
    double scale;   // unused by the kernels (set to 1)
    double b_next;
    double a_next;
};

// A workgroup tile of TX x TY points, one per thread.  TX = 68 (whole RK4
// steps on 1024 threads only): rows of 68 points, whose 64-point output rows
// cover a 256-point extent in four tiles; its 15 rows take 1020 threads, and
// the last four threads repeat thread 1019's loads, LDS writes and results.
template <int TX, int NW>
struct Tile {
    static constexpr int NT = NW * 64;         // threads per workgroup
    static constexpr int TY = NT / TX;         // rows per tile
    static constexpr int NTL = TX * TY;        // threads on tile points
    static constexpr int LX = TX + 4;          // LDS plane row length (2-point halo each side)
    static constexpr int LY = TY + 4;
    static constexpr int NH = 4 * (TX + TY);   // halo points per plane
    static constexpr int HS = (NH + NTL - 1) / NTL; // halo slots per thread
    static_assert(TX == 16 || TX == 32 || TX == 64 || (TX == 68 && NW == 16), "tile x extent");
    static_assert(NT % TX == 0 || TX == 68, "rows");
};

// the tile point of thread t (threads past the tile's whole rows take the last one)
template <int TX, int NW>
S4_HD inline int tile_thread(int t)
{
    return t < Tile<TX, NW>::NTL ? t : Tile<TX, NW>::NTL - 1;
}

// Position p along an axis of n interior points mapped to an index that may
// be read.  Callers never go below -2.  With `clamp`, points past n+1, which
// only lanes outside the box touch and whose values no radius-2 stencil
// uses, are clamped to n+1, so idle lanes re-read a line already in flight
// instead of fetching more rows; traversals whose outer lanes compute values
// that are used (the widened-tile stage pairs) pass clamp = false.  Periodic
// addressing then wraps into [0, n); ghost addressing keeps the index
// (ghosts -2 .. n+1) and always clamps.
S4_HD inline int readable(int p, int n, bool wrap, bool clamp = true)
{
    if (clamp || !wrap)
        p = p < n + 1 ? p : n + 1;
    if (wrap) {
        int r = p % n;
        return r < 0 ? r + n : r;
    }
    return p;
}

// element offset of point (i, j, k) from the box's ghost corner
S4_HD inline int64_t elem(const DevBox &B, int i, int j, int k)
{
    return (int64_t)(i + B.g) + (int64_t)(j + B.g) * B.sy + (int64_t)(k + B.g) * B.sz;
}

// work item (local to its box) -> tile origin and z range
struct ItemPos {
    int x0, y0, z0, z1;
};

S4_HD inline ItemPos item_pos(const DevBox &B, int local, int tx_extent, int ty_extent)
{
    ItemPos P;
    int tx = local % B.tiles[0];
    int rest = local / B.tiles[0];
    int ty = rest % B.tiles[1];
    int tzi = rest / B.tiles[1];
    P.x0 = tx * tx_extent;
    P.y0 = ty * ty_extent;
    P.z0 = tzi * B.tz;
    P.z1 = P.z0 + B.tz < B.n[2] ? P.z0 + B.tz : B.n[2];
    return P;
}

// Balanced work of the whole-step kernel: the box's xy tiles times its nz
// planes form one sequence (tile after tile, planes inside a tile), cut into
// runs of `run` planes, one run per workgroup, so every workgroup of a
// single-round launch gets the same work.  A run may end in one tile and go
// on in the next: run_piece gives the pieces of the run [s, e) one at a time
// (advancing s), each one tile and a z range; false once the run is done.
S4_HD inline bool run_piece(const DevBox &B, int txo, int tyo, int64_t &s, int64_t e, ItemPos &P)
{
    if (s >= e)
        return false;
    const int nz = B.n[2];
    const int t = (int)(s / nz);
    P.x0 = (t % B.tiles[0]) * txo;
    P.y0 = (t / B.tiles[0]) * tyo;
    P.z0 = (int)(s % nz);
    P.z1 = (int)(e - s < (int64_t)(nz - P.z0) ? P.z0 + (e - s) : nz);
    s += P.z1 - P.z0;
    return true;
}

// halo slot h of a tile: LDS (row, col) and the tile-relative point (dx, dy)
template <int TX, int NW>
S4_HD inline void halo_slot(int h, int &lrow, int &lcol, int &dx, int &dy)
{
    using T = Tile<TX, NW>;
    if (h < 2 * TX) { // two rows below the tile
        dy = h / TX - 2;
        dx = h % TX;
    } else if (h < 4 * TX) { // two rows above
        int e = h - 2 * TX;
        dy = T::TY + e / TX;
        dx = e % TX;
    } else if (h < 4 * TX + 2 * T::TY) { // two columns left
        int e = h - 4 * TX;
        dy = e / 2;
        dx = e % 2 - 2;
    } else { // two columns right
        int e = h - 4 * TX - 2 * T::TY;
        dy = e / 2;
        dx = TX + e % 2;
    }
    lrow = dy + 2;
    lcol = dx + 2;
}

// Per-thread addressing of one work item, shared by the kernels and the
// host-side geometry test: the thread's own column, its halo slots, the LDS
// slots it writes, and the element offsets of plane k.
template <int TX, int NW, bool WRAP, bool CLAMP = true>
struct Walker {
    using T = Tile<TX, NW>;
    int i, j;          // interior point of this thread (may lie outside the box)
    bool active;       // inside the box: computes and stores
    int64_t col;       // x,y part of the element offset of the thread's column
    int64_t hcol[T::HS];
    int hl[T::HS];     // LDS index of each halo slot, -1 if unused
    int lc;            // LDS index of the thread's own point
    int nz, g;
    int64_t sz;

    S4_HD Walker(const DevBox &B, const ItemPos &P, int t)
    {
        const int lx = t % TX, ly = t / TX;
        const int nx = B.n[0], ny = B.n[1];
        nz = B.n[2];
        g = B.g;
        sz = B.sz;
        i = P.x0 + lx;
        j = P.y0 + ly;
        active = i < nx && j < ny;
        col = (int64_t)(readable(i, nx, WRAP, CLAMP) + g) + (int64_t)(readable(j, ny, WRAP, CLAMP) + g) * B.sy;
        for (int s = 0; s < T::HS; ++s) {
            const int h = t + s * T::NTL;
            int lrow = 0, lcol = 0, dx = 0, dy = 0;
            if (h < T::NH)
                halo_slot<TX, NW>(h, lrow, lcol, dx, dy);
            hl[s] = h < T::NH ? lrow * T::LX + lcol : -1;
            hcol[s] = (int64_t)(readable(P.x0 + dx, nx, WRAP, CLAMP) + g) +
                      (int64_t)(readable(P.y0 + dy, ny, WRAP, CLAMP) + g) * B.sy;
        }
        lc = (ly + 2) * T::LX + (lx + 2);
    }
    // z part of the offset of plane k (k may be a stencil neighbour outside [0, nz))
    S4_HD int64_t zoff(int k) const { return (int64_t)(readable(k, nz, WRAP, CLAMP) + g) * sz; }
    // element offset of the thread's interior point in plane k (active threads only)
    S4_HD int64_t point(const DevBox &B, int k) const
    {
        return (int64_t)(i + g) + (int64_t)(j + g) * B.sy + (int64_t)(k + g) * sz;
    }
};


// ---------------------------------------------------------------------------
// Row-register traversal (the third kernel set).  A work item is an x extent
// of 64*WX points, a y extent of RY*WY rows and a z chunk; its WX x WY
// wavefronts work independently (no LDS, no barriers).  A wavefront owns 64
// consecutive x points (one per lane) of RY consecutive rows and marches
// along z keeping, per row, the five z values of its column in registers.
// Per plane it loads its RY rows, the two rows on either side (the y taps of
// the outer rows) and, on lanes 0..3, the x points x0-2, x0-1, x0+64, x0+65;
// x taps travel between lanes by wavefront-wide shifts.  Every lane loads
// the readable point of its own column (clamped or wrapped like the tile
// traversal), so the shifted values are the true taps of every lane inside
// the box.

template <int WX, int WY, int RY, bool WRAP>
struct RowWalker {
    static constexpr int NW = WX * WY;
    static constexpr int TXE = 64 * WX; // item x extent
    static constexpr int TYE = RY * WY; // item y extent
    int i;            // this lane's x
    int j0;           // first row of the wavefront
    bool active_x;    // lane inside the box along x
    bool live;        // the wavefront has points in the box
    int64_t xc;       // x part of the lane's column offset
    int64_t hx;       // x part of the halo point of lanes 0..3 (x0 on other lanes)
    int64_t roff[RY + 4]; // y parts of rows j0-2 .. j0+RY+1
    int nz, ny, g;
    int64_t sz;

    S4_HD RowWalker(const DevBox &B, const ItemPos &P, int wave, int lane)
    {
        const int nx = B.n[0];
        ny = B.n[1];
        nz = B.n[2];
        g = B.g;
        sz = B.sz;
        const int x0 = P.x0 + 64 * (wave % WX);
        j0 = P.y0 + RY * (wave / WX);
        live = x0 < nx && j0 < ny;
        i = x0 + lane;
        active_x = i < nx;
        xc = (int64_t)(readable(i, nx, WRAP) + g);
        const int h = lane < 2 ? x0 - 2 + lane : lane < 4 ? x0 + 62 + lane : x0;
        hx = (int64_t)(readable(h, nx, WRAP) + g);
        for (int t = 0; t < RY + 4; ++t)
            roff[t] = (int64_t)(readable(j0 - 2 + t, ny, WRAP) + g) * B.sy;
    }
    S4_HD int64_t zoff(int k) const { return (int64_t)(readable(k, nz, WRAP) + g) * sz; }
    // element offset of the lane's point in row j0 + r, plane k (inside the box only)
    S4_HD int64_t point(const DevBox &B, int r, int k) const
    {
        return (int64_t)(i + g) + (int64_t)(j0 + r + g) * B.sy + (int64_t)(k + g) * sz;
    }
    S4_HD bool row_in(int r) const { return j0 + r < ny; }
};

// ---------------------------------------------------------------------------
// Mixed-derivative traversal.  The LDS plane holds the plane being loaded
// with a full 5x5 neighbourhood (corners included, which the xy cross
// derivative reads); a second LDS plane holds D1_x of that plane on the
// tile's rows and its two rows above and below.

template <int TX, int NW>
struct MixTile {
    using T = Tile<TX, NW>;
    static constexpr int LX = TX + 4, LY = T::TY + 4;
    static constexpr int PF = LX * LY;          // f plane
    static constexpr int PD = TX * LY;          // D1_x plane
    static constexpr int NHC = T::NH + 16;      // halo incl. 16 corner points
    static constexpr int HS = (NHC + T::NT - 1) / T::NT;
    static constexpr int ND = 4 * TX;           // D1_x points on the halo rows
    static constexpr int DS = (ND + T::NT - 1) / T::NT;
};

// halo slot h of the mixed tile: edges as halo_slot, then the 16 corners
template <int TX, int NW>
S4_HD inline void halo_slot_c(int h, int &dx, int &dy)
{
    using T = Tile<TX, NW>;
    if (h < T::NH) {
        int lrow, lcol;
        halo_slot<TX, NW>(h, lrow, lcol, dx, dy);
        return;
    }
    const int e = h - T::NH;
    const int ox = e % 4, oy = e / 4;
    dx = ox < 2 ? ox - 2 : TX + ox - 2;
    dy = oy < 2 ? oy - 2 : T::TY + oy - 2;
}

template <int TX, int NW>
struct MixWalker {
    using T = Tile<TX, NW>;
    using M = MixTile<TX, NW>;
    int i, j;
    bool active;
    int64_t col;
    int64_t hcol[M::HS];
    int hl[M::HS];   // f-plane LDS index of each halo slot, -1 if unused
    int lf;          // f-plane LDS index of the own point
    int ld;          // D1_x-plane LDS index of the own point
    int dlf[M::DS];  // f-plane LDS index of each halo-row D1_x point, -1 if unused
    int dld[M::DS];  // D1_x-plane LDS index of it
    int nz, g;
    int64_t sz;

    S4_HD MixWalker(const DevBox &B, const ItemPos &P, int t)
    {
        const int lx = t % TX, ly = t / TX;
        const int nx = B.n[0], ny = B.n[1];
        nz = B.n[2];
        g = B.g;
        sz = B.sz;
        i = P.x0 + lx;
        j = P.y0 + ly;
        active = i < nx && j < ny;
        col = (int64_t)(readable(i, nx, false) + g) + (int64_t)(readable(j, ny, false) + g) * B.sy;
        for (int s = 0; s < M::HS; ++s) {
            const int h = t + s * T::NT;
            int dx = 0, dy = 0;
            if (h < M::NHC)
                halo_slot_c<TX, NW>(h, dx, dy);
            hl[s] = h < M::NHC ? (dy + 2) * M::LX + dx + 2 : -1;
            // rows and columns left of the box start at -2 >= -g; right and
            // above are clamped like the own point
            hcol[s] = (int64_t)(readable(P.x0 + dx, nx, false) + g) +
                      (int64_t)(readable(P.y0 + dy, ny, false) + g) * B.sy;
        }
        lf = (ly + 2) * M::LX + lx + 2;
        ld = (ly + 2) * TX + lx;
        for (int s = 0; s < M::DS; ++s) {
            const int h = t + s * T::NT;
            if (h < M::ND) {
                const int r = h / TX, dx = h % TX;
                const int dy = r < 2 ? r - 2 : T::TY + r - 2;
                dlf[s] = (dy + 2) * M::LX + dx + 2;
                dld[s] = (dy + 2) * TX + dx;
            } else {
                dlf[s] = dld[s] = -1;
            }
        }
    }
    S4_HD int64_t zoff(int k) const { return (int64_t)(readable(k, nz, false) + g) * sz; }
    S4_HD int64_t point(const DevBox &B, int k) const
    {
        return (int64_t)(i + g) + (int64_t)(j + g) * B.sy + (int64_t)(k + g) * sz;
    }
};

// Ghost shell of a box, enumerated for a one-thread-per-point fill: two z
// slabs over the full x, y extent, two y slabs over the full x extent and
// interior z, two x slabs over interior y, z.  Returns false for t past the
// last ghost point.
S4_HD inline int64_t ghost_count(const DevBox &B)
{
    const int64_t g = B.g, X = B.n[0] + 2 * g, Y = B.n[1] + 2 * g;
    return 2 * g * X * Y + (int64_t)B.n[2] * 2 * g * X + (int64_t)B.n[2] * B.n[1] * 2 * g;
}

S4_HD inline bool ghost_point(const DevBox &B, int64_t t, int &i, int &j, int &k)
{
    const int g = B.g, nx = B.n[0], ny = B.n[1], nz = B.n[2];
    const int64_t X = nx + 2 * g, Y = ny + 2 * g;
    const int64_t nA = 2 * g * X * Y, nB = (int64_t)nz * 2 * g * X, nC = (int64_t)nz * ny * 2 * g;
    if (t < 0)
        return false;
    if (t < nA) {
        const int64_t pz = t / (X * Y), rem = t % (X * Y);
        k = pz < g ? (int)pz - g : nz + (int)pz - g;
        j = (int)(rem / X) - g;
        i = (int)(rem % X) - g;
        return true;
    }
    if ((t -= nA) < nB) {
        k = (int)(t / (2 * g * X));
        const int64_t rem = t % (2 * g * X);
        const int r = (int)(rem / X);
        j = r < g ? r - g : ny + r - g;
        i = (int)(rem % X) - g;
        return true;
    }
    if ((t -= nB) < nC) {
        k = (int)(t / ((int64_t)ny * 2 * g));
        const int64_t rem = t % ((int64_t)ny * 2 * g);
        j = (int)(rem / (2 * g));
        const int cc = (int)(rem % (2 * g));
        i = cc < g ? cc - g : nx + cc - g;
        return true;
    }
    return false;
}

S4_HD inline int wrap_index(int p, int n)
{
    int r = p % n;
    return r < 0 ? r + n : r;
}

// One copy piece of a level's ghost exchange as the sync kernel sees it:
// n[0] x n[1] x n[2] points from field F[src] at element offset soff (then
// strides ssy, ssz) to field F[dst] at doff (strides dsy, dsz).  The piece
// owns workgroups blk0 .. blk0 + ceil(volume / 256) - 1 of the launch (a
// table of one piece index per workgroup maps them back).
struct SyncPiece {
    int32_t dst, src;
    int32_t n[3];
    int32_t blk0;
    int64_t doff, soff;
    int64_t dsy, dsz, ssy, ssz;
};

// Work queue of a persistent launch over a table of boxes.  The nitems items
// (box after box; inside a box x tiles, then y tiles, then z chunks, so that
// consecutive items are neighbours) are cut into nq contiguous ranges.
// Workgroup b starts on range b % nq: the hardware places workgroups on the
// XCDs round-robin, so with nq equal to the XCD count each range is worked
// under one L2 and neighbouring tiles share their halo lines there.  A
// workgroup whose range is used up takes items from the following ranges in
// turn, and stops after finding all nq ranges used up.  counter[0] counts
// finished workgroups and counter[1 + q] hands out range q; the last
// workgroup to finish clears them all, so each launch starts from zero
// without a memset.
constexpr int QUEUE_INTS = 16; // ints reserved per launch; nq <= QUEUE_INTS - 1

struct ItemQueue {
    int *counter; // 1 + nq ints, zero before the launch
    int nitems;
    int nq;
};

// first item of range q
S4_HD inline int queue_lo(int q, int nitems, int nq)
{
    return (int)((int64_t)nitems * q / nq);
}

// Next item of a workgroup, or Q.nitems once every range is used up.  q is
// the range being worked (start: workgroup index % Q.nq), left the ranges
// not yet found used up (start: Q.nq).  fetch_add(p) adds one to *p and
// returns the old value (an atomic on the GPU).
template <class FetchAdd>
S4_HD inline int queue_next(const ItemQueue &Q, int &q, int &left, FetchAdd fetch_add)
{
    while (left > 0) {
        const int lo = queue_lo(q, Q.nitems, Q.nq), hi = queue_lo(q + 1, Q.nitems, Q.nq);
        if (lo < hi) {
            const int i = fetch_add(&Q.counter[1 + q]);
            if (i < hi - lo)
                return lo + i;
        }
        q = q + 1 == Q.nq ? 0 : q + 1;
        --left;
    }
    return Q.nitems;
}

// split a launch of `nblocks` workgroups so that the hardware's round-robin
// placement (block b runs on XCD b % nxcd) gives each XCD a contiguous range
// of logical items: neighbouring tiles then share that XCD's L2.
S4_HD inline int xcd_remap(int b, int nblocks, int nxcd)
{
    if (nxcd <= 1 || nblocks < nxcd)
        return b;
    int q = nblocks / nxcd, r = nblocks % nxcd;
    int x = b % nxcd, l = b / nxcd;
    return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

} // namespace s4
