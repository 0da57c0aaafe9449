// s4_kernels.hip -- FP64 4th-order stencil kernels for gfx950.
//
// All stencil work rides on one traversal (see s4_internal.h): a workgroup
// takes an xy tile and a z chunk of a box, keeps each column's five
// z-values in registers, stages the current plane with its 2-point halo in
// LDS (double buffered, one barrier per plane) and hands the Laplacian at
// each interior point to a pointwise epilogue (the "op").  The path is bound
// by HBM bandwidth, not arithmetic, so there is no MFMA: the design goal is
// one HBM read of every input point and one write of every output point.
//
// Arithmetic: FP64 throughout, written with explicit fma() and compiled
// without automatic contraction, so every tile shape and launch mode
// produces bit-identical results.

#include "s4_internal.h"
#include "s4_launch.h"
#include "sten4.h"

#include <map>
#include <mutex>
#include <type_traits>

namespace s4 {

// L f at a point from its 13 taps (4th-order centred five-point formula per
// axis): sum_a (16 (f_{-1} + f_{+1}) - (f_{-2} + f_{+2}) - 30 f_0) / (12 h_a^2)
__device__ __forceinline__ double lap4(const DevBox &B, double c, double xm2, double xm1,
                                       double xp1, double xp2, double ym2, double ym1,
                                       double yp1, double yp2, double zm2, double zm1,
                                       double zp1, double zp2)
{
    double sx = fma(16.0, xm1 + xp1, -(xm2 + xp2));
    double sy = fma(16.0, ym1 + yp1, -(ym2 + yp2));
    double sz = fma(16.0, zm1 + zp1, -(zm2 + zp2));
    double r = B.c0 * c;
    r = fma(B.cx, sx, r);
    r = fma(B.cy, sy, r);
    r = fma(B.cz, sz, r);
    return r;
}

// lap4 in parts, with the same roundings: one axis's tap sum, then the sum
// over the axes
__device__ __forceinline__ double axis4(double m2, double m1, double p1, double p2)
{
    return fma(16.0, m1 + p1, -(m2 + p2));
}
__device__ __forceinline__ double lap4s(const DevBox &B, double c, double sx, double sy, double sz)
{
    double r = B.c0 * c;
    r = fma(B.cx, sx, r);
    r = fma(B.cy, sy, r);
    r = fma(B.cz, sz, r);
    return r;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also drains the
// wave's global loads and stores before the barrier; a kernel whose
// threads never read global memory written in the same launch needs only
// its LDS writes visible, and its loads and stores in flight keep flying.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Non-temporal store of v at byte offset off of the nbytes at base (a
// wave-uniform address), dropped by the hardware's buffer range check when
// off >= nbytes.  Lanes with nothing to store pass such an offset: the
// instruction still issues, so the number of memory operations that a later
// wait counts does not depend on which lanes store.
typedef unsigned int s4_u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned NO_STORE = 0x80000000u;

__device__ __forceinline__ void st_or_drop(double *base, unsigned nbytes, unsigned off, double v)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)nbytes, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(s4_u32x2, v), r, off, 0, 2 /* nt */);
}

// load through a buffer resource over one z plane of nbytes at base (an
// address uniform over the workgroup): the byte offset stays a 32-bit lane
// value across planes (AUX: cache policy bits, 2 = non-temporal)
template <int AUX>
__device__ __forceinline__ double ld_plane(const double *base, unsigned nbytes, unsigned off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base), 0, (int)nbytes, 0x00020000);
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}

__device__ __forceinline__ void st(double *p, double v)
{
    __builtin_nontemporal_store(v, p);
}

// load of a stream read only at the point itself: non-temporal, so it does
// not evict the stencil input's planes that neighbouring tiles still read
__device__ __forceinline__ double ldp(const double *p)
{
    return __builtin_nontemporal_load(p);
}

// ---------------------------------------------------------------------------
// pointwise epilogues, split in two so the loads of plane k+1 can be issued
// before plane k is computed.  pw_load reads the streams an op needs at the
// point c; pw_apply combines them with the stencil result and stores.
// center: the stencil input at the point (after the input transform);
// lap: L of the transformed input.

struct PW {
    double v[6];
};

template <int OPK>
__device__ __forceinline__ void pw_load(const DevBox &B, const StageCoef &K, int64_t c, PW &w)
{
    if constexpr (OPK == OP_RHS) {
        w.v[0] = B.p[0] ? ldp(B.p[0] + c) : 1.0; // c^2
    } else if constexpr (OPK == OP_STAGE) {
        w.v[0] = B.p[5] ? ldp(B.p[5] + c) : 1.0; // c^2
        w.v[1] = ldp(B.p[0] + c);                // rho_s
        if (K.stage == 2 || K.stage == 3) {
            w.v[2] = ldp(B.p[1] + c); // u_n
            w.v[3] = ldp(B.p[2] + c); // rho_n
        }
        if (K.stage >= 3) {
            w.v[4] = ldp(B.p[3] + c); // acc_u
            w.v[5] = ldp(B.p[4] + c); // acc_rho
        }
    } else if constexpr (OPK == OP_ADJRHS) {
        w.v[0] = ldp(B.p[0] + c); // lu
    }
}

template <int OPK>
__device__ __forceinline__ void pw_apply(const DevBox &B, const StageCoef &K, int64_t c, double center, double lap,
                                         const PW &w)
{
    if constexpr (OPK == OP_RHS) {
        // rho_t = c^2 L u   (c2 optional)
        st(B.q[0] + c, B.p[0] ? w.v[0] * lap : lap);
    } else if constexpr (OPK == OP_STAGE) {
        // k_s = (rho_s, c^2 L u_s).  Stage s writes the next stage input
        // y_n + a_s dt k_s; the running sum acc = y_n + dt sum_r b_r k_r is
        // first formed in stage 2 from y_2 = y_n + dt/2 k1 (so dt/6 k1 is
        // (y_2 - y_n)/3), which saves stage 1 writing it and stage 2 reading it.
        const double kr = B.p[5] ? w.v[0] * lap : lap;
        const double ku = w.v[1];
        if (K.stage == 1) { // y_s = y_n: u_n is the centre value, rho_n = rho_s
            st(B.q[0] + c, fma(K.a, ku, center));
            st(B.q[1] + c, fma(K.a, kr, ku));
        } else if (K.stage == 2) { // centre = u_2, ku = rho_2
            const double un = w.v[2], rn = w.v[3];
            st(B.q[0] + c, fma(K.a, ku, un));
            st(B.q[1] + c, fma(K.a, kr, rn));
            st(B.q[2] + c, fma(K.b, ku, fma(1.0 / 3.0, center - un, un)));
            st(B.q[3] + c, fma(K.b, kr, fma(1.0 / 3.0, ku - rn, rn)));
        } else if (K.stage == 3) {
            st(B.q[0] + c, fma(K.a, ku, w.v[2]));
            st(B.q[1] + c, fma(K.a, kr, w.v[3]));
            st(B.q[2] + c, fma(K.b, ku, w.v[4]));
            st(B.q[3] + c, fma(K.b, kr, w.v[5]));
        } else { // y_{n+1} = acc + dt/6 k4
            st(B.q[0] + c, fma(K.b, ku, w.v[4]));
            st(B.q[1] + c, fma(K.b, kr, w.v[5]));
        }
    } else if constexpr (OPK == OP_ADJRHS) {
        // F^T(lu, lrho) = (L(c^2 lrho), lu)
        st(B.q[0] + c, lap);
        st(B.q[1] + c, w.v[0]);
    }
}

// ---------------------------------------------------------------------------
// one work item: an xy tile marched over its z chunk.  Software pipelined:
// the loads step k needs (its halo and pointwise streams, the column's plane
// k+2) are issued PD steps ahead, right after a barrier, into one of PD
// buffers used in turn, so no register a load is still filling is copied.
// PD = 3 for the one-input ops (RHS, adjoint RHS); 1 for the RK4 stages,
// whose six pointwise streams would cost occupancy.

template <int TX, int NW, bool WRAP, int OPK>
__device__ __forceinline__ void run_item(const DevBox &B, const ItemPos &P, const StageCoef &K,
                                         double *lds)
{
    using T = Tile<TX, NW>;
    constexpr int PLANE = T::LY * T::LX;
    constexpr int PD = OPK == OP_STAGE ? 1 : 3;
    const Walker<TX, NW, WRAP> w(B, P, threadIdx.x);
    const int lc = w.lc;
    const double *in = B.in;
    const double *mul = B.inmul;

    // input transform: mul * in (mul optional)
    auto ldw = [&](int64_t e) -> double { return mul ? mul[e] * in[e] : in[e]; };
    struct Fetched {
        double q4, hv[T::HS];
        PW pw;
    };
    auto fetch = [&](int k, Fetched &X) {
        X.q4 = ldw(w.col + w.zoff(k + 2));
        const int64_t zo = w.zoff(k);
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0)
                X.hv[s] = ldw(w.hcol[s] + zo);
        if (w.active)
            pw_load<OPK>(B, K, w.point(B, k), X.pw);
    };
    // the column's planes k-2 .. k+2 at step k (q4 arrives with the step)
    double q0 = 0.0, q1 = ldw(w.col + w.zoff(P.z0 - 2)), q2 = ldw(w.col + w.zoff(P.z0 - 1)),
           q3 = ldw(w.col + w.zoff(P.z0)), q4 = ldw(w.col + w.zoff(P.z0 + 1));
    auto step = [&](const int k, Fetched &X) {
        q0 = q1;
        q1 = q2;
        q2 = q3;
        q3 = q4;
        q4 = X.q4;
        double *L = lds + ((k - P.z0) & 1) * PLANE;
        L[lc] = q2;
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0)
                L[w.hl[s]] = X.hv[s];
        const PW pw = X.pw;
        if (k + PD < P.z1)
            fetch(k + PD, X);
        lds_barrier();
        if (w.active) {
            const double lap = lap4(B, q2, L[lc - 2], L[lc - 1], L[lc + 1], L[lc + 2],
                                    L[lc - 2 * T::LX], L[lc - T::LX], L[lc + T::LX], L[lc + 2 * T::LX],
                                    q0, q1, q3, q4);
            pw_apply<OPK>(B, K, w.point(B, k), q2, lap, pw);
        }
    };
    Fetched F0, F1, F2;
    fetch(P.z0, F0);
    if constexpr (PD == 3) {
        if (P.z0 + 1 < P.z1)
            fetch(P.z0 + 1, F1);
        if (P.z0 + 2 < P.z1)
            fetch(P.z0 + 2, F2);
        for (int k = P.z0; k < P.z1; k += 3) {
            step(k, F0);
            if (k + 1 < P.z1)
                step(k + 1, F1);
            if (k + 2 < P.z1)
                step(k + 2, F2);
        }
    } else {
        (void)F1;
        (void)F2;
        for (int k = P.z0; k < P.z1; ++k)
            step(k, F0);
    }
}

template <int TX, int NW, bool WRAP, int OPK>
__global__ __launch_bounds__(NW * 64) void k_tiles_single(DevBox B, StageCoef K, int nxcd)
{
    using T = Tile<TX, NW>;
    __shared__ double lds[2 * T::LY * T::LX];
    const int item = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const ItemPos P = item_pos(B, item, TX, T::TY);
    run_item<TX, NW, WRAP, OPK>(B, P, K, lds);
}

// ---------------------------------------------------------------------------
// Pair-lane tiles: the tile traversal with two x points per lane, for the
// wave RHS on boxes whose rows hold an even number of interior points and
// start 16-byte aligned.  Every lane moves 16-byte vectors (its column, the
// halo pairs, the c^2 pair, the output pair) and reads its x taps as two
// 16-byte LDS words, so a wavefront covers 128 contiguous points of a row;
// the loads of a plane are issued PD planes ahead (6, or 4 with c^2 or two
// halo slots per lane), from PD buffers used in turn, and G planes share one
// barrier (3, or 2 where PD is 4).  Per point the arithmetic is that of run_item, so both give the
// same values bit for bit.  Tile: 2 TXL x TY points, TY = NW * 64 / TXL; the
// halo is two full rows below and above (corner pairs included) and one pair
// on each side of every tile row.

typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int TXL, int NW>
struct PairTile {
    static constexpr int NT = NW * 64;
    static constexpr int TY = NT / TXL;
    static constexpr int TXP = 2 * TXL;                // points along x
    static constexpr int LX = TXP + 4, LY = TY + 4;    // LDS plane (doubles)
    static constexpr int NH = 4 * (TXL + 2) + 2 * TY;  // halo pairs per plane
    static constexpr int HS = (NH + NT - 1) / NT;      // halo slots per lane
};

template <int TXL, int NW, bool HASC2>
__global__ __launch_bounds__(NW * 64, 4) void k_pairs_rhs(DevBox B, int nxcd)
{
    using T = PairTile<TXL, NW>;
    // six planes of loads in flight; four where the c^2 pairs or a second
    // halo slot would otherwise spill registers at four waves per SIMD
    constexpr int PLANE = T::LY * T::LX, PD = HASC2 || T::HS > 1 ? 4 : 6;
    __shared__ __attribute__((aligned(16))) double lds[(PD % 3 == 0 ? 6 : 4) * PLANE];
    const int item = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const ItemPos P = item_pos(B, item, T::TXP, T::TY);
    const int t = threadIdx.x, lx = t % TXL, ly = t / TXL;
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2], g = B.g;
    const int i = P.x0 + 2 * lx, j = P.y0 + ly;
    const bool active = i < nx && j < ny; // nx is even: the pair (i, i + 1) is inside or outside together
    // readable pair origins: x up to nx (the pair nx, nx + 1 is a ghost pair), y up to ny + 1
    const int64_t col = (int64_t)((i < nx ? i : nx) + g) + (int64_t)((j < ny + 1 ? j : ny + 1) + g) * B.sy;
    const int lc = (ly + 2) * T::LX + 2 * lx + 2;
    int hl[T::HS];
    int64_t hcol[T::HS];
#pragma unroll
    for (int s = 0; s < T::HS; ++s) {
        int h = t + s * T::NT;
        hl[s] = -1;
        hcol[s] = 0;
        if (h < T::NH) {
            int row, pc; // LDS row and pair column
            constexpr int RP = TXL + 2; // pairs per full row
            if (h < 4 * RP) {
                row = h / RP;
                row = row < 2 ? row : T::TY + row; // rows 0, 1 and TY + 2, TY + 3
                pc = h % RP;
            } else {
                const int e = h - 4 * RP;
                row = 2 + e / 2;
                pc = e % 2 ? RP - 1 : 0;
            }
            hl[s] = row * T::LX + 2 * pc;
            const int gx = P.x0 - 2 + 2 * pc, gy = P.y0 - 2 + row;
            hcol[s] = (int64_t)((gx < nx ? gx : nx) + g) + (int64_t)((gy < ny + 1 ? gy : ny + 1) + g) * B.sy;
        }
    }
    const double *in = B.in;
    const double *c2 = HASC2 ? B.p[0] : nullptr;
    auto zo = [&](int k) { return (int64_t)((k < nz + 1 ? k : nz + 1) + g) * B.sz; };
    auto ld2 = [&](const double *p) { return *(const dvec2 *)p; };
    struct Fetched {
        dvec2 q4, h[T::HS], c;
    };
    auto fetch = [&](int k, Fetched &X) {
        X.q4 = ld2(in + col + zo(k + 2));
        const int64_t z = zo(k);
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (hl[s] >= 0)
                X.h[s] = ld2(in + hcol[s] + z);
        if (HASC2 && active)
            X.c = __builtin_nontemporal_load((const dvec2 *)(c2 + col + z));
    };
    // the column at planes k - 2 .. k + 1 before plane k (k + 2 arrives with its fetch)
    dvec2 q1 = ld2(in + col + zo(P.z0 - 2)), q2 = ld2(in + col + zo(P.z0 - 1)), q3 = ld2(in + col + zo(P.z0)),
          q4 = ld2(in + col + zo(P.z0 + 1));
    Fetched F[PD];
#pragma unroll
    for (int p = 0; p < PD; ++p) {
        F[p].c = 0.0;
        if (P.z0 + p < P.z1)
            fetch(P.z0 + p, F[p]);
    }
    // the stencil of one plane from its LDS plane L and its column's five z
    // values a0 .. a4, stored
    auto plane = [&](const int k, const double *L, dvec2 a0, dvec2 a1, dvec2 a2, dvec2 a3, dvec2 a4, dvec2 cc) {
        const dvec2 xm = *(const dvec2 *)(L + lc - 2), xp = *(const dvec2 *)(L + lc + 2);
        const dvec2 ym2 = *(const dvec2 *)(L + lc - 2 * T::LX), ym1 = *(const dvec2 *)(L + lc - T::LX);
        const dvec2 yp1 = *(const dvec2 *)(L + lc + T::LX), yp2 = *(const dvec2 *)(L + lc + 2 * T::LX);
        dvec2 r;
        r.x = lap4(B, a2.x, xm.x, xm.y, a2.y, xp.x, ym2.x, ym1.x, yp1.x, yp2.x, a0.x, a1.x, a3.x, a4.x);
        r.y = lap4(B, a2.y, xm.y, a2.x, xp.x, xp.y, ym2.y, ym1.y, yp1.y, yp2.y, a0.y, a1.y, a3.y, a4.y);
        if (HASC2) {
            r.x = cc.x * r.x;
            r.y = cc.y * r.y;
        }
        __builtin_nontemporal_store(r, (dvec2 *)(B.q[0] + col + zo(k)));
    };
    // G planes per barrier: planes k .. k + G - 1 (from buffers p .. p + G - 1)
    // go to the G LDS planes of one half of the double buffer, so a
    // workgroup synchronises once per G planes.
    constexpr int G = PD % 3 == 0 ? 3 : 2; // planes per barrier
    auto stepg = [&](const int k, const int p) {
        // column values at planes k - 2 .. k + G + 1
        dvec2 a[G + 4];
        a[0] = q1;
        a[1] = q2;
        a[2] = q3;
        a[3] = q4;
#pragma unroll
        for (int m = 0; m < G; ++m)
            a[4 + m] = F[p + m].q4;
        double *L = lds + (((k - P.z0) / G) & 1) * G * PLANE;
        dvec2 cc[G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            if (m == 0 || k + m < P.z1) {
                *(dvec2 *)(L + m * PLANE + lc) = a[2 + m];
#pragma unroll
                for (int s = 0; s < T::HS; ++s)
                    if (hl[s] >= 0)
                        *(dvec2 *)(L + m * PLANE + hl[s]) = F[p + m].h[s];
            }
            cc[m] = F[p + m].c;
        }
#pragma unroll
        for (int m = 0; m < G; ++m)
            if (k + m + PD < P.z1)
                fetch(k + m + PD, F[p + m]);
        lds_barrier();
        if (active) {
#pragma unroll
            for (int m = 0; m < G; ++m)
                if (m == 0 || k + m < P.z1)
                    plane(k + m, L + m * PLANE, a[m], a[m + 1], a[m + 2], a[m + 3], a[m + 4], cc[m]);
        }
        q1 = a[G];
        q2 = a[G + 1];
        q3 = a[G + 2];
        q4 = a[G + 3];
    };
    for (int k = P.z0; k < P.z1; k += PD) {
#pragma unroll
        for (int p = 0; p < PD; p += G)
            if (k + p < P.z1)
                stepg(k + p, p);
    }
}

// next item of the calling workgroup (thread 0 only), see queue_next
__device__ inline int queue_take(const ItemQueue &Q, int &q, int &left)
{
    return queue_next(Q, q, left, [](int *p) { return atomicAdd(p, 1); });
}

// thread 0, after its workgroup's last item: the last workgroup clears the counters
__device__ inline void queue_finish(const ItemQueue &Q)
{
    __threadfence();
    if (atomicAdd(&Q.counter[0], 1) == (int)gridDim.x - 1)
        for (int q = 0; q <= Q.nq; ++q)
            atomicExch(&Q.counter[q], 0);
}

// box of global item `item`: last box with item0 <= item
__device__ inline int box_of(const DevBox *__restrict__ tab, int nbox, int item)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].item0 <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Persistent form: a fixed grid pulls the items of all boxes from the
// per-XCD work queue Q.
template <int TX, int NW, bool WRAP, int OPK>
__global__ __launch_bounds__(NW * 64) void k_tiles_batched(const DevBox *__restrict__ tab, int nbox, ItemQueue Q,
                                                          StageCoef K)
{
    using T = Tile<TX, NW>;
    __shared__ double lds[2 * T::LY * T::LX];
    __shared__ int s_item;
    int q = blockIdx.x % Q.nq, left = Q.nq;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_item = queue_take(Q, q, left);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= Q.nitems)
            break;
        const DevBox B = tab[box_of(tab, nbox, item)];
        const ItemPos P = item_pos(B, item - B.item0, TX, T::TY);
        run_item<TX, NW, WRAP, OPK>(B, P, K, lds);
    }
    if (threadIdx.x == 0)
        queue_finish(Q);
}


// ---------------------------------------------------------------------------
// Row-register traversal (RowWalker): x taps by wavefront-wide DPP shifts,
// y taps from the rows a wavefront holds (plus two rows either side), z taps
// from per-row register queues; the loads of planes k+1 and k+2 are in
// flight while plane k is computed (three plane buffers that rotate with a
// three-fold unrolled loop, so no buffer is copied).

// a double moved across the wavefront by one lane; lanes whose source lies
// outside the wavefront take `edge`
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double edge, double src)
{
    const uint64_t o = __builtin_bit_cast(uint64_t, edge), v = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

constexpr int DPP_WAVE_SHL1 = 0x130; // lane l reads lane l + 1
constexpr int DPP_WAVE_SHR1 = 0x138; // lane l reads lane l - 1

__device__ __forceinline__ double lane_value(double v, int l)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int RY, int OPK>
struct RowPlane {
    double c[RY];    // rows j0 .. j0+RY-1 at plane p+2 (transformed)
    double ym[2];    // rows j0-2, j0-1 at plane p
    double yp[2];    // rows j0+RY, j0+RY+1 at plane p
    double h[RY];    // x halo of each row at plane p (lanes 0..3)
    PW pw[RY];       // pointwise streams of each row at plane p
};

template <int WX, int WY, int RY, bool WRAP, int OPK>
__device__ __forceinline__ void run_rows(const DevBox &B, const ItemPos &P, const StageCoef &K, int wave, int lane)
{
    const RowWalker<WX, WY, RY, WRAP> w(B, P, wave, lane);
    if (!w.live)
        return;
    const double *in = B.in;
    const double *mul = B.inmul;
    auto ldw = [&](int64_t e) -> double { return mul ? mul[e] * in[e] : in[e]; };
    auto load = [&](int p, RowPlane<RY, OPK> &L) {
        const int64_t z2 = w.zoff(p + 2), z0 = w.zoff(p);
#pragma unroll
        for (int r = 0; r < RY; ++r)
            L.c[r] = ldw(w.xc + w.roff[r + 2] + z2);
        L.ym[0] = ldw(w.xc + w.roff[0] + z0);
        L.ym[1] = ldw(w.xc + w.roff[1] + z0);
        L.yp[0] = ldw(w.xc + w.roff[RY + 2] + z0);
        L.yp[1] = ldw(w.xc + w.roff[RY + 3] + z0);
#pragma unroll
        for (int r = 0; r < RY; ++r)
            L.h[r] = lane < 4 ? ldw(w.hx + w.roff[r + 2] + z0) : 0.0;
#pragma unroll
        for (int r = 0; r < RY; ++r)
            if (w.active_x && w.row_in(r))
                pw_load<OPK>(B, K, w.point(B, r, p), L.pw[r]);
    };
    // per-row z queues of the transformed input (planes k-2 .. k+2)
    double q[RY][5];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        q[r][1] = ldw(w.xc + w.roff[r + 2] + w.zoff(P.z0 - 2));
        q[r][2] = ldw(w.xc + w.roff[r + 2] + w.zoff(P.z0 - 1));
        q[r][3] = ldw(w.xc + w.roff[r + 2] + w.zoff(P.z0));
        q[r][4] = ldw(w.xc + w.roff[r + 2] + w.zoff(P.z0 + 1));
    }
    auto compute = [&](int k, const RowPlane<RY, OPK> &L) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int d = 0; d < 4; ++d)
                q[r][d] = q[r][d + 1];
            q[r][4] = L.c[r];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const double c0 = q[r][2];
            const double xm1 = dpp_shift<DPP_WAVE_SHR1>(lane_value(L.h[r], 1), c0);
            const double xm2 = dpp_shift<DPP_WAVE_SHR1>(lane_value(L.h[r], 0), xm1);
            const double xp1 = dpp_shift<DPP_WAVE_SHL1>(lane_value(L.h[r], 2), c0);
            const double xp2 = dpp_shift<DPP_WAVE_SHL1>(lane_value(L.h[r], 3), xp1);
            const double ym2 = r >= 2 ? q[r >= 2 ? r - 2 : 0][2] : L.ym[r < 2 ? r : 0];
            const double ym1 = r >= 1 ? q[r >= 1 ? r - 1 : 0][2] : L.ym[1];
            const double yp1 = r + 1 < RY ? q[r + 1 < RY ? r + 1 : 0][2] : L.yp[r + 1 - RY >= 0 ? r + 1 - RY : 0];
            const double yp2 = r + 2 < RY ? q[r + 2 < RY ? r + 2 : 0][2] : L.yp[r + 2 - RY >= 0 ? r + 2 - RY : 0];
            const double lap = lap4(B, c0, xm2, xm1, xp1, xp2, ym2, ym1, yp1, yp2, q[r][0], q[r][1], q[r][3], q[r][4]);
            if (w.active_x && w.row_in(r))
                pw_apply<OPK>(B, K, w.point(B, r, k), c0, lap, L.pw[r]);
        }
    };
    const int z0 = P.z0, z1 = P.z1;
    RowPlane<RY, OPK> b0, b1, b2;
    load(z0, b0);
    if (z0 + 1 < z1)
        load(z0 + 1, b1);
    for (int k = z0; k < z1; k += 3) {
        if (k + 2 < z1)
            load(k + 2, b2);
        compute(k, b0);
        if (k + 1 >= z1)
            break;
        if (k + 3 < z1)
            load(k + 3, b0);
        compute(k + 1, b1);
        if (k + 2 >= z1)
            break;
        if (k + 4 < z1)
            load(k + 4, b1);
        compute(k + 2, b2);
    }
}

template <int WX, int WY, int RY, bool WRAP, int OPK>
__global__ __launch_bounds__(WX *WY * 64) void k_rows_single(DevBox B, StageCoef K, int nxcd)
{
    const int item = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const ItemPos P = item_pos(B, item, 64 * WX, RY * WY);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    run_rows<WX, WY, RY, WRAP, OPK>(B, P, K, wave, threadIdx.x % 64);
}

// persistent form over the per-XCD work queue, as k_tiles_batched
template <int WX, int WY, int RY, bool WRAP, int OPK>
__global__ __launch_bounds__(WX *WY * 64) void k_rows_batched(const DevBox *__restrict__ tab, int nbox, ItemQueue Q,
                                                             StageCoef K)
{
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    int q = blockIdx.x % Q.nq, left = Q.nq;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_item = queue_take(Q, q, left);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= Q.nitems)
            break;
        const DevBox B = tab[box_of(tab, nbox, item)];
        const ItemPos P = item_pos(B, item - B.item0, 64 * WX, RY * WY);
        run_rows<WX, WY, RY, WRAP, OPK>(B, P, K, wave, threadIdx.x % 64);
    }
    if (threadIdx.x == 0)
        queue_finish(Q);
}

// ---------------------------------------------------------------------------
// Two RK4 stages fused in one pass (temporal blocking by a stage pair).
//
// Pair 0 runs stages 1 and 2: reads y_n, writes y_3 = y_n + dt/2 k2 and the
// running sum y_n + dt/6 k1 + dt/3 k2.  Pair 1 runs stages 3 and 4: reads
// y_3, y_n and the running sum, writes y_{n+1} (to another buffer: its
// first stage reads y_n around the tile, which neighbouring tiles would
// otherwise overwrite).  A workgroup of TXE x TYE lanes computes the first
// stage of the pair on its whole region and the second stage on the inner
// (TXE-4) x (TYE-4) output tile; the second stage trails the first by two z
// planes.  The first stage's input plane (with a 2-point halo) lives in a
// 4-plane LDS ring, its output in a 3-plane ring, and each lane keeps the
// z-queues of both stage inputs and short delay lines of its pointwise
// values in registers.  One barrier per plane; the next plane's loads are
// issued right after it.  The per-point formulas are the stage kernel's, so
// the two paths give bit-identical results.

__device__ __forceinline__ int mod3(int p)
{
    const int r = p % 3;
    return r < 0 ? r + 3 : r;
}

template <int TXE, int NW, int PAIR, bool HASC2>
__global__ __launch_bounds__(NW * 64) void k_rk4_pair(DevBox B, StageCoef K1, StageCoef K2, int nxcd)
{
    using T = Tile<TXE, NW>;
    constexpr int TYE = T::TY;
    constexpr int TXO = TXE - 4, TYO = TYE - 4;
    constexpr int P1 = T::LY * T::LX; // ring-1 plane: first-stage input with halo
    constexpr int P2 = TXE * TYE;     // ring-2 plane: first-stage output
    __shared__ double ring1[4 * P1];
    __shared__ double ring2[3 * P2];
    const int item = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const ItemPos P = item_pos(B, item, TXO, TYO);
    ItemPos Pe = P;
    Pe.x0 -= 2;
    Pe.y0 -= 2;
    const Walker<TXE, NW, true, false> w(B, Pe, threadIdx.x);
    const int lx = threadIdx.x % TXE, ly = threadIdx.x / TXE;
    const bool out = lx >= 2 && lx < TXE - 2 && ly >= 2 && ly < TYE - 2 && w.i < B.n[0] && w.j < B.n[1];
    const int l2 = ly * TXE + lx;
    const double *__restrict__ in = B.in;
    const double *c2 = HASC2 ? B.p[5] : nullptr;

    double qa0 = 0, qa1 = 0, qa2 = 0, qa3 = 0, qa4 = 0; // first-stage input, planes f-4 .. f
    double qb0 = 0, qb1 = 0, qb2 = 0, qb3 = 0, qb4 = 0; // first-stage output u, planes f-6 .. f-2
    double da0 = 0, da1 = 0, da2 = 0;                   // pair 0: rho_n   pair 1: rho_4
    double db0 = 0, db1 = 0, db2 = 0;                   // pair 0: rho_2   pair 1: acc_u after stage 3
    double dd0 = 0, dd1 = 0, dd2 = 0;                   //                 pair 1: acc_rho after stage 3
    double dc0 = 1, dc1 = 1, dc2 = 1;                   // c^2
    // loads one plane ahead: the input column and halo of plane f, and the
    // first stage's pointwise streams at plane f - 2
    const bool acc_lane = PAIR == 1 && out;
    auto load_pw = [&](int p, double *v) {
        const int64_t e = w.col + w.zoff(p);
        if (HASC2)
            v[0] = ldp(c2 + e);
        v[1] = ldp(B.p[0] + e); // pair 0: rho_n   pair 1: rho_3
        if (PAIR == 1) {
            v[2] = ldp(B.p[1] + e); // u_n
            v[3] = ldp(B.p[2] + e); // rho_n
            if (acc_lane && p >= P.z0 && p < P.z1) {
                v[4] = ldp(B.p[3] + e); // acc_u
                v[5] = ldp(B.p[4] + e); // acc_rho
            }
        }
    };
    double nown, nhv[T::HS], npw[6] = {1, 0, 0, 0, 0, 0}, pw[6] = {1, 0, 0, 0, 0, 0};
    {
        const int f = P.z0 - 4;
        const int64_t zo = w.zoff(f);
        nown = in[w.col + zo];
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0)
                nhv[s] = in[w.hcol[s] + zo];
    }
    for (int f = P.z0 - 4; f <= P.z1 + 3; ++f) {
        qa0 = qa1;
        qa1 = qa2;
        qa2 = qa3;
        qa3 = qa4;
        qa4 = nown;
        double *R1 = ring1 + (f & 3) * P1;
        R1[w.lc] = qa4;
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0)
                R1[w.hl[s]] = nhv[s];
#pragma unroll
        for (int v = 0; v < 6; ++v)
            pw[v] = npw[v];
        lds_barrier();
        const int p1 = f - 2;
        if (f + 1 <= P.z1 + 3) {
            const int64_t zo = w.zoff(f + 1);
            nown = in[w.col + zo];
#pragma unroll
            for (int s = 0; s < T::HS; ++s)
                if (w.hl[s] >= 0)
                    nhv[s] = in[w.hcol[s] + zo];
            if (p1 + 1 >= P.z0 - 2)
                load_pw(p1 + 1, npw);
        }
        if (p1 >= P.z0 - 2) {
            // first stage of the pair at plane p1, on the whole region
            const double *L = ring1 + (p1 & 3) * P1;
            const int lc = w.lc;
            const double lap = lap4(B, qa2, L[lc - 2], L[lc - 1], L[lc + 1], L[lc + 2], L[lc - 2 * T::LX],
                                    L[lc - T::LX], L[lc + T::LX], L[lc + 2 * T::LX], qa0, qa1, qa3, qa4);
            const double cc = pw[0];
            const double kr = HASC2 ? cc * lap : lap;
            double next_u, next_r;
            if (PAIR == 0) { // stage 1: y_2 = y_n + dt/2 k1
                const double un = qa2, rn = pw[1];
                next_u = fma(K1.a, rn, un);
                next_r = fma(K1.a, kr, rn);
                db0 = next_r;
                da0 = rn;
            } else { // stage 3: y_4 = y_n + dt k3; acc += dt/3 k3
                const double ku = pw[1], un = pw[2], rn = pw[3];
                next_u = fma(K1.a, ku, un);
                next_r = fma(K1.a, kr, rn);
                da0 = next_r;
                if (acc_lane && p1 >= P.z0 && p1 < P.z1) {
                    db0 = fma(K1.b, ku, pw[4]);
                    dd0 = fma(K1.b, kr, pw[5]);
                }
            }
            if (HASC2)
                dc0 = cc;
            ring2[mod3(p1) * P2 + l2] = next_u;
            qb0 = qb1;
            qb1 = qb2;
            qb2 = qb3;
            qb3 = qb4;
            qb4 = next_u;
        }
        const int p2 = f - 4;
        if (out && p2 >= P.z0 && p2 < P.z1) {
            // second stage of the pair at plane p2 = p1 - 2, on the output tile
            const double *L = ring2 + mod3(p2) * P2;
            const double lap = lap4(B, qb2, L[l2 - 2], L[l2 - 1], L[l2 + 1], L[l2 + 2], L[l2 - 2 * TXE],
                                    L[l2 - TXE], L[l2 + TXE], L[l2 + 2 * TXE], qb0, qb1, qb3, qb4);
            const double kr = HASC2 ? dc2 * lap : lap;
            const int64_t c = w.point(B, p2);
            if (PAIR == 0) { // stage 2: y_3 = y_n + dt/2 k2; acc = y_n + (y_2 - y_n)/3 + dt/3 k2
                const double un = qa0, rn = da2, u2 = qb2, r2 = db2;
                st(B.q[0] + c, fma(K2.a, r2, un));
                st(B.q[1] + c, fma(K2.a, kr, rn));
                st(B.q[2] + c, fma(K2.b, r2, fma(1.0 / 3.0, u2 - un, un)));
                st(B.q[3] + c, fma(K2.b, kr, fma(1.0 / 3.0, r2 - rn, rn)));
            } else { // stage 4: y_{n+1} = acc + dt/6 k4
                st(B.q[0] + c, fma(K2.b, da2, db2));
                st(B.q[1] + c, fma(K2.b, kr, dd2));
            }
        }
        if (p1 >= P.z0 - 2) {
            da2 = da1;
            da1 = da0;
            db2 = db1;
            db1 = db0;
            dd2 = dd1;
            dd1 = dd0;
            if (HASC2) {
                dc2 = dc1;
                dc1 = dc0;
            }
        }
    }
}


// ---------------------------------------------------------------------------
// One whole RK4 step in one pass: the stage pairs carried one level further.
// Stage 3's stencil input u_3 = u_n + dt/2 rho_2 depends on k_1 = c^2 L u_n
// at the point, and stage 4's u_4 = u_n + dt rho_3 on k_2 = c^2 L u_2, so a
// step reaches radius 4 on u_n and rho_n.  A workgroup of TXE x TYE lanes
// covers an output tile widened by 2 on each side (the traversal of
// k_rk4_pair):
//   phase A, every lane, plane p1: L u_n and L u_2 (u_2 = u_n + dt/2 rho_n
//     formed at every tap), then the pointwise rho_2, u_3, rho_3, u_4 and
//     the running sums acc_u (through stage 3) and acc_rho (through stage
//     2); u_3 and u_4 go to the LDS ring and the column's register queues;
//   phase B, the inner (TXE-4) x (TYE-4) lanes, plane p1 - 2: L u_3 and
//     L u_4, rho_4 = rho_n + dt k_3, acc_rho += dt/3 k_3, and
//     y_{n+1} = acc + dt/6 k_4.
// Every intermediate is the fma the per-stage kernels store, so results are
// bit for bit theirs.  Per output point the pass reads u_n, rho_n and c^2
// and writes u_{n+1}, rho_{n+1}, to other buffers than u_n and rho_n, which
// neighbouring tiles still read.  With Y3 it also writes the third stage
// state y_3 = (u_3, rho_3) of phase A's plane on the output tile (B.q[2],
// B.q[3]), which the backward step reads.

// The rings hold each point's two fields side by side, (u_n, u_2) and
// (u_3, u_4), so that one 16-byte LDS access moves a tap of both: 16-byte
// LDS reads deliver about 1.5 times the bytes per clock of 8-byte ones.
template <int TXE, int NW>
struct Step4Lds {
    static constexpr int P1 = Tile<TXE, NW>::LY * Tile<TXE, NW>::LX; // (u_n, u_2) with halo
    static constexpr int P2 = TXE * Tile<TXE, NW>::TY;                // (u_3, u_4)
    static constexpr int SIZE = 4 * 2 * P1 + 4 * 2 * P2;              // doubles
};

// stage coefficients of a whole step: a_1, a_2, b_2, a_3, b_3, b_4 of StageCoef
struct Step4Coef {
    double a1, a2, b2, a3, b3, b4;
};

// one tile and z range of a whole step (C2PD2: with c^2, load two planes
// ahead too where the workgroup has 1024 lanes).  WRAP: the box is its own
// periodic neighbour (stencil neighbours at wrapped indices); otherwise
// ghost addressing, for the boxes of a level whose ghost zones of width 4
// hold the neighbours' values (a step reaches 4 points beyond the output
// tile: indices -4 .. n + 3, read clamped to n + 3 by lanes past the box)
template <int TXE, int NW, bool HASC2, bool Y3, bool C2PD2 = false, bool WRAP = true>
__device__ __forceinline__ void run_step4(const DevBox &B, const ItemPos &P, const Step4Coef &K, double *lds)
{
    using T = Tile<TXE, NW>;
    using S = Step4Lds<TXE, NW>;
    constexpr int TYE = T::TY;
    constexpr int P1 = S::P1, P2 = S::P2;
    dvec2 *const ring1 = (dvec2 *)lds;      // 4 slots of (u_n, u_2) pairs
    dvec2 *const ring2 = ring1 + 4 * P1;    // 4 slots of (u_3, u_4) pairs
    ItemPos Pe = P;
    Pe.x0 -= 2;
    Pe.y0 -= 2;
    const int tl = tile_thread<TXE, NW>(threadIdx.x);
    const Walker<TXE, NW, true, false> w(B, Pe, tl);
    const int lx = tl % TXE, ly = tl / TXE;
    const bool out = lx >= 2 && lx < TXE - 2 && ly >= 2 && ly < TYE - 2 && w.i < B.n[0] && w.j < B.n[1];
    const int l2 = ly * TXE + lx;
    // byte offset of the lane's output point within a z plane
    const unsigned xy = (unsigned)(w.i + w.g + (int64_t)(w.j + w.g) * B.sy) * 8u;
    const double *__restrict__ uf = B.in;
    const double *__restrict__ rf = B.p[0];
    const double *c2 = HASC2 ? B.p[5] : nullptr;
    // bytes of one z plane of the outputs, the range of the buffer stores
    // (below 2^31, checked at launch)
    const unsigned plane_bytes = (unsigned)(B.sz * 8);
    const double a1 = K.a1, a2 = K.a2, b2 = K.b2, a3 = K.a3, b3 = K.b3, b4 = K.b4;

    // Column queues, five planes each: f-4 .. f of u_n, rho_n and c^2 (u_2 at
    // a plane is fma(a1, rho_n, u_n), formed where needed), f-6 .. f-2 of
    // u_3 and u_4.  Step t writes the newest plane of a queue to slot t mod 5,
    // so the planes rotate through fixed registers: the loop below is
    // unrolled ten-fold (five queue slots times the two fetch buffers) and
    // every slot index is a compile-time constant, with no register copies.
    // Phase A's running sums are delayed to phase B through du0..du2 and
    // dr0..dr2.
    double qa[5] = {0, 0, 0, 0, 0}, qr[5] = {0, 0, 0, 0, 0}, qc[5] = {1, 1, 1, 1, 1};
    double qb[5] = {0, 0, 0, 0, 0}, qd[5] = {0, 0, 0, 0, 0};
    double du0 = 0, du1 = 0, du2 = 0; // acc_u after stage 3
    double dr0 = 0, dr1 = 0, dr2 = 0; // acc_rho after stage 2
    double y3u = 0, y3r = 0;          // u_3, rho_3 of phase A's plane (Y3)

    // Plane step t = 0 .. nt-1 takes plane f = z0 - 4 + t into ring 1 (slot
    // t mod 4), computes phase A at f - 2 from the plane taken at step t - 2
    // (from t = 4 on) into ring 2 (slot t mod 4), and phase B at f - 4 from
    // the ring-2 plane written at step t - 2 (for t - 8 in [0, tz)).  The
    // plane fetched next is tracked as a wrapped index (no division per
    // plane).
    const int nt = P.z1 - P.z0 + 8, tz = P.z1 - P.z0;
    const int nz = B.n[2];
    // index of the plane fetched next (wrapped, or -4 .. nz + 3 with ghosts)
    int kz = WRAP ? readable(P.z0 - 4, nz, true, false) : P.z0 - 4;
    // The loads of a plane are issued PD steps before it is taken: PD = 2,
    // from two buffers used by alternate steps, so that no register a load
    // is still filling is ever copied (a copy would wait for the load).
    // With the c^2 queue on 512-lane workgroups the second buffer would
    // cost a wavefront per SIMD, so those load one plane ahead; 1024-lane
    // workgroups are held to 128 VGPRs anyway, and the plain whole-step
    // kernel gains from it (C2PD2; the batched and y_3 forms would spill).
    // Plane loads go through buffer resources: one 32-bit lane offset serves
    // every plane.
    constexpr int PD = HASC2 && !(C2PD2 && NW * 64 == 1024) ? 1 : 2;
    struct Fetched {
        double u, r, c, hu[T::HS], hr[T::HS];
    };
    Fetched F0, F1;
    F0.c = F1.c = 1.0;
    // byte offsets within a plane of the lane's column and halo slots
    unsigned col8, h8[T::HS];
    if constexpr (WRAP) {
        col8 = (unsigned)w.col * 8u;
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            h8[s] = (unsigned)w.hcol[s] * 8u;
    } else {
        auto gi = [](int p, int n) { return p < n + 3 ? p : n + 3; };
        const int nx = B.n[0], ny = B.n[1];
        col8 = (unsigned)((gi(Pe.x0 + lx, nx) + w.g) + (int64_t)(gi(Pe.y0 + ly, ny) + w.g) * B.sy) * 8u;
#pragma unroll
        for (int s = 0; s < T::HS; ++s) {
            const int h = tl + s * T::NTL;
            int lrow = 0, lcol = 0, dx = 0, dy = 0;
            if (h < T::NH)
                halo_slot<TXE, NW>(h, lrow, lcol, dx, dy);
            h8[s] = (unsigned)((gi(Pe.x0 + dx, nx) + w.g) + (int64_t)(gi(Pe.y0 + dy, ny) + w.g) * B.sy) * 8u;
        }
    }
    auto fetch = [&](Fetched &F) {
        const int64_t zo = (int64_t)(kz + w.g) * w.sz;
        const double *pu = uf + zo, *pr = rf + zo;
        F.u = ld_plane<0>(pu, plane_bytes, col8);
        F.r = ld_plane<0>(pr, plane_bytes, col8);
        if (HASC2) // per box in a batched launch: no c^2 reads as 1, an exact factor
            F.c = c2 ? ld_plane<2>(c2 + zo, plane_bytes, col8) : 1.0;
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0) { // whole wavefronts without halo points skip these
                F.hu[s] = ld_plane<0>(pu, plane_bytes, h8[s]);
                F.hr[s] = ld_plane<0>(pr, plane_bytes, h8[s]);
            }
        kz = WRAP && kz + 1 == nz ? 0 : kz + 1;
    };
    // step t = t0 + J with t0 a multiple of 10: queue slot of plane f - 4 + m
    // (m = 0 .. 4) is (J + 1 + m) mod 5
    auto step = [&](auto Jc, const int t) {
        constexpr int J = decltype(Jc)::value;
        constexpr int S0 = (J + 1) % 5, S1 = (J + 2) % 5, S2 = (J + 3) % 5, S3 = (J + 4) % 5, S4 = J % 5;
        Fetched &F = PD == 2 && (J & 1) ? F1 : F0;
        const int k = t & 3;
        const double nu = F.u, nr = F.r;
        qa[S4] = nu;
        qr[S4] = nr;
        if (HASC2)
            qc[S4] = F.c;
        dvec2 *R1 = ring1 + k * P1;
        R1[w.lc] = dvec2{nu, fma(a1, nr, nu)};
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0)
                R1[w.hl[s]] = dvec2{F.hu[s], fma(a1, F.hr[s], F.hu[s])};
        // the loads of the plane taken PD steps on fly across the barrier
        // (this buffer's registers were consumed just above), as do the
        // stores of the last plane
        if (t + PD < nt)
            fetch(F);
        lds_barrier();
        if (t >= 4) {
            // phase A (stages 1 and 2) at plane f - 2, every lane
            // (x taps, then y taps: four 16-byte taps in registers at a time)
            const dvec2 *L = ring1 + ((k + 2) & 3) * P1; // taken at step t - 2
            const int lc = w.lc;
            double sxa, sxv, sya, syv;
            {
                const dvec2 m2 = L[lc - 2], m1 = L[lc - 1], p1 = L[lc + 1], p2 = L[lc + 2];
                sxa = axis4(m2.x, m1.x, p1.x, p2.x);
                sxv = axis4(m2.y, m1.y, p1.y, p2.y);
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                const dvec2 m2 = L[lc - 2 * T::LX], m1 = L[lc - T::LX], p1 = L[lc + T::LX], p2 = L[lc + 2 * T::LX];
                sya = axis4(m2.x, m1.x, p1.x, p2.x);
                syv = axis4(m2.y, m1.y, p1.y, p2.y);
            }
            const double la = lap4s(B, qa[S2], sxa, sya, axis4(qa[S0], qa[S1], qa[S3], qa[S4]));
            const double un = qa[S2], rn = qr[S2], u2 = fma(a1, qr[S2], qa[S2]);
            const double lv = lap4s(B, u2, sxv, syv,
                                    axis4(fma(a1, qr[S0], qa[S0]), fma(a1, qr[S1], qa[S1]),
                                          fma(a1, qr[S3], qa[S3]), fma(a1, qr[S4], qa[S4])));
            const double kr1 = HASC2 ? qc[S2] * la : la;
            const double kr2 = HASC2 ? qc[S2] * lv : lv;
            const double r2 = fma(a1, kr1, rn);
            const double u3 = fma(a2, r2, un);
            const double r3 = fma(a2, kr2, rn);
            const double u4 = fma(a3, r3, un);
            if (Y3) {
                y3u = u3;
                y3r = r3;
            }
            du0 = fma(b3, r3, fma(b2, r2, fma(1.0 / 3.0, u2 - un, un)));
            dr0 = fma(b2, kr2, fma(1.0 / 3.0, r2 - rn, rn));
            ring2[k * P2 + l2] = dvec2{u3, u4};
            qb[S4] = u3;
            qd[S4] = u4;
        }
        const bool wr = out && t >= 8 && t - 8 < tz;
        double yu = 0.0, yr = 0.0;
        if (wr) {
            // phase B (stages 3 and 4) at plane f - 4, the output tile; u_3
            // and u_4 of planes f - 6 .. f - 2 sit in the slots of steps
            // t - 4 .. t, rho_n and c^2 of plane f - 4 in slot S0
            const dvec2 *L = ring2 + ((k + 2) & 3) * P2; // written at step t - 2
            double sx3, sx4, sy3, sy4;
            {
                const dvec2 m2 = L[l2 - 2], m1 = L[l2 - 1], p1 = L[l2 + 1], p2 = L[l2 + 2];
                sx3 = axis4(m2.x, m1.x, p1.x, p2.x);
                sx4 = axis4(m2.y, m1.y, p1.y, p2.y);
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                const dvec2 m2 = L[l2 - 2 * TXE], m1 = L[l2 - TXE], p1 = L[l2 + TXE], p2 = L[l2 + 2 * TXE];
                sy3 = axis4(m2.x, m1.x, p1.x, p2.x);
                sy4 = axis4(m2.y, m1.y, p1.y, p2.y);
            }
            const double l3 = lap4s(B, qb[S2], sx3, sy3, axis4(qb[S0], qb[S1], qb[S3], qb[S4]));
            const double l4 = lap4s(B, qd[S2], sx4, sy4, axis4(qd[S0], qd[S1], qd[S3], qd[S4]));
            const double kr3 = HASC2 ? qc[S0] * l3 : l3;
            const double kr4 = HASC2 ? qc[S0] * l4 : l4;
            const double r4 = fma(a3, kr3, qr[S0]);
            yu = fma(b4, r4, du2);
            yr = fma(b4, kr4, fma(b3, kr3, dr2));
        }
        // Two stores on every step and lane (dropped where there is no
        // output point), so the count of memory operations after the next
        // plane's loads is fixed and the wait for those loads does not
        // drain these stores.
        const int p2 = P.z0 + t - 8, pc = p2 < 0 ? 0 : p2 < nz ? p2 : nz - 1;
        const int64_t pz = (int64_t)(pc + w.g) * w.sz;
        const unsigned off = wr ? xy : NO_STORE;
        st_or_drop(B.q[0] + pz, plane_bytes, off, yu);
        st_or_drop(B.q[1] + pz, plane_bytes, off, yr);
        if (Y3) { // phase A's plane f - 2 = z0 + t - 6, when it is an output plane
            const int p3 = P.z0 + t - 6, pc3 = p3 < 0 ? 0 : p3 < nz ? p3 : nz - 1;
            const unsigned off3 = out && t >= 6 && t - 6 < tz ? xy : NO_STORE;
            const int64_t pz3 = (int64_t)(pc3 + w.g) * w.sz;
            st_or_drop(B.q[2] + pz3, plane_bytes, off3, y3u);
            st_or_drop(B.q[3] + pz3, plane_bytes, off3, y3r);
        }
        if (t >= 4) {
            du2 = du1;
            du1 = du0;
            dr2 = dr1;
            dr1 = dr0;
        }
    };
    fetch(F0);
    if (PD == 2 && nt > 1)
        fetch(F1);
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using I6 = std::integral_constant<int, 6>;
    using I7 = std::integral_constant<int, 7>;
    using I8 = std::integral_constant<int, 8>;
    using I9 = std::integral_constant<int, 9>;
    for (int t = 0; t < nt; t += 10) {
        step(I0{}, t);
        if (t + 1 < nt) step(I1{}, t + 1);
        if (t + 2 < nt) step(I2{}, t + 2);
        if (t + 3 < nt) step(I3{}, t + 3);
        if (t + 4 < nt) step(I4{}, t + 4);
        if (t + 5 < nt) step(I5{}, t + 5);
        if (t + 6 < nt) step(I6{}, t + 6);
        if (t + 7 < nt) step(I7{}, t + 7);
        if (t + 8 < nt) step(I8{}, t + 8);
        if (t + 9 < nt) step(I9{}, t + 9);
    }
}

// persistent form over the per-XCD work queue of a table of periodic boxes
// (items: box, tile, z chunk of B.tz planes), as k_tiles_batched
template <int TXE, int NW, bool HASC2, bool WRAP = true>
__global__ __launch_bounds__(NW * 64, 4) void k_rk4_step4_batched(const DevBox *__restrict__ tab, int nbox,
                                                               ItemQueue Q, Step4Coef K)
{
    __shared__ __attribute__((aligned(16))) double lds[Step4Lds<TXE, NW>::SIZE];
    __shared__ int s_item;
    constexpr int TYE = Tile<TXE, NW>::TY;
    int q = blockIdx.x % Q.nq, left = Q.nq;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_item = queue_take(Q, q, left);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= Q.nitems)
            break;
        const DevBox B = tab[box_of(tab, nbox, item)];
        run_step4<TXE, NW, HASC2, false, false, WRAP>(B, item_pos(B, item - B.item0, TXE - 4, TYE - 4), K, lds);
    }
    if (threadIdx.x == 0)
        queue_finish(Q);
}

// Workgroup g (placed so that each XCD holds a contiguous range of g) runs
// work item g -- tiles in order within z chunks of B.tz planes, so that the
// workgroups of one XCD march a compact patch of tiles through the same
// planes and share their halo lines in its L2 -- or, with run > 0, planes
// [g * run, (g + 1) * run) of the box's tile-plane sequence.
template <int TXE, int NW, bool HASC2, bool Y3, bool WRAP = true>
__device__ __forceinline__ void step4_grid(const DevBox &B, const Step4Coef &K, int run, int nxcd, double *lds)
{
    constexpr int TYE = Tile<TXE, NW>::TY;
    const int g = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    if (run == 0) {
        run_step4<TXE, NW, HASC2, Y3, !Y3, WRAP>(B, item_pos(B, g, TXE - 4, TYE - 4), K, lds);
        return;
    }
    const int64_t total = (int64_t)B.tiles[0] * B.tiles[1] * B.n[2];
    int64_t s = (int64_t)g * run;
    const int64_t e = s + run < total ? s + run : total;
    ItemPos P;
    while (run_piece(B, TXE - 4, TYE - 4, s, e, P)) {
        run_step4<TXE, NW, HASC2, Y3, !Y3, WRAP>(B, P, K, lds);
        __syncthreads(); // the next piece rewrites the LDS rings
    }
}

// (the launch bound asks for four wavefronts per SIMD: two 512-lane or one
// 1024-lane workgroup per CU, as many as the LDS rings allow)
template <int TXE, int NW, bool HASC2, bool WRAP = true>
__global__ __launch_bounds__(NW * 64, 4) void k_rk4_step4(DevBox B, Step4Coef K, int run, int nxcd)
{
    __shared__ __attribute__((aligned(16))) double lds[Step4Lds<TXE, NW>::SIZE];
    step4_grid<TXE, NW, HASC2, false, WRAP>(B, K, run, nxcd, lds);
}

// the same step, also storing the third stage state (u_3, rho_3)
template <int TXE, int NW, bool HASC2>
__global__ __launch_bounds__(NW * 64, 4) void k_rk4_step4_y3(DevBox B, Step4Coef K, int run, int nxcd)
{
    __shared__ __attribute__((aligned(16))) double lds[Step4Lds<TXE, NW>::SIZE];
    step4_grid<TXE, NW, HASC2, true>(B, K, run, nxcd, lds);
}


// ---------------------------------------------------------------------------
// Two RK4 stages in one pass without a widened tile.  In the first-order
// wave equation the next stage's u is pointwise in the current state
// (u_{s+1} = u_n + a_s rho_s), so the second stage's stencil input at each
// tap is formed from taps of fields the pass already reads:
//   pair 0 (stages 1, 2): taps of u_n give L u_n; u_2 = u_n + dt/2 rho_n at
//     every tap (from taps of u_n and rho_n) gives L u_2;
//   pair 1 (stages 3, 4): taps of u_3 give L u_3; u_4 = u_n + dt rho_3 at
//     every tap (from taps of rho_3 and u_n) gives L u_4.
// Each tap value of u_{s+1} is the fma the stage kernel stores there, so
// results are bit for bit those of the per-stage kernels.  The traversal is
// the tile traversal's (radius-2 halo; periodic addressing, or ghost
// addressing on a level whose ghost zones are exchanged) over NF stencil
// fields: each field's column's five z values sit in registers, and the
// current plane of the two stencil inputs, (u_n, u_2) or (u_3, u_4), in LDS
// as 16-byte pairs (double buffered), each pair formed once by the lane that
// loaded the point.  Reads and writes per point: pair 0
// reads u_n, rho_n and writes u_3, rho_3, acc_u, acc_rho; pair 1 reads u_3,
// rho_3, u_n, rho_n, acc_u, acc_rho and writes u_{n+1}, rho_{n+1} (to
// another buffer than u_n, which neighbouring tiles still read).

template <int TX, int NW, int PAIR>
struct Pair2Lds {
    static constexpr int NF = PAIR == 0 ? 2 : 3; // fields loaded per tap
    static constexpr int PLANE = Tile<TX, NW>::LY * Tile<TX, NW>::LX;
    static constexpr int SIZE = 2 * 2 * PLANE; // doubles: two planes of pairs
};

// one work item of a stage pair; c^2 (B.p[5]) is optional per box: without
// it the stencil is multiplied by 1.0, which is exact
template <int TX, int NW, int PAIR, bool WRAP>
__device__ __forceinline__ void run_pair2(const DevBox &B, const ItemPos &P, const StageCoef &K1, const StageCoef &K2,
                                          double *lds)
{
    using T = Tile<TX, NW>;
    constexpr int NF = Pair2Lds<TX, NW, PAIR>::NF;
    constexpr int PLANE = Pair2Lds<TX, NW, PAIR>::PLANE;
    const Walker<TX, NW, WRAP> w(B, P, threadIdx.x);
    const bool hasc2 = B.p[5] != nullptr;
    const int lc = w.lc;
    // stencil fields: pair 0: u_n, rho_n; pair 1: u_3, rho_3, u_n
    const double *F[3] = {B.in, B.p[0], B.p[1]};

    // The loads of plane k (halo, pointwise streams) and of the column's
    // plane k+2 are issued two steps before step k, into one of two buffers
    // used by alternate steps, so no register a load is still filling is
    // copied.
    struct Fetched {
        double q4[NF], hv[NF][T::HS], pw[4];
    };
    auto load_pw = [&](int k, double *v) {
        const int64_t c = w.point(B, k);
        if (hasc2)
            v[0] = ldp(B.p[5] + c);
        if constexpr (PAIR == 1) {
            v[1] = ldp(B.p[2] + c);
            v[2] = ldp(B.p[3] + c);
            v[3] = ldp(B.p[4] + c);
        }
    };
    auto fetch = [&](int k, Fetched &X) {
        const int64_t z2 = w.zoff(k + 2), z0 = w.zoff(k);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            X.q4[f] = F[f][w.col + z2];
#pragma unroll
            for (int s = 0; s < T::HS; ++s)
                if (w.hl[s] >= 0)
                    X.hv[f][s] = F[f][w.hcol[s] + z0];
        }
        if (w.active)
            load_pw(k, X.pw);
    };
    // the column's planes k-2 .. k+2 at step k (q[f][4] arrives with the step)
    double q[NF][5];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int d = 1; d < 5; ++d)
            q[f][d] = F[f][w.col + w.zoff(P.z0 - 3 + d)];
    Fetched F0, F1;
#pragma unroll
    for (int v = 0; v < 4; ++v)
        F0.pw[v] = F1.pw[v] = v == 0 ? 1.0 : 0.0;
    // the second stencil input at a point: u_2 = u_n + a rho_n (pair 0),
    // u_4 = u_n + a rho_3 (pair 1), from that point's loaded fields
    constexpr int FU = PAIR == 0 ? 0 : 2; // field of u_n
    const double a1 = K1.a;
    auto second = [&](const double *v) { return fma(a1, v[1], v[FU]); };
    auto step = [&](const int k, Fetched &X) {
        dvec2 *L = (dvec2 *)lds + ((k - P.z0) & 1) * PLANE;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            q[f][0] = q[f][1];
            q[f][1] = q[f][2];
            q[f][2] = q[f][3];
            q[f][3] = q[f][4];
            q[f][4] = X.q4[f];
        }
        {
            const double v[3] = {q[0][2], q[1][2], q[NF - 1][2]};
            L[lc] = dvec2{v[0], second(v)};
        }
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0) {
                const double v[3] = {X.hv[0][s], X.hv[1][s], X.hv[NF - 1][s]};
                L[w.hl[s]] = dvec2{v[0], second(v)};
            }
        double pwc[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            pwc[v] = X.pw[v];
        if (k + 2 < P.z1)
            fetch(k + 2, X);
        lds_barrier();
        if (w.active) {
            const double a2 = K2.a;
            const double c2 = pwc[0];
            // x and y tap sums of both stencil inputs (four 16-byte taps in
            // registers at a time)
            double sx0, sx1, sy0, sy1;
            {
                const dvec2 m2 = L[lc - 2], m1 = L[lc - 1], p1 = L[lc + 1], p2 = L[lc + 2];
                sx0 = axis4(m2.x, m1.x, p1.x, p2.x);
                sx1 = axis4(m2.y, m1.y, p1.y, p2.y);
            }
            __builtin_amdgcn_sched_barrier(0);
            {
                const dvec2 m2 = L[lc - 2 * T::LX], m1 = L[lc - T::LX], p1 = L[lc + T::LX], p2 = L[lc + 2 * T::LX];
                sy0 = axis4(m2.x, m1.x, p1.x, p2.x);
                sy1 = axis4(m2.y, m1.y, p1.y, p2.y);
            }
            if constexpr (PAIR == 0) {
                // stage 1: L u_n
                const double un = q[0][2], rn = q[1][2];
                const double lap1 = lap4s(B, un, sx0, sy0, axis4(q[0][0], q[0][1], q[0][3], q[0][4]));
                const double kr1 = c2 * lap1;
                const double u2 = fma(a1, rn, un);
                const double r2 = fma(a1, kr1, rn);
                // stage 2: L u_2 with u_2 = u_n + a1 rho_n at every tap
                auto tz = [&](int d) { return fma(a1, q[1][d], q[0][d]); };
                const double lap2 = lap4s(B, u2, sx1, sy1, axis4(tz(0), tz(1), tz(3), tz(4)));
                const double kr2 = c2 * lap2;
                const int64_t c = w.point(B, k);
                st(B.q[0] + c, fma(a2, r2, un));
                st(B.q[1] + c, fma(a2, kr2, rn));
                if (B.q[2]) { // the running sums (not needed when only u_3, rho_3 are wanted)
                    st(B.q[2] + c, fma(K2.b, r2, fma(1.0 / 3.0, u2 - un, un)));
                    st(B.q[3] + c, fma(K2.b, kr2, fma(1.0 / 3.0, r2 - rn, rn)));
                }
            } else {
                // stage 3: L u_3
                const double u3 = q[0][2], r3 = q[1][2], un = q[2][2];
                const double rn = pwc[1], au = pwc[2], ar = pwc[3];
                const double lap3 = lap4s(B, u3, sx0, sy0, axis4(q[0][0], q[0][1], q[0][3], q[0][4]));
                const double kr3 = c2 * lap3;
                const double u4 = fma(a1, r3, un);
                const double r4 = fma(a1, kr3, rn);
                const double au4 = fma(K1.b, r3, au);
                const double ar4 = fma(K1.b, kr3, ar);
                // stage 4: L u_4 with u_4 = u_n + a3 rho_3 at every tap
                auto tz = [&](int d) { return fma(a1, q[1][d], q[2][d]); };
                const double lap4v = lap4s(B, u4, sx1, sy1, axis4(tz(0), tz(1), tz(3), tz(4)));
                const double kr4 = c2 * lap4v;
                const int64_t c = w.point(B, k);
                st(B.q[0] + c, fma(K2.b, r4, au4));
                st(B.q[1] + c, fma(K2.b, kr4, ar4));
            }
        }
    };
    fetch(P.z0, F0);
    if (P.z0 + 1 < P.z1)
        fetch(P.z0 + 1, F1);
    for (int k = P.z0; k < P.z1; k += 2) {
        step(k, F0);
        if (k + 1 < P.z1)
            step(k + 1, F1);
    }
}


template <int TX, int NW, int PAIR, bool WRAP>
__global__ __launch_bounds__(NW * 64, 4) void k_pair2(DevBox B, StageCoef K1, StageCoef K2, int nxcd)
{
    __shared__ __attribute__((aligned(16))) double lds[Pair2Lds<TX, NW, PAIR>::SIZE];
    const int item = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const ItemPos P = item_pos(B, item, TX, Tile<TX, NW>::TY);
    run_pair2<TX, NW, PAIR, WRAP>(B, P, K1, K2, lds);
}

// persistent form over the per-XCD work queue, as k_tiles_batched
template <int TX, int NW, int PAIR, bool WRAP>
__global__ __launch_bounds__(NW * 64, 4) void k_pair2_batched(const DevBox *__restrict__ tab, int nbox, ItemQueue Q,
                                                          StageCoef K1, StageCoef K2)
{
    __shared__ __attribute__((aligned(16))) double lds[Pair2Lds<TX, NW, PAIR>::SIZE];
    __shared__ int s_item;
    int q = blockIdx.x % Q.nq, left = Q.nq;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_item = queue_take(Q, q, left);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= Q.nitems)
            break;
        const DevBox B = tab[box_of(tab, nbox, item)];
        const ItemPos P = item_pos(B, item - B.item0, TX, Tile<TX, NW>::TY);
        run_pair2<TX, NW, PAIR, WRAP>(B, P, K1, K2, lds);
    }
    if (threadIdx.x == 0)
        queue_finish(Q);
}


// ---------------------------------------------------------------------------
// One backward RK4 step in two passes.  The adjoint of F(u, rho) =
// (rho, c^2 L u) is F^T(a, b) = (L(c^2 b), a) (L symmetric under periodic
// addressing).  With kb_s = (ku_s, kr_s) and lambda = (lu, lr) = dJ/dy_{n+1}:
//   ku4 = dt/6 lu, kr4 = dt/6 lr, kr3 = dt/3 lr + dt ku4          (pointwise)
//   ku3 = dt/3 lu + dt L(c^2 kr4),   ku2 = dt/3 lu + dt/2 L(c^2 kr3)
//   kr2 = dt/3 lr + dt/2 ku3,        kr1 = dt/6 lr + dt/2 ku2
//   ku1 = dt/6 lu + dt/2 L(c^2 kr2)
//   dJ/dy_n = (lu + sum_s L(c^2 kr_s), lr + sum_s ku_s)
//   c2bar  += sum_s kr_s L u_s
// Pass A stencils c^2 kr4 and c^2 kr3, formed at every tap from taps of lu,
// lr and c^2, and stores kr2, kr1 and the partial sums; pass B stencils
// c^2 kr2 and c^2 kr1 and writes dJ/dy_n over lambda (pass B reads lambda
// only at the point).  With c2bar, pass A also applies L to u_3 and to
// u_4 = u_n + dt rho_3 (formed per tap; u_3, rho_3 from the forward
// stage-pair kernel) and pass B to u_1 = u_n and u_2 = u_n + dt/2 rho_n.
// The LDS and the z queues hold the transformed values t (NL fields, in
// LDS as 16-byte pairs of fields 0, 1 and 2, 3); the raw values two planes
// ahead are loaded into registers first.
//   pass A:  in lu, p0 lr, p1 u_3, p2 u_n, p3 rho_3, p5 c^2, p6 c2bar;
//            out q0 kr2, q1 kr1, q2 acc_u, q3 acc_rho, q4 c2bar
//   pass B:  in kr2, p0 kr1, p1 u_n, p2 rho_n, p3 acc_u, p4 acc_rho, p5 c^2,
//            p6 c2bar; out q0 lambda_u (read first), q1 lambda_rho, q4 c2bar
// K: a = dt, b = dt/6, a_next = dt/3, b_next = dt/2.

template <int PASS, bool C2BAR>
struct AdjPass {
    static constexpr int NL = C2BAR ? 4 : 2; // transformed stencil fields
    static constexpr int NR = C2BAR ? 6 : 3; // raw fields read per tap
};

template <int PASS, bool C2BAR>
__device__ __forceinline__ void adj_raw(const DevBox &B, int64_t e, double *r)
{
    r[0] = B.in[e];
    r[1] = B.p[0][e];
    r[2] = B.p[5] ? B.p[5][e] : 1.0;
    if constexpr (C2BAR) {
        if constexpr (PASS == 0) {
            r[3] = B.p[1][e]; // u_3
            r[4] = B.p[2][e]; // u_n
            r[5] = B.p[3][e]; // rho_3
        } else {
            r[3] = B.p[1][e]; // u_n
            r[4] = B.p[2][e]; // rho_n
        }
    }
}

// transformed values from the raw ones
template <int PASS, bool C2BAR>
__device__ __forceinline__ void adj_tf(const StageCoef &K, const double *r, double *t)
{
    if constexpr (PASS == 0) {
        const double ku4 = K.b * r[0], kr4 = K.b * r[1];
        const double kr3 = fma(K.a, ku4, K.a_next * r[1]);
        t[0] = r[2] * kr4;
        t[1] = r[2] * kr3;
        if constexpr (C2BAR) {
            t[2] = r[3];
            t[3] = fma(K.a, r[5], r[4]);
        }
    } else {
        t[0] = r[2] * r[0];
        t[1] = r[2] * r[1];
        if constexpr (C2BAR) {
            t[2] = r[3];
            t[3] = fma(K.b_next, r[4], r[3]);
        }
    }
}

template <int TX, int NW, int PASS, bool C2BAR>
__global__ __launch_bounds__(NW * 64) void k_adj2(DevBox B, StageCoef K, int nxcd)
{
    using T = Tile<TX, NW>;
    using A = AdjPass<PASS, C2BAR>;
    constexpr int NL = A::NL, NR = A::NR;
    constexpr int PLANE = T::LY * T::LX;
    constexpr int NP = NL / 2; // LDS planes of field pairs
    __shared__ __attribute__((aligned(16))) double lds[2 * NL * PLANE];
    const int item = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const ItemPos P = item_pos(B, item, TX, T::TY);
    const Walker<TX, NW, true> w(B, P, threadIdx.x);
    const int lc = w.lc;

    // z queues of the transformed fields (planes k-2 .. k+2) and of the two
    // raw values needed at the point (planes k .. k+2)
    double q[NL][5], rq[2][3];
    double nr[NR], nh[T::HS][NR]; // raw loads of the next plane: own column (plane k+3), halo (plane k+1)
    double hv[NL][T::HS];
    {
        double r[NR], t[NL];
        for (int d = 0; d < 5; ++d) {
            adj_raw<PASS, C2BAR>(B, w.col + w.zoff(P.z0 - 2 + d), r);
            adj_tf<PASS, C2BAR>(K, r, t);
#pragma unroll
            for (int f = 0; f < NL; ++f)
                q[f][d] = t[f];
            if (d >= 2) {
                rq[0][d - 2] = r[0];
                rq[1][d - 2] = r[1];
            }
        }
        const int64_t zo = w.zoff(P.z0);
#pragma unroll
        for (int s = 0; s < T::HS; ++s)
            if (w.hl[s] >= 0) {
                adj_raw<PASS, C2BAR>(B, w.hcol[s] + zo, r);
                adj_tf<PASS, C2BAR>(K, r, t);
#pragma unroll
                for (int f = 0; f < NL; ++f)
                    hv[f][s] = t[f];
            }
    }
    int buf = 0;
    for (int k = P.z0; k < P.z1; ++k) {
        dvec2 *L = (dvec2 *)lds + buf * NP * PLANE;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            L[p * PLANE + lc] = dvec2{q[2 * p][2], q[2 * p + 1][2]};
#pragma unroll
            for (int s = 0; s < T::HS; ++s)
                if (w.hl[s] >= 0)
                    L[p * PLANE + w.hl[s]] = dvec2{hv[2 * p][s], hv[2 * p + 1][s]};
        }
        lds_barrier();
        const bool more = k + 1 < P.z1;
        if (more) {
            adj_raw<PASS, C2BAR>(B, w.col + w.zoff(k + 3), nr);
            const int64_t z1 = w.zoff(k + 1);
#pragma unroll
            for (int s = 0; s < T::HS; ++s)
                if (w.hl[s] >= 0)
                    adj_raw<PASS, C2BAR>(B, w.hcol[s] + z1, nh[s]);
        }
        if (w.active) {
            const int64_t c = w.point(B, k);
            // L of fields 2p and 2p+1 (x taps, then y taps: four 16-byte
            // taps in registers at a time)
            auto lapp = [&](int p, double &la, double &lb) {
                const dvec2 *Lp = L + p * PLANE;
                double sxa, sxb, sya, syb;
                {
                    const dvec2 m2 = Lp[lc - 2], m1 = Lp[lc - 1], p1 = Lp[lc + 1], p2 = Lp[lc + 2];
                    sxa = axis4(m2.x, m1.x, p1.x, p2.x);
                    sxb = axis4(m2.y, m1.y, p1.y, p2.y);
                }
                __builtin_amdgcn_sched_barrier(0);
                {
                    const dvec2 m2 = Lp[lc - 2 * T::LX], m1 = Lp[lc - T::LX], p1 = Lp[lc + T::LX],
                                p2 = Lp[lc + 2 * T::LX];
                    sya = axis4(m2.x, m1.x, p1.x, p2.x);
                    syb = axis4(m2.y, m1.y, p1.y, p2.y);
                }
                const int fa = 2 * p, fb = 2 * p + 1;
                la = lap4s(B, q[fa][2], sxa, sya, axis4(q[fa][0], q[fa][1], q[fa][3], q[fa][4]));
                lb = lap4s(B, q[fb][2], sxb, syb, axis4(q[fb][0], q[fb][1], q[fb][3], q[fb][4]));
            };
            const double dt = K.a, d6 = K.b, d3 = K.a_next, d2 = K.b_next;
            if constexpr (PASS == 0) {
                const double lu = rq[0][0], lr = rq[1][0];
                double Y4, Y3;
                lapp(0, Y4, Y3);
                const double ku4 = d6 * lu, kr4 = d6 * lr;
                const double kr3 = fma(dt, ku4, d3 * lr);
                const double ku3 = fma(dt, Y4, d3 * lu);
                const double ku2 = fma(d2, Y3, d3 * lu);
                const double kr2 = fma(d2, ku3, d3 * lr);
                const double kr1 = fma(d2, ku2, d6 * lr);
                st(B.q[0] + c, kr2);
                st(B.q[1] + c, kr1);
                st(B.q[2] + c, lu + Y4 + Y3);
                st(B.q[3] + c, lr + ku4 + ku3 + ku2);
                if constexpr (C2BAR) {
                    double Lu3, Lu4;
                    lapp(1, Lu3, Lu4);
                    st(B.q[4] + c, fma(kr4, Lu4, fma(kr3, Lu3, ldp(B.p[6] + c))));
                }
            } else {
                const double kr2 = rq[0][0], kr1 = rq[1][0];
                double Y2, Y1;
                lapp(0, Y2, Y1);
                const double lu = ldp(B.q[0] + c);
                const double ku1 = fma(d2, Y2, d6 * lu);
                st(B.q[0] + c, ldp(B.p[3] + c) + Y2 + Y1);
                st(B.q[1] + c, ldp(B.p[4] + c) + ku1);
                if constexpr (C2BAR) {
                    double Lu1, Lu2;
                    lapp(1, Lu1, Lu2);
                    st(B.q[4] + c, fma(kr2, Lu2, fma(kr1, Lu1, ldp(B.p[6] + c))));
                }
            }
        }
#pragma unroll
        for (int f = 0; f < NL; ++f) {
            q[f][0] = q[f][1];
            q[f][1] = q[f][2];
            q[f][2] = q[f][3];
            q[f][3] = q[f][4];
        }
        rq[0][0] = rq[0][1];
        rq[0][1] = rq[0][2];
        rq[1][0] = rq[1][1];
        rq[1][1] = rq[1][2];
        if (more) {
            double t[NL];
            adj_tf<PASS, C2BAR>(K, nr, t);
#pragma unroll
            for (int f = 0; f < NL; ++f)
                q[f][4] = t[f];
            rq[0][2] = nr[0];
            rq[1][2] = nr[1];
#pragma unroll
            for (int s = 0; s < T::HS; ++s)
                if (w.hl[s] >= 0) {
                    adj_tf<PASS, C2BAR>(K, nh[s], t);
#pragma unroll
                    for (int f = 0; f < NL; ++f)
                        hv[f][s] = t[f];
                }
        }
        buf ^= 1;
    }
}

// ---------------------------------------------------------------------------
// multi-field mixed-derivative kernel:
//   out = sum_a D2_a f + sum_{a<b} D_ab f + sum_{a,b} A_ab (D1_a f)(D1_b f)
// D_ab is the tensor product of two D1 stencils, evaluated factored: D_xy as
// D1_y of the D1_x plane (second LDS plane), D_xz and D_yz as D1_z of the
// register queues of D1_x f and D1_y f.  The LDS plane is the one being
// loaded (the leading plane k+2); its in-plane terms are computed on arrival
// and queued until plane k is complete.  Ghost zones (edges included) are
// read.

template <int TX, int NW>
__global__ __launch_bounds__(NW * 64) void k_mixed(MixArgs M, int nxcd)
{
    using T = Tile<TX, NW>;
    using MT = MixTile<TX, NW>;
    constexpr int LX = MT::LX;
    __shared__ double sf[2 * MT::PF];
    __shared__ double sd[2 * MT::PD];
    const int lin = xcd_remap(blockIdx.x, gridDim.x, nxcd);
    const int field = lin / M.items;
    const int item = lin - field * M.items;
    const DevBox &B = M.B;
    const ItemPos P = item_pos(B, item, TX, T::TY);
    const MixWalker<TX, NW> w(B, P, threadIdx.x);
    const double *__restrict__ f = M.f[field];
    double *__restrict__ out = M.out[field];
    const double d1x = M.d1[0], d1y = M.d1[1], d1z = M.d1[2];
    const double d2x = M.d2[0], d2y = M.d2[1], d2z = M.d2[2];
    const double cc = -30.0 * (d2x + d2y + d2z); // centre weight of the three D2

    // Column queues of f, D1_x f, D1_y f and D1_x f + D1_y f at planes kk-4
    // .. kk: plane step t writes the newest plane to slot t mod 5, so the
    // planes rotate through fixed registers (the loop below is unrolled
    // ten-fold: five slots times two fetch buffers; every slot index is a
    // compile-time constant).  D_xz + D_yz is D1_z of the sum queue.
    double fq[5] = {0, 0, 0, 0, 0}, xq[5] = {0, 0, 0, 0, 0}, yq[5] = {0, 0, 0, 0, 0};
    double sq[5] = {0, 0, 0, 0, 0};
    double pq0 = 0, pq1 = 0, pq2 = 0; // off-centre D2_x + D2_y taps plus D_xy, at kk-2 .. kk
    // The loads of plane kk+1 are issued as plane kk starts, into the one of
    // two buffers that alternate planes (so no register a load is still
    // filling is copied), and fly across the plane's two barriers.
    struct Fetched {
        double fv, hv[MT::HS];
    };
    auto fetch = [&](int kk, Fetched &X) {
        const int64_t zo = w.zoff(kk);
        X.fv = f[w.col + zo];
#pragma unroll
        for (int s = 0; s < MT::HS; ++s)
            if (w.hl[s] >= 0)
                X.hv[s] = f[w.hcol[s] + zo];
    };
    const int kfirst = P.z0 - 2, klast = P.z1 + 1;
    Fetched F0, F1;
    // plane step t = kk - kfirst = t0 + J with t0 a multiple of 10
    auto plane = [&](auto Jc, const int kk) {
        constexpr int J = decltype(Jc)::value;
        constexpr int S0 = (J + 1) % 5, S1 = (J + 2) % 5, S2 = (J + 3) % 5, S3 = (J + 4) % 5, S4 = J % 5;
        const Fetched &X = (J & 1) ? F1 : F0;
        Fetched &Y = (J & 1) ? F0 : F1;
        if (kk < klast)
            fetch(kk + 1, Y);
        const double fv = X.fv;
        double *F = sf + (J & 1) * MT::PF;
        double *D = sd + (J & 1) * MT::PD;
        F[w.lf] = fv;
#pragma unroll
        for (int s = 0; s < MT::HS; ++s)
            if (w.hl[s] >= 0)
                F[w.hl[s]] = X.hv[s];
        lds_barrier();
        const int c = w.lf;
        const double xm2 = F[c - 2], xm1 = F[c - 1], xp1 = F[c + 1], xp2 = F[c + 2];
        const double ym2 = F[c - 2 * LX], ym1 = F[c - LX], yp1 = F[c + LX], yp2 = F[c + 2 * LX];
        const double gx = d1x * fma(8.0, xp1 - xm1, -(xp2 - xm2));
        const double gy = d1y * fma(8.0, yp1 - ym1, -(yp2 - ym2));
        const double sx = fma(16.0, xm1 + xp1, -(xm2 + xp2));
        const double sy = fma(16.0, ym1 + yp1, -(ym2 + yp2));
        D[w.ld] = gx;
#pragma unroll
        for (int s = 0; s < MT::DS; ++s)
            if (w.dlf[s] >= 0) {
                const int e = w.dlf[s];
                D[w.dld[s]] = d1x * fma(8.0, F[e + 1] - F[e - 1], -(F[e + 2] - F[e - 2]));
            }
        lds_barrier();
        const int dd = w.ld;
        const double gxy = d1y * fma(8.0, D[dd + TX] - D[dd - TX], -(D[dd + 2 * TX] - D[dd - 2 * TX]));
        const double pin = fma(d2x, sx, fma(d2y, sy, gxy));
        fq[S4] = fv;
        xq[S4] = gx;
        yq[S4] = gy;
        sq[S4] = gx + gy;
        pq0 = pq1;
        pq1 = pq2;
        pq2 = pin;
        if (kk >= P.z0 + 2 && w.active) {
            const double gz = d1z * fma(8.0, fq[S3] - fq[S1], -(fq[S4] - fq[S0]));
            // the centre taps of D2_x, D2_y and D2_z, and D2_z's others
            const double d2c = fma(cc, fq[S2], d2z * fma(16.0, fq[S1] + fq[S3], -(fq[S0] + fq[S4])));
            const double gxyz = d1z * fma(8.0, sq[S3] - sq[S1], -(sq[S4] - sq[S0]));
            const double ex = xq[S2], ey = yq[S2];
            // the quadratic form in Horner-like groups:
            // ex (A_xx ex + A_xy' ey + A_xz' gz) + ey (A_yy ey + A_yz' gz) + A_zz gz gz
            double q = ex * fma(M.a[4], gz, fma(M.a[3], ey, M.a[0] * ex));
            q = fma(ey, fma(M.a[5], gz, M.a[1] * ey), q);
            q = fma(gz, M.a[2] * gz, q);
            st(out + w.point(B, kk - 2), (pq0 + d2c + gxyz) + q);
        }
    };
    fetch(kfirst, F0);
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using I6 = std::integral_constant<int, 6>;
    using I7 = std::integral_constant<int, 7>;
    using I8 = std::integral_constant<int, 8>;
    using I9 = std::integral_constant<int, 9>;
    for (int kk = kfirst; kk <= klast; kk += 10) {
        plane(I0{}, kk);
        if (kk + 1 <= klast) plane(I1{}, kk + 1);
        if (kk + 2 <= klast) plane(I2{}, kk + 2);
        if (kk + 3 <= klast) plane(I3{}, kk + 3);
        if (kk + 4 <= klast) plane(I4{}, kk + 4);
        if (kk + 5 <= klast) plane(I5{}, kk + 5);
        if (kk + 6 <= klast) plane(I6{}, kk + 6);
        if (kk + 7 <= klast) plane(I7{}, kk + 7);
        if (kk + 8 <= klast) plane(I8{}, kk + 8);
        if (kk + 9 <= klast) plane(I9{}, kk + 9);
    }
}

// ---------------------------------------------------------------------------
// periodic ghost fill: every ghost point copies the interior point at its
// wrapped coordinates.  One thread per ghost point; the ghost shell of a box
// is enumerated as two z slabs (full x, y extent), two y slabs (full x
// extent, interior z) and two x slabs (interior y, z).

__global__ __launch_bounds__(256) void k_fill_periodic(DevBox B)
{
    int i, j, k;
    if (!ghost_point(B, (int64_t)blockIdx.x * 256 + threadIdx.x, i, j, k))
        return;
    double *f = B.q[0];
    f[elem(B, i, j, k)] = f[elem(B, wrap_index(i, B.n[0]), wrap_index(j, B.n[1]), wrap_index(k, B.n[2]))];
}

// ---------------------------------------------------------------------------
// level ghost exchange: every workgroup copies up to 256 points of one piece
// (W[blockIdx.x] names it), x fastest so rows of a piece coalesce.  Sources
// are interior points and destinations ghost points, so the pieces of one
// launch never read what another writes.

__global__ __launch_bounds__(256) void k_sync(const SyncPiece *__restrict__ P, const int *__restrict__ W,
                                              double *const *__restrict__ F, int nf, int nbox)
{
    const SyncPiece &q = P[W[blockIdx.x]];
    // piece volumes are below 2^31 (checked on the host): 32-bit index arithmetic
    const unsigned t = (unsigned)(blockIdx.x - q.blk0) * 256u + threadIdx.x;
    const unsigned nx = (unsigned)q.n[0], ny = (unsigned)q.n[1];
    if (t >= nx * ny * (unsigned)q.n[2])
        return;
    const unsigned r = t / nx, i = t - r * nx;
    const unsigned k = r / ny, j = r - k * ny;
    const int64_t so = q.soff + i + (int64_t)j * q.ssy + (int64_t)k * q.ssz;
    const int64_t d = q.doff + i + (int64_t)j * q.dsy + (int64_t)k * q.dsz;
    for (int f = 0; f < nf; ++f) {
        double *const *Ff = F + (size_t)f * nbox;
        Ff[q.dst][d] = Ff[q.src][so];
    }
}

// ---------------------------------------------------------------------------
// streaming copy probe: one 16-byte vector per lane and one launch-wide pass
// (workgroup w copies bytes [4096 w, 4096 (w + 1))), non-temporal both ways.
// Workgroups are dispatched in index order, so the waves in flight at any
// time cover one compact window of both buffers.  On MI355X this pattern
// streams faster than a fixed grid that strides through the buffers.


__global__ __launch_bounds__(256) void k_copy(dvec2 *__restrict__ dst, const dvec2 *__restrict__ src,
                                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ---------------------------------------------------------------------------
// host-side launchers

template <int TX, int NW, bool WRAP, int OPK>
static hipError_t launch_single_t(const DevBox &B, const StageCoef &K, int nitems, int nxcd, hipStream_t s)
{
    hipLaunchKernelGGL((k_tiles_single<TX, NW, WRAP, OPK>), dim3(nitems), dim3(NW * 64), 0, s, B, K, nxcd);
    return hipGetLastError();
}

template <int TX, int NW, bool WRAP, int OPK>
static hipError_t launch_batched_t(const DevBox *tab, int nbox, const ItemQueue &Q, int grid,
                                   const StageCoef &K, hipStream_t s)
{
    hipLaunchKernelGGL((k_tiles_batched<TX, NW, WRAP, OPK>), dim3(grid), dim3(NW * 64), 0, s, tab, nbox, Q, K);
    return hipGetLastError();
}

#define S4_FOR_OPS(X, TX, NW)                                                                          \
    X(TX, NW, false, OP_RHS)                                                                           \
    X(TX, NW, true, OP_STAGE)                                                                          \
    X(TX, NW, false, OP_STAGE)                                                                         \
    X(TX, NW, true, OP_ADJRHS)

#define S4_FOR_SHAPES(X)                                                                               \
    S4_FOR_OPS(X, 64, 4)                                                                               \
    S4_FOR_OPS(X, 64, 8)                                                                               \
    S4_FOR_OPS(X, 32, 4)                                                                               \
    S4_FOR_OPS(X, 32, 8)                                                                               \
    S4_FOR_OPS(X, 16, 4)                                                                               \
    S4_FOR_OPS(X, 16, 8)

// periodic addressing for every op but the RHS, unless the caller's ghost
// zones hold the neighbours (a level whose boxes exchange ghosts)
static bool wrap_of(int op, bool ghosted)
{
    return op != OP_RHS && !ghosted;
}

hipError_t launch_tiles_single(int op, int tx, int nw, const DevBox &B, const StageCoef &K, int nitems,
                               int nxcd, hipStream_t s, bool ghosted)
{
    const bool wrap = wrap_of(op, ghosted);
#define X(TX_, NW_, W_, O_)                                                                            \
    if (tx == TX_ && nw == NW_ && wrap == W_ && op == O_)                                              \
        return launch_single_t<TX_, NW_, W_, O_>(B, K, nitems, nxcd, s);
    S4_FOR_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_tiles_batched(int op, int tx, int nw, const DevBox *tab, int nbox, const ItemQueue &Q,
                                int grid, const StageCoef &K, hipStream_t s, bool ghosted)
{
    const bool wrap = wrap_of(op, ghosted);
#define X(TX_, NW_, W_, O_)                                                                            \
    if (tx == TX_ && nw == NW_ && wrap == W_ && op == O_)                                              \
        return launch_batched_t<TX_, NW_, W_, O_>(tab, nbox, Q, grid, K, s);
    S4_FOR_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_pairs_rhs(int txl, int nw, const DevBox &B, int nitems, int nxcd, hipStream_t s)
{
#define X(TXL_, NW_)                                                                                   \
    if (txl == TXL_ && nw == NW_) {                                                                    \
        if (B.p[0])                                                                                    \
            hipLaunchKernelGGL((k_pairs_rhs<TXL_, NW_, true>), dim3(nitems), dim3(NW_ * 64), 0, s, B,  \
                               nxcd);                                                                  \
        else                                                                                           \
            hipLaunchKernelGGL((k_pairs_rhs<TXL_, NW_, false>), dim3(nitems), dim3(NW_ * 64), 0, s, B, \
                               nxcd);                                                                  \
        return hipGetLastError();                                                                      \
    }
    X(64, 8) X(64, 4) X(32, 8) X(32, 4)
#undef X
    return hipErrorInvalidValue;
}

int max_blocks_per_cu(int op, int tx, int nw, bool ghosted)
{
    const bool wrap = wrap_of(op, ghosted);
    int nb = 0;
#define X(TX_, NW_, W_, O_)                                                                            \
    if (tx == TX_ && nw == NW_ && wrap == W_ && op == O_) {                                            \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiles_batched<TX_, NW_, W_, O_>,        \
                                                         NW_ * 64, 0) != hipSuccess)                   \
            return 0;                                                                                  \
        return nb;                                                                                     \
    }
    S4_FOR_SHAPES(X)
#undef X
    return 0;
}


// row-register kernels: (WX, RY) with WX * WY = 4 wavefronts
template <int WX, int RY, bool WRAP, int OPK>
static hipError_t launch_rows_single_t(const DevBox &B, const StageCoef &K, int nitems, int nxcd, hipStream_t s)
{
    constexpr int WY = 4 / WX;
    hipLaunchKernelGGL((k_rows_single<WX, WY, RY, WRAP, OPK>), dim3(nitems), dim3(WX * WY * 64), 0, s, B, K, nxcd);
    return hipGetLastError();
}

template <int WX, int RY, bool WRAP, int OPK>
static hipError_t launch_rows_batched_t(const DevBox *tab, int nbox, const ItemQueue &Q, int grid,
                                        const StageCoef &K, hipStream_t s)
{
    constexpr int WY = 4 / WX;
    hipLaunchKernelGGL((k_rows_batched<WX, WY, RY, WRAP, OPK>), dim3(grid), dim3(WX * WY * 64), 0, s, tab, nbox,
                       Q, K);
    return hipGetLastError();
}

#define S4_ROW_OPS(X, WX, RY)                                                                          \
    X(WX, RY, false, OP_RHS)                                                                           \
    X(WX, RY, true, OP_STAGE)                                                                          \
    X(WX, RY, false, OP_STAGE)

#define S4_ROW_SHAPES(X)                                                                               \
    S4_ROW_OPS(X, 4, 4)                                                                                \
    S4_ROW_OPS(X, 4, 2)                                                                                \
    S4_ROW_OPS(X, 2, 4)                                                                                \
    S4_ROW_OPS(X, 2, 2)                                                                                \
    S4_ROW_OPS(X, 1, 4)                                                                                \
    S4_ROW_OPS(X, 1, 2)

hipError_t launch_rows_single(int op, int wx, int ry, const DevBox &B, const StageCoef &K, int nitems, int nxcd,
                              hipStream_t s, bool ghosted)
{
    const bool wrap = wrap_of(op, ghosted);
#define X(WX_, RY_, W_, O_)                                                                            \
    if (wx == WX_ && ry == RY_ && wrap == W_ && op == O_)                                              \
        return launch_rows_single_t<WX_, RY_, W_, O_>(B, K, nitems, nxcd, s);
    S4_ROW_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_rows_batched(int op, int wx, int ry, const DevBox *tab, int nbox, const ItemQueue &Q,
                               int grid, const StageCoef &K, hipStream_t s, bool ghosted)
{
    const bool wrap = wrap_of(op, ghosted);
#define X(WX_, RY_, W_, O_)                                                                            \
    if (wx == WX_ && ry == RY_ && wrap == W_ && op == O_)                                              \
        return launch_rows_batched_t<WX_, RY_, W_, O_>(tab, nbox, Q, grid, K, s);
    S4_ROW_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

int max_blocks_rows(int op, int wx, int ry, bool ghosted)
{
    const bool wrap = wrap_of(op, ghosted);
    int nb = 0;
#define X(WX_, RY_, W_, O_)                                                                            \
    if (wx == WX_ && ry == RY_ && wrap == W_ && op == O_) {                                            \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rows_batched<WX_, 4 / WX_, RY_, W_, O_>, \
                                                         256, 0) != hipSuccess)                        \
            return 0;                                                                                  \
        return nb;                                                                                     \
    }
    S4_ROW_SHAPES(X)
#undef X
    return 0;
}

hipError_t launch_mixed(int tx, int nw, const MixArgs &M, int nfield, int nxcd, hipStream_t s)
{
    const int64_t grid = (int64_t)M.items * nfield;
    if (grid <= 0 || grid > 0x7fffffff)
        return hipErrorInvalidValue;
#define X(TX_, NW_)                                                                                    \
    if (tx == TX_ && nw == NW_) {                                                                      \
        hipLaunchKernelGGL((k_mixed<TX_, NW_>), dim3((unsigned)grid), dim3(NW_ * 64), 0, s, M, nxcd);  \
        return hipGetLastError();                                                                      \
    }
    X(64, 4) X(64, 8) X(32, 4) X(32, 8) X(16, 4) X(16, 8)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_rk4_pair(int pair, int txe, int nw, const DevBox &B, const StageCoef &K1, const StageCoef &K2,
                           int nitems, int nxcd, hipStream_t s)
{
#define Y(TXE_, NW_, P_, C_)                                                                           \
    hipLaunchKernelGGL((k_rk4_pair<TXE_, NW_, P_, C_>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K1, K2, nxcd)
#define X(TXE_, NW_)                                                                                   \
    if (txe == TXE_ && nw == NW_) {                                                                    \
        const bool c2 = B.p[5] != nullptr;                                                             \
        if (pair == 0 && c2)                                                                           \
            Y(TXE_, NW_, 0, true);                                                                     \
        else if (pair == 0)                                                                            \
            Y(TXE_, NW_, 0, false);                                                                    \
        else if (c2)                                                                                   \
            Y(TXE_, NW_, 1, true);                                                                     \
        else                                                                                           \
            Y(TXE_, NW_, 1, false);                                                                    \
        return hipGetLastError();                                                                      \
    }
    X(32, 8) X(64, 8) X(64, 16) X(32, 16)
#undef X
#undef Y
    return hipErrorInvalidValue;
}

hipError_t launch_rk4_step4(int txe, int nw, const DevBox &B, const StageCoef K[4], int run, int nxcd,
                            hipStream_t s, bool ghosted)
{
    const int64_t total = (int64_t)B.tiles[0] * B.tiles[1] * B.n[2];
    // the output stores address one z plane with 31-bit byte offsets; y_3
    // goes to q[2] and q[3] when both are given
    const bool y3 = B.q[2] != nullptr;
    if (run < 0 || total <= 0 || B.sz * 8 >= (int64_t)NO_STORE || y3 != (B.q[3] != nullptr) ||
        (ghosted && (y3 || B.g < 4)))
        return hipErrorInvalidValue;
    const int64_t grid = run == 0 ? (int64_t)B.tiles[0] * B.tiles[1] * B.tiles[2] : (total + run - 1) / run;
    const Step4Coef C{K[0].a, K[1].a, K[1].b, K[2].a, K[2].b, K[3].b};
#define Y(K_, TXE_, NW_, C_)                                                                           \
    hipLaunchKernelGGL((K_<TXE_, NW_, C_>), dim3((unsigned)grid), dim3(NW_ * 64), 0, s, B, C, run, nxcd)
#define G(TXE_, NW_, C_)                                                                               \
    hipLaunchKernelGGL((k_rk4_step4<TXE_, NW_, C_, false>), dim3((unsigned)grid), dim3(NW_ * 64), 0, s, B, C, \
                       run, nxcd)
#define X(TXE_, NW_)                                                                                   \
    if (txe == TXE_ && nw == NW_) {                                                                    \
        if (ghosted && B.p[5] != nullptr)                                                              \
            G(TXE_, NW_, true);                                                                        \
        else if (ghosted)                                                                              \
            G(TXE_, NW_, false);                                                                       \
        else if (y3 && B.p[5] != nullptr)                                                              \
            Y(k_rk4_step4_y3, TXE_, NW_, true);                                                        \
        else if (y3)                                                                                   \
            Y(k_rk4_step4_y3, TXE_, NW_, false);                                                       \
        else if (B.p[5] != nullptr)                                                                    \
            Y(k_rk4_step4, TXE_, NW_, true);                                                           \
        else                                                                                           \
            Y(k_rk4_step4, TXE_, NW_, false);                                                          \
        return hipGetLastError();                                                                      \
    }
    X(32, 8) X(64, 16) X(32, 16) X(68, 16)
#undef X
#undef Y
#undef G
    return hipErrorInvalidValue;
}

hipError_t launch_rk4_step4_batched(int txe, int nw, bool hasc2, const DevBox *tab, int nbox, const ItemQueue &Q,
                                    int grid, const StageCoef K[4], hipStream_t s, bool ghosted)
{
    const Step4Coef C{K[0].a, K[1].a, K[1].b, K[2].a, K[2].b, K[3].b};
#define Y(TXE_, NW_, C_, W_)                                                                           \
    hipLaunchKernelGGL((k_rk4_step4_batched<TXE_, NW_, C_, W_>), dim3(grid), dim3(NW_ * 64), 0, s, tab, nbox, Q, C)
#define X(TXE_, NW_)                                                                                   \
    if (txe == TXE_ && nw == NW_) {                                                                    \
        if (hasc2 && ghosted)                                                                          \
            Y(TXE_, NW_, true, false);                                                                 \
        else if (hasc2)                                                                                \
            Y(TXE_, NW_, true, true);                                                                  \
        else if (ghosted)                                                                              \
            Y(TXE_, NW_, false, false);                                                                \
        else                                                                                           \
            Y(TXE_, NW_, false, true);                                                                 \
        return hipGetLastError();                                                                      \
    }
    X(32, 8) X(64, 16) X(32, 16) X(68, 16)
#undef X
#undef Y
    return hipErrorInvalidValue;
}

int max_blocks_step4(int txe, int nw)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define X(TXE_, NW_)                                                                                   \
    if (txe == TXE_ && nw == NW_)                                                                      \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_step4<TXE_, NW_, true>, NW_ * 64, 0);
    X(32, 8) X(64, 16) X(32, 16) X(68, 16)
#undef X
    return e == hipSuccess ? nb : 0;
}


#define S4_PAIR2_SHAPES(X)                                                                             \
    X(64, 4) X(64, 8) X(32, 4) X(32, 8) X(16, 4) X(16, 8)

hipError_t launch_pair2(int pair, int tx, int nw, const DevBox &B, const StageCoef &K1, const StageCoef &K2,
                        int nitems, int nxcd, hipStream_t s, bool ghosted)
{
#define X(TX_, NW_)                                                                                    \
    if (tx == TX_ && nw == NW_) {                                                                      \
        if (pair == 0 && !ghosted)                                                                     \
            hipLaunchKernelGGL((k_pair2<TX_, NW_, 0, true>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K1, K2, nxcd); \
        else if (pair == 0)                                                                            \
            hipLaunchKernelGGL((k_pair2<TX_, NW_, 0, false>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K1, K2, nxcd); \
        else if (!ghosted)                                                                             \
            hipLaunchKernelGGL((k_pair2<TX_, NW_, 1, true>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K1, K2, nxcd); \
        else                                                                                           \
            hipLaunchKernelGGL((k_pair2<TX_, NW_, 1, false>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K1, K2, nxcd); \
        return hipGetLastError();                                                                      \
    }
    S4_PAIR2_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_pair2_batched(int pair, int tx, int nw, const DevBox *tab, int nbox, const ItemQueue &Q,
                                int grid, const StageCoef &K1, const StageCoef &K2, hipStream_t s, bool ghosted)
{
#define X(TX_, NW_)                                                                                    \
    if (tx == TX_ && nw == NW_) {                                                                      \
        if (pair == 0 && !ghosted)                                                                     \
            hipLaunchKernelGGL((k_pair2_batched<TX_, NW_, 0, true>), dim3(grid), dim3(NW_ * 64), 0, s, tab, nbox, \
                               Q, K1, K2);                                               \
        else if (pair == 0)                                                                            \
            hipLaunchKernelGGL((k_pair2_batched<TX_, NW_, 0, false>), dim3(grid), dim3(NW_ * 64), 0, s, tab, nbox, \
                               Q, K1, K2);                                               \
        else if (!ghosted)                                                                             \
            hipLaunchKernelGGL((k_pair2_batched<TX_, NW_, 1, true>), dim3(grid), dim3(NW_ * 64), 0, s, tab, nbox, \
                               Q, K1, K2);                                               \
        else                                                                                           \
            hipLaunchKernelGGL((k_pair2_batched<TX_, NW_, 1, false>), dim3(grid), dim3(NW_ * 64), 0, s, tab, nbox, \
                               Q, K1, K2);                                               \
        return hipGetLastError();                                                                      \
    }
    S4_PAIR2_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

int max_blocks_pair2(int pair, int tx, int nw, bool ghosted)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define X(TX_, NW_)                                                                                    \
    if (tx == TX_ && nw == NW_) {                                                                      \
        if (pair == 0)                                                                                 \
            e = ghosted ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair2_batched<TX_, NW_, 0, false>, NW_ * 64, 0) \
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair2_batched<TX_, NW_, 0, true>, NW_ * 64, 0); \
        else                                                                                           \
            e = ghosted ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair2_batched<TX_, NW_, 1, false>, NW_ * 64, 0) \
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair2_batched<TX_, NW_, 1, true>, NW_ * 64, 0); \
    }
    S4_PAIR2_SHAPES(X)
#undef X
    return e == hipSuccess ? nb : 0;
}


hipError_t launch_adj2(int pass, int tx, int nw, bool c2bar, const DevBox &B, const StageCoef &K, int nitems,
                       int nxcd, hipStream_t s)
{
#define X(TX_, NW_)                                                                                    \
    if (tx == TX_ && nw == NW_) {                                                                      \
        if (pass == 0 && !c2bar)                                                                       \
            hipLaunchKernelGGL((k_adj2<TX_, NW_, 0, false>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K, nxcd); \
        else if (pass == 0)                                                                            \
            hipLaunchKernelGGL((k_adj2<TX_, NW_, 0, true>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K, nxcd); \
        else if (!c2bar)                                                                               \
            hipLaunchKernelGGL((k_adj2<TX_, NW_, 1, false>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K, nxcd); \
        else                                                                                           \
            hipLaunchKernelGGL((k_adj2<TX_, NW_, 1, true>), dim3(nitems), dim3(NW_ * 64), 0, s, B, K, nxcd); \
        return hipGetLastError();                                                                      \
    }
    X(64, 8) X(64, 4) X(32, 8) X(32, 4) X(16, 8) X(16, 4)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_fill(const DevBox &B, hipStream_t s)
{
    const int64_t nblk = (ghost_count(B) + 255) / 256;
    if (nblk > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_periodic, dim3((unsigned)nblk), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_sync(const SyncPiece *P, const int *W, double *const *F, int nf, int nbox, int nblocks,
                       hipStream_t s)
{
    if (nblocks <= 0 || nf <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_sync, dim3((unsigned)nblocks), dim3(256), 0, s, P, W, F, nf, nbox);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (dvec2 *)dst,
                       (const dvec2 *)src, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch memory of s4_rk4_noalloc: one array per device, zero when the code
// object loads, held until the process ends.  Its name in host code stands
// for the host-side shadow, not a device address, so it is never passed to
// a kernel or a copy: noalloc_scratch looks the device address up once per
// device (with that device current) and callers use that address.

static __device__ __attribute__((aligned(256))) unsigned char scratch[S4_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void **ptr)
{
    static std::mutex mu;
    static std::map<int, void *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        it = addr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

} // namespace s4
