// s4_api.cpp -- the C ABI of libsten4 (declared in include/sten4.h): argument
// validation, workspace layout, tile choice and tuning, box tables for the
// persistent batched launch, the hipGraph cache of one RK4 step, and the
// device side of a level's ghost exchange (s4_level_sync, s4_level_rk4).
//
// Tile choice follows the paper's LoopControl (Sec. III-B): every "loop
// setup" (operation, box sizes, ghost width, strides, device) gets initial
// execution parameters from a heuristic fed by the device's properties, and
// measured timings replace them with faster candidates: either an explicit
// sweep (s4_tune) or, as in the paper, on-line random-restart hill climbing
// inside the calls (s4_set_online_tuning).  Sweep results persist in a JSON
// file, the keeping of tuned parameters across runs that the paper proposes
// as future work (Sec. III-C).  Each entry names its candidate by its
// parameters, so a file written against another candidate table is read
// safely: entries that match no candidate, or one the op cannot run on
// those boxes, are dropped.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "s4_bboxset.h"
#include "s4_internal.h"
#include "s4_launch.h"
#include "sten4.h"

using namespace s4;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace s4 {
int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
} // namespace s4

static int hip_fail(hipError_t e, const char *where)
{
    return fail(S4_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define S4_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return hip_fail(e_, #call);                                                                \
    } while (0)

// ---------------------------------------------------------------------------
// tile candidates (the tuner's search space) and choices

// A candidate is a kernel set and its tile (the paper's "execution
// parameters" plus its future-work choice between sets of loop kernels,
// Sec. III-C).  variant 0: one kernel per operation or RK4 stage on the LDS
// tile traversal, tile tx x (nw*64/tx); variant 2: the same kernels on the
// row-register traversal, nw = 4 wavefronts of which tx/64 lie along x,
// each holding ry rows (item tx x ry*nw*64/tx); variants 1 and 3 (RK4 on one
// box only for variant 1): two kernels per step, each running two RK4
// stages -- variant 1 recomputes the first stage on a widened workgroup tile
// tx x (nw*64/tx) with output tile (tx-4) x (nw*64/tx - 4), variant 3 forms
// the second stage's stencil input at each tap on the plain tile
// tx x (nw*64/tx) (any number of boxes, levels included); variant 4 (any
// number of periodic boxes, or a wide level) runs a whole RK4 step per pass
// on the widened tile of variant 1 (tx 68: 68 x 15 on 1020 of 1024 lanes),
// stages 1-2 on all lanes and 3-4 on the output tile; variant 5 (the wave
// RHS on boxes with an even n[0] and even strides) is the tile traversal
// with two x points per lane, tile 2 tx x (nw*64/tx).  tz is the z chunk (0 = whole box; for variant 4 on one
// box, equal shares of the tile-plane sequence).  Candidate indices are
// stable across ops: an op skips the candidates it cannot use.
struct Cand {
    int tx, nw, tz;
    int variant;
    int ry;
};

static const std::vector<Cand> &cands()
{
    static const std::vector<Cand> v = [] {
        std::vector<Cand> c;
        for (int tx : {64, 32, 16})
            for (int nw : {8, 4})
                for (int tz : {0, 64, 32, 16, 8})
                    c.push_back({tx, nw, tz, 0, 0});
        for (int tx : {256, 128, 64})
            for (int ry : {4, 2})
                for (int tz : {64, 32, 16})
                    c.push_back({tx, 4, tz, 2, ry});
        for (auto tn : {std::pair<int, int>{64, 4}, {64, 8}, {32, 8}, {32, 4}, {16, 8}, {16, 4}})
            for (int tz : {64, 32, 16})
                c.push_back({tn.first, tn.second, tz, 3, 0});
        // (64 x 8 wastes half its lanes; 68 x 15 covers a 256-point row in
        // four output tiles)
        for (auto tn : {std::pair<int, int>{64, 16}, {32, 16}, {32, 8}, {68, 16}})
            for (int tz : {0, 128, 64, 32, 16})
                c.push_back({tn.first, tn.second, tz, 4, 0});
        for (auto tn : {std::pair<int, int>{32, 8}, {64, 8}, {64, 16}, {32, 16}})
            for (int tz : {64, 32, 16})
                c.push_back({tn.first, tn.second, tz, 1, 0});
        for (int tx : {64, 32}) // pair-lane tiles: tx lanes of two points (wave RHS)
            for (int nw : {8, 4})
                for (int tz : {64, 32, 16})
                    c.push_back({tx, nw, tz, 5, 0});
        return c;
    }();
    return v;
}

static int cand_index(int tx, int nw, int tz, int variant = 0, int ry = 0)
{
    const auto &c = cands();
    for (size_t i = 0; i < c.size(); ++i)
        if (c[i].tx == tx && c[i].nw == nw && c[i].tz == tz && c[i].variant == variant && c[i].ry == ry)
            return (int)i;
    return 0;
}

// whether candidate c may run op on nbox boxes
static bool cand_allowed(const Cand &c, int op, int nbox)
{
    if (c.variant == 0)
        return true;
    if (c.variant == 2)
        return op == S4_OP_WAVE_RHS || op == S4_OP_RK4;
    if (c.variant == 5)
        return op == S4_OP_WAVE_RHS;
    if (c.variant == 3 || c.variant == 4)
        return op == S4_OP_RK4;
    return op == S4_OP_RK4 && nbox == 1; // variant 1
}

// whether candidate c can run on these boxes: the whole-step kernels address
// one z plane with 31-bit byte offsets
static bool cand_fits(const Cand &c, const s4_box *b, int nbox)
{
    if (c.variant == 5) { // pair-lane tiles: 16-byte pairs along whole rows
        for (int i = 0; i < nbox; ++i)
            if (b[i].n[0] % 2 || b[i].stride[1] % 2 || b[i].stride[2] % 2)
                return false;
        return true;
    }
    if (c.variant != 4)
        return true;
    for (int i = 0; i < nbox; ++i)
        if (b[i].stride[2] * 8 >= (int64_t)0x80000000)
            return false;
    return true;
}

// Levels: 1 = a level whose exchanges fill ghost zones of width 2 or 3
// (ghost-addressed stencils of radius 2), 2 = a wide level (exchanges of
// the full ghost shell of width 4 or more, every box with 4 or more ghost
// layers), on which a whole RK4 step reads its radius-4 neighbourhood from
// the ghost zones after one exchange per step.
static const int LEVEL_NARROW = 1, LEVEL_WIDE = 2;

// whether candidate c can run RK4 on a level of that kind: the widened-tile
// stage pairs wrap around one box; the whole steps need a wide level
static bool level_capable(const Cand &c, int level)
{
    return c.variant != 1 && (c.variant != 4 || level == LEVEL_WIDE);
}

static int kernel_op(int op)
{
    switch (op) {
    case S4_OP_WAVE_RHS: return OP_RHS;
    case S4_OP_RK4: return OP_STAGE;
    case S4_OP_ADJOINT_RHS: return OP_ADJRHS;
    case S4_OP_ADJOINT_STEP: return OP_ADJSTEP;
    case S4_OP_DERIV_MIXED: return OP_COUNT; // its own kernel, k_mixed
    default: return -1;
    }
}

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr; // recorded after the entry's latest launches
    uint64_t used = 0;         // context tick of the latest use (LRU eviction)
};

// Wait for an entry's launches, then free it.
static void graph_free(GraphEntry &ge)
{
    if (ge.done) {
        (void)hipEventSynchronize(ge.done);
        (void)hipEventDestroy(ge.done);
    }
    if (ge.exec)
        (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph)
        (void)hipGraphDestroy(ge.graph);
    ge = GraphEntry{};
}

// ---------------------------------------------------------------------------
// On-line tuning of one loop setup: the paper's run-time random-restart hill
// climbing (Sec. III-B).  Starting from the heuristic setting, each timing
// of a call is fed back; the neighbourhood of the best setting so far is
// tried one setting per call, the best moves to any neighbour that is
// faster, and once the neighbourhood is exhausted a random setting is tried
// with a small probability per call and its neighbourhood explored.  A trial
// that is much slower than the best is abandoned after that one call, so
// excursions stay cheap: the aim is a short total run time, not the optimum.

// position of a candidate's parameters in their value orders
static int ord_tx(int tx) { return tx == 16 ? 0 : tx == 32 ? 1 : tx == 64 || tx == 68 ? 2 : tx == 128 ? 3 : 4; }
static int ord_ry(int ry) { return ry == 4 ? 1 : 0; }
static int ord_nw(int nw) { return nw == 4 ? 0 : nw == 8 ? 1 : 2; }
static int ord_tz(int tz) { return tz == 8 ? 0 : tz == 16 ? 1 : tz == 32 ? 2 : tz == 64 ? 3 : tz == 128 ? 4 : 5; }

struct Hill {
    std::vector<int> allowed;     // candidates this setup may use
    int best = -1;                // best setting so far and its time per unit
    double best_t = 0.0;
    std::vector<int> todo;        // neighbours still to try
    bool excursion = false;       // exploring around a random restart
    double restart_prob = 0.02;
    double improve = 0.02;        // a move needs this relative gain (timing noise)
    double abort_ratio = 1.5;     // a trial this much slower than the best ends an excursion
    uint64_t rng = 0x9E3779B97F4A7C15ull;
    std::map<int, double> seen;   // fastest time measured per setting
    int start = 0;

    double uniform()
    {
        // splitmix64 step (Steele, Lea and Flood 2014)
        uint64_t z = (rng += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    }

    // settings one step away: one parameter moved to its neighbouring value
    // in the same kernel set, or the nearest settings of each other set
    std::vector<int> neighbours(int c) const;

    int next()
    {
        if (best < 0)
            return start;
        while (!todo.empty()) {
            const int c = todo.back();
            todo.pop_back();
            if (!seen.count(c))
                return c;
        }
        excursion = false;
        if (allowed.size() > 1 && uniform() < restart_prob) {
            const int r = allowed[(size_t)(uniform() * allowed.size()) % allowed.size()];
            if (r != best) {
                excursion = true;
                todo = neighbours(r);
                return r;
            }
        }
        return best;
    }

    void measured(int c, double t)
    {
        auto it = seen.find(c);
        seen[c] = it == seen.end() ? t : std::min(it->second, t);
        if (best < 0) {
            best = c;
            best_t = t;
            todo = neighbours(c);
            return;
        }
        if (c == best) {
            best_t = std::min(best_t, t);
            return;
        }
        if (t < best_t * (1.0 - improve)) { // move uphill
            best = c;
            best_t = t;
            todo = neighbours(c);
            excursion = false;
            return;
        }
        if (excursion && t > best_t * abort_ratio) { // abandon a bad excursion at once
            todo.clear();
            excursion = false;
        }
    }
};

struct OnlinePending {
    hipEvent_t a, b;
    int cand;
    double units;
};

struct OnlineSetup {
    Hill hill;
    std::deque<OnlinePending> pending;
    std::vector<hipEvent_t> pool;
};

struct s4_ctx {
    int device = 0;
    int ncu = 256;
    int nxcd = 8;
    // resident workgroups per CU of the whole-step shapes 32 x 16, 64 x 16,
    // 32 x 32 and 68 x 15 lanes (LDS-bound; queried from the device at
    // creation)
    int step4_per[4] = {2, 1, 1, 1};
    std::string name;
    std::string cache_path;
    hipStream_t cap = nullptr; // private stream used only to capture graphs
    void *scratch = nullptr;   // device address of s4_rk4_noalloc's array on this device
    std::string scratch_err;   // why it has none
    std::map<std::string, int> tuned;
    std::map<std::string, int> forced;
    std::map<std::string, GraphEntry> graphs;
    uint64_t graph_tick = 0;
    std::mutex cap_mu; // one capture at a time on the private stream
    bool online = false; // on-line hill climbing of every loop setup
    double restart_prob = 0.02;
    uint64_t seed = 1;
    std::map<std::string, OnlineSetup> online_state;
    std::mutex mu;
};

// c2: RK4 calls that pass a variable c^2 (one more field read per point
// and different register pressure) form a loop setup of their own
static std::string setup_key_on(const std::string &device, int op, const s4_box *b, int nbox, bool c2 = false)
{
    std::ostringstream o;
    o << "op" << op << "|" << device << "|" << nbox;
    for (int i = 0; i < nbox; ++i)
        o << "|" << b[i].n[0] << "," << b[i].n[1] << "," << b[i].n[2] << ",g" << b[i].ghost << ",s"
          << b[i].stride[1] << "," << b[i].stride[2];
    if (c2)
        o << "|c2";
    return o.str();
}

static std::string setup_key(const s4_ctx *ctx, int op, const s4_box *b, int nbox, bool c2 = false)
{
    return setup_key_on(ctx->name, op, b, nbox, c2);
}

// whether an RK4 call passes c^2 for any box
static bool has_c2(const double *const *c2, int nbox)
{
    for (int i = 0; c2 && i < nbox; ++i)
        if (c2[i])
            return true;
    return false;
}

// strips S4_WITH_C2 from op; only S4_OP_RK4 takes it
static int split_op(int &op, bool &c2)
{
    c2 = (op & S4_WITH_C2) != 0;
    op &= ~S4_WITH_C2;
    if (c2 && op != S4_OP_RK4)
        return fail(S4_EINVAL, "S4_WITH_C2 applies to S4_OP_RK4 only (op %d)", op);
    return S4_OK;
}

static int tile_ty(const Cand &c)
{
    if (c.variant == 2)
        return c.ry * (c.nw * 64 / c.tx);
    return c.nw * 64 / c.tx;
}

// output tile extents in x and y
static int out_tx(const Cand &c)
{
    return c.variant == 1 || c.variant == 4 ? c.tx - 4 : c.variant == 5 ? 2 * c.tx : c.tx;
}

static int out_ty(const Cand &c)
{
    return c.variant == 1 || c.variant == 4 ? tile_ty(c) - 4 : tile_ty(c);
}

static int64_t items_of(const s4_box &b, const Cand &c)
{
    const int tx = out_tx(c), ty = out_ty(c);
    const int tz = c.tz > 0 ? std::min(c.tz, b.n[2]) : b.n[2];
    return (int64_t)((b.n[0] + tx - 1) / tx) * ((b.n[1] + ty - 1) / ty) * ((b.n[2] + tz - 1) / tz);
}

// LoopControl-style initial parameters of the per-operation kernels
// (variant 0): the widest x tile the boxes fill, 8 wavefronts, and the
// longest z chunk that still gives every CU about four workgroups.
static int tile_heuristic(const s4_ctx *ctx, const s4_box *b, int nbox)
{
    int maxnx = 0;
    for (int i = 0; i < nbox; ++i)
        maxnx = std::max(maxnx, b[i].n[0]);
    const int tx = maxnx >= 48 ? 64 : maxnx >= 24 ? 32 : 16;
    const int nw = 8;
    for (int tz : {0, 64, 32, 16}) {
        int64_t items = 0;
        for (int i = 0; i < nbox; ++i)
            items += items_of(b[i], {tx, nw, tz, 0, 0});
        if (items >= 4 * (int64_t)ctx->ncu)
            return cand_index(tx, nw, tz);
    }
    return cand_index(tx, nw, 8);
}

// Starting setting of an op.  RK4 runs a whole step per pass (variant 4):
// on one box the setting of least modelled cost (step4_single), on a set of
// boxes 32 x 16 lanes (two workgroups per CU) in 32-plane chunks, the
// sweep's pick on the 60-box set.  On a level (level: radius-2 ghost zones
// only), and for z planes of 2 GiB or more, RK4 runs two stages per pass
// with
// the per-tap stage pairs (variant 3): tile 64 x 4 (whole 512-byte rows)
// unless idle lanes of ragged boxes would pass a fifth of the lanes, then
// 32 x 16; the longest z chunk that gives every CU four items (eight over
// several boxes, whose uneven sizes the work queue balances best in small
// pieces).
// Equal runs of a box's tile-plane sequence (total tile-planes) for the
// whole-step kernel: shared by one round of resident workgroups (slots),
// but no shorter than min(4, total / CUs) planes.  Each run pays the
// pipeline's 8-plane start-up, so long runs amortise it; a box too small to
// give every CU 4 planes instead spreads over the CUs in shorter runs (its
// data sit in cache, and the step's latency is what is left).  On periodic
// cubes of side 32 and 48 that took 10.1 and 11.4 us per step, against 15.5
// and 16.4 us with runs of at least 8 planes.
static int64_t step4_run_length(int64_t total, int64_t slots, int ncu)
{
    const int64_t rmin = std::max<int64_t>(1, std::min<int64_t>(4, (total + ncu - 1) / ncu));
    return std::max<int64_t>(rmin, (total + slots - 1) / slots);
}

// Whole-step setting for one periodic box, by a cost model of the two work
// orders.  z chunks: rounds of resident workgroups times the planes one item
// streams (its chunk plus the 8-plane start-up of the pipeline).  Equal runs
// (tz 0): the planes of the busiest run plus 8 for every tile column it
// touches, in one round.  Each shape and order has its own cost per plane
// (relative to 32 x 16 lanes in 32-plane chunks), fitted to the measured
// step times of all 20 settings on periodic cubes of side 128, 192, 224,
// 256, 320, 384, 448 and 512: each within 12 % of its mean ratio of time to
// modelled planes, and with them the model picks the fastest measured
// setting on each of those cubes.  Equal runs lose L2 locality, a 1024-lane
// workgroup alone on its CU hides less latency per lane, and 68 x 15 lanes
// trade idle lanes for whole output rows on boxes 64 points wide in x.
static int step4_single(const s4_ctx *ctx, const s4_box &b)
{
    struct Opt {
        int tx, nw, tz, shape;
        double per_plane;
    };
    static const Opt opts[] = {
        {32, 8, 0, 0, 1.368},   {32, 8, 128, 0, 1.004},  {32, 8, 64, 0, 1.028},  {32, 8, 32, 0, 1.015},
        {32, 8, 16, 0, 0.984},  {64, 16, 0, 1, 1.196},   {64, 16, 128, 1, 1.152}, {64, 16, 64, 1, 1.087},
        {64, 16, 32, 1, 1.035}, {64, 16, 16, 1, 1.060},  {32, 16, 0, 2, 1.371},  {32, 16, 128, 2, 1.288},
        {32, 16, 64, 2, 1.361}, {32, 16, 32, 2, 1.166},  {32, 16, 16, 2, 1.125}, {68, 16, 0, 3, 1.295},
        {68, 16, 128, 3, 1.252}, {68, 16, 64, 3, 1.102}, {68, 16, 32, 3, 1.101}, {68, 16, 16, 3, 1.139}};
    int best = cand_index(32, 8, 32, 4);
    {
        // too few tile-planes to give every resident 512-lane workgroup 8
        // planes: equal runs on that shape (a larger workgroup would
        // sit alone on its CU with twice the lanes per plane)
        const Cand &c = cands()[cand_index(32, 8, 0, 4)];
        const int64_t tiles = (int64_t)((b.n[0] + out_tx(c) - 1) / out_tx(c)) * ((b.n[1] + out_ty(c) - 1) / out_ty(c));
        if (cand_fits(c, &b, 1) && tiles * b.n[2] <= 8 * (int64_t)std::max(1, ctx->step4_per[0]) * ctx->ncu)
            return cand_index(32, 8, 0, 4);
    }
    double best_cost = 1e300;
    for (const Opt &o : opts) {
        const int ci = cand_index(o.tx, o.nw, o.tz, 4);
        const Cand &c = cands()[ci];
        if (!cand_fits(c, &b, 1))
            continue;
        const int64_t slots = (int64_t)std::max(1, ctx->step4_per[o.shape]) * ctx->ncu;
        const int64_t nz = b.n[2];
        const int64_t tiles = (int64_t)((b.n[0] + out_tx(c) - 1) / out_tx(c)) * ((b.n[1] + out_ty(c) - 1) / out_ty(c));
        double planes;
        if (o.tz > 0) {
            const int64_t tz = std::min<int64_t>(o.tz, nz);
            const int64_t items = tiles * ((nz + tz - 1) / tz);
            planes = (double)((items + slots - 1) / slots) * (double)(tz + 8);
        } else {
            // the runs step4_run hands out: R planes each (the last one shorter)
            const int64_t total = tiles * nz;
            const int64_t R = step4_run_length(total, slots, ctx->ncu);
            int64_t worst = 0;
            for (int64_t s0 = 0; s0 < total; s0 += R) {
                const int64_t e = std::min(total, s0 + R);
                worst = std::max(worst, (e - s0) + 8 * ((e - 1) / nz - s0 / nz + 1));
            }
            planes = (double)worst;
        }
        const double cost = planes * o.per_plane;
        if (cost < best_cost) {
            best_cost = cost;
            best = ci;
        }
    }
    return best;
}

// Multi-field kernel: workgroups of 32 x 8 lanes (four wavefronts; the
// kernel's two barriers per plane favour many small workgroups per CU) and
// the longest z chunk that gives every CU one item per field.  A launch
// covers several fields (each a range of items of its own), so that is
// several items per CU, of long chunks that pay the 4-plane start-up
// rarely.
static int mixed_heuristic(const s4_ctx *ctx, const s4_box &b)
{
    const int tx = b.n[0] >= 24 ? 32 : 16, nw = 4;
    for (int tz : {0, 64, 32, 16})
        if (items_of(b, {tx, nw, tz, 0, 0}) >= (int64_t)ctx->ncu)
            return cand_index(tx, nw, tz);
    return cand_index(tx, nw, 8);
}

static int heuristic(const s4_ctx *ctx, int op, const s4_box *b, int nbox, int level = 0)
{
    if (op == S4_OP_DERIV_MIXED)
        return mixed_heuristic(ctx, b[0]);
    if (op == S4_OP_WAVE_RHS) {
        // pair-lane tiles (two x points per lane, 128 x 8 points, 32-plane
        // chunks) where the boxes fit them and give every CU two items
        const int pl = cand_index(64, 8, 32, 5);
        int64_t items = 0;
        for (int i = 0; i < nbox; ++i)
            items += items_of(b[i], cands()[pl]);
        if (cand_fits(cands()[pl], b, nbox) && items >= 2 * (int64_t)ctx->ncu)
            return pl;
    }
    if (op != S4_OP_RK4)
        return tile_heuristic(ctx, b, nbox);
    const int whole = cand_index(32, 8, 32, 4);
    if (level != LEVEL_NARROW && cand_fits(cands()[whole], b, nbox))
        return nbox == 1 ? step4_single(ctx, b[0]) : whole;
    double pts = 0, lanes = 0;
    for (int i = 0; i < nbox; ++i) {
        pts += (double)b[i].n[0] * b[i].n[1] * b[i].n[2];
        lanes += (double)((b[i].n[0] + 63) / 64 * 64) * ((b[i].n[1] + 3) / 4 * 4) * b[i].n[2];
    }
    const int tx = pts >= 0.8 * lanes ? 64 : 32, nw = tx == 64 ? 4 : 8;
    const int64_t want = (nbox > 1 ? 8 : 4) * (int64_t)ctx->ncu;
    for (int tz : {64, 32}) {
        int64_t items = 0;
        for (int i = 0; i < nbox; ++i)
            items += items_of(b[i], {tx, nw, tz, 3, 0});
        if (items >= want)
            return cand_index(tx, nw, tz, 3);
    }
    return cand_index(tx, nw, 16, 3);
}

// settings one step away: one parameter moved to its neighbouring value in
// the same kernel set, and the nearest settings of each other kernel set
std::vector<int> Hill::neighbours(int c) const
{
    const Cand &a = cands()[c];
    // (68-point rows sit one step from 64-point ones)
    auto dist = [&](const Cand &e) {
        return std::abs(ord_tx(e.tx) - ord_tx(a.tx)) + std::abs(ord_nw(e.nw) - ord_nw(a.nw)) +
               std::abs(ord_tz(e.tz) - ord_tz(a.tz)) + std::abs(ord_ry(e.ry) - ord_ry(a.ry)) +
               ((e.tx == 68) != (a.tx == 68));
    };
    std::vector<int> out;
    int nearest[6] = {1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30}; // per other kernel set
    for (int d : allowed)
        if (cands()[d].variant != a.variant)
            nearest[cands()[d].variant] = std::min(nearest[cands()[d].variant], dist(cands()[d]));
    for (int d : allowed) {
        if (d == c)
            continue;
        const Cand &e = cands()[d];
        if (e.variant == a.variant ? dist(e) == 1 : dist(e) == nearest[e.variant])
            out.push_back(d);
    }
    return out;
}

static std::vector<int> allowed_cands(int op, const s4_box *b, int nbox, int level = 0)
{
    std::vector<int> v;
    for (int i = 0; i < (int)cands().size(); ++i)
        if (cand_allowed(cands()[i], op, nbox) && cand_fits(cands()[i], b, nbox) &&
            (!level || level_capable(cands()[i], level)))
            v.push_back(i);
    return v;
}

// whether a tuned or loaded choice ci can serve op on these boxes (as a
// level: level-capable candidates only)
static bool cand_valid(int ci, int op, const s4_box *b, int nbox, int level)
{
    if (ci < 0 || ci >= (int)cands().size())
        return false;
    const Cand &c = cands()[ci];
    return cand_allowed(c, op, nbox) && cand_fits(c, b, nbox) && (!level || level_capable(c, level));
}

// setup key of the RK4 steps of a level: the boxes' key, marked, so that a
// level keeps its own choice among the level-capable candidates
static const char *const LEVEL_SUFFIX = "|level";
static const char *const WIDE_LEVEL_SUFFIX = "|level4";

static std::string level_key(const std::string &bkey, int level)
{
    return level == LEVEL_WIDE ? bkey + WIDE_LEVEL_SUFFIX : level ? bkey + LEVEL_SUFFIX : bkey;
}

struct Choice {
    int cand;
    int tuned; // 0 heuristic or forced, 1 from s4_tune, 2 on-line
    std::string key;
};

static void online_harvest(OnlineSetup &st);

// The settings the on-line search may visit: those the op can run, less
// those whose launches hand fewer work items than a quarter of the CUs
// while another setting gives every CU one (with most of the device idle
// they cannot win, and one call on them costs many: on a 128^3 box a
// whole-box z chunk of 64 x 8 tiles runs 32 workgroups and takes ten times
// the best setting's time).  Whole steps in equal runs count their runs.
static std::vector<int> online_allowed(const s4_ctx *ctx, int op, const s4_box *b, int nbox, int level)
{
    const std::vector<int> all = allowed_cands(op, b, nbox, level);
    auto work = [&](int ci) {
        const Cand &c = cands()[ci];
        if (c.variant == 4 && c.tz == 0 && nbox == 1) {
            const int64_t total = items_of(b[0], c); // tile columns x one whole-box chunk
            const int64_t planes = total * b[0].n[2];
            const int shape = c.tx == 32 ? (c.nw == 8 ? 0 : 2) : c.tx == 64 ? 1 : 3;
            const int64_t per = std::max(1, ctx->step4_per[shape]);
            const int64_t R = step4_run_length(planes, per * ctx->ncu, ctx->ncu);
            return (planes + R - 1) / R;
        }
        int64_t n = 0;
        for (int i = 0; i < nbox; ++i)
            n += items_of(b[i], c);
        return n;
    };
    int64_t most = 0;
    for (int ci : all)
        most = std::max(most, work(ci));
    if (most < ctx->ncu)
        return all;
    std::vector<int> v;
    for (int ci : all)
        if (4 * work(ci) >= ctx->ncu)
            v.push_back(ci);
    return v;
}

// caller holds ctx->mu
static OnlineSetup &online_setup(s4_ctx *ctx, const std::string &key, int op, const s4_box *b, int nbox,
                                 int level)
{
    auto it = ctx->online_state.find(key);
    if (it != ctx->online_state.end())
        return it->second;
    OnlineSetup &st = ctx->online_state[key];
    st.hill.allowed = online_allowed(ctx, op, b, nbox, level);
    auto t = ctx->tuned.find(key);
    st.hill.start = t != ctx->tuned.end() && cand_valid(t->second, op, b, nbox, level)
                        ? t->second
                        : heuristic(ctx, op, b, nbox, level);
    st.hill.restart_prob = ctx->restart_prob;
    st.hill.rng ^= ctx->seed * 0xD1342543DE82EF95ull + std::hash<std::string>()(key);
    return st;
}

// peek: report the choice without advancing the on-line tuner.  level: the
// RK4 steps of a level (LEVEL_NARROW or LEVEL_WIDE: its own setup key;
// candidates capable of that level only, a forced or tuned choice of the
// boxes is taken if it is one)
// c2: the call passes c^2 (its own setup; a choice forced without c^2
// applies to it too, a tuned one does not)
static Choice choose(s4_ctx *ctx, int op, const s4_box *b, int nbox, bool peek = false, int level = 0,
                     bool c2 = false)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    const std::string bkey = setup_key(ctx, op, b, nbox, c2);
    const std::string key = level_key(bkey, level);
    auto ok = [&](int c) { return !level || level_capable(cands()[c], level); };
    for (const std::string &k : {bkey, setup_key(ctx, op, b, nbox)}) {
        auto f = ctx->forced.find(k);
        if (f != ctx->forced.end() && ok(f->second))
            return {f->second, 0, key};
    }
    if (ctx->online) {
        OnlineSetup &st = online_setup(ctx, key, op, b, nbox, level);
        online_harvest(st);
        if (peek)
            return {st.hill.best >= 0 ? st.hill.best : st.hill.start, 2, key};
        return {st.hill.next(), 2, key};
    }
    for (const std::string &k : {key, bkey}) {
        auto t = ctx->tuned.find(k);
        if (t != ctx->tuned.end() && cand_valid(t->second, op, b, nbox, level))
            return {t->second, 1, key};
    }
    return {heuristic(ctx, op, b, nbox, level), 0, key};
}

// Timing of one call for the on-line tuner: events around the call's
// launches on its stream, read back lazily by a later call of the same setup
// (never waited for).
static void online_harvest(OnlineSetup &st)
{
    while (!st.pending.empty()) {
        OnlinePending &p = st.pending.front();
        if (hipEventQuery(p.b) != hipSuccess)
            break;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess && p.units > 0)
            st.hill.measured(p.cand, ms / p.units);
        st.pool.push_back(p.a);
        st.pool.push_back(p.b);
        st.pending.pop_front();
    }
    (void)hipGetLastError();
}

struct OnlineTimer;
// the timer of the call running on this thread, if any (graph_run restarts it
// after capturing a new graph, so a setting's first call is timed on its
// launches and not on the one-off capture)
static thread_local OnlineTimer *g_timer = nullptr;

struct OnlineTimer {
    s4_ctx *ctx = nullptr;
    std::string key;
    int cand = -1;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = nullptr;

    void restart()
    {
        if (ctx && hipEventRecord(a, s) != hipSuccess)
            (void)hipGetLastError();
    }
    ~OnlineTimer()
    {
        if (g_timer == this)
            g_timer = nullptr;
        if (ctx) { // never stopped (the call failed): return the events
            std::lock_guard<std::mutex> lk(ctx->mu);
            OnlineSetup &st = ctx->online_state[key];
            st.pool.push_back(a);
            st.pool.push_back(b);
        }
    }

    OnlineTimer(s4_ctx *c, const Choice &ch, hipStream_t stream)
    {
        if (ch.tuned != 2)
            return;
        std::lock_guard<std::mutex> lk(c->mu);
        OnlineSetup &st = c->online_state[ch.key];
        if (st.pending.size() > 64) // results not coming back: stop adding timers
            return;
        for (hipEvent_t *e : {&a, &b}) {
            if (!st.pool.empty()) {
                *e = st.pool.back();
                st.pool.pop_back();
            } else if (hipEventCreate(e) != hipSuccess) {
                *e = nullptr;
            }
        }
        if (!a || !b || hipEventRecord(a, stream) != hipSuccess) {
            for (hipEvent_t e : {a, b})
                if (e)
                    st.pool.push_back(e);
            a = b = nullptr;
            (void)hipGetLastError();
            return;
        }
        ctx = c;
        key = ch.key;
        cand = ch.cand;
        s = stream;
        g_timer = this;
    }
    // after the call's launches; units: what one time is divided by (RK4 steps)
    void stop(double units)
    {
        if (!ctx)
            return;
        std::lock_guard<std::mutex> lk(ctx->mu);
        OnlineSetup &st = ctx->online_state[key];
        if (hipEventRecord(b, s) != hipSuccess) {
            st.pool.push_back(a);
            st.pool.push_back(b);
            (void)hipGetLastError();
        } else {
            st.pending.push_back({a, b, cand, units});
        }
        ctx = nullptr;
        if (g_timer == this)
            g_timer = nullptr;
    }
};

// ---------------------------------------------------------------------------
// validation (host only, before anything is launched)

static int64_t box_elems(const s4_box &b)
{
    return b.stride[2] * ((int64_t)b.n[2] + 2 * b.ghost);
}

static size_t round256(size_t x)
{
    return (x + 255) & ~(size_t)255;
}

// Workspace fields copy the box's strides.  Each starts `field_shift` bytes
// past a 256-byte boundary so that its interior rows start on 128-byte lines
// whenever the strides are multiples of 16 elements (the padded layout).
static size_t field_shift(const s4_box &b)
{
    return (size_t)((16 - b.ghost % 16) % 16) * sizeof(double);
}

static size_t field_bytes(const s4_box &b)
{
    return round256((size_t)box_elems(b) * sizeof(double) + field_shift(b));
}

static double *ws_field(char *base, const s4_box &b)
{
    return (double *)(base + field_shift(b));
}

static int check_box(const s4_box &b, int i, int op)
{
    for (int a = 0; a < 3; ++a) {
        if (b.n[a] < 1)
            return fail(S4_EINVAL, "box %d: n[%d] = %d < 1", i, a, b.n[a]);
        if (b.n[a] > (1 << 24))
            return fail(S4_EINVAL, "box %d: n[%d] = %d too large", i, a, b.n[a]);
        if (!(std::isfinite(b.dx[a]) && b.dx[a] > 0.0))
            return fail(S4_EINVAL, "box %d: dx[%d] must be finite and > 0", i, a);
    }
    if (b.ghost < 2)
        return fail(S4_EGHOST, "box %d: ghost width %d < 2 (stencil radius)", i, b.ghost);
    if (b.ghost > 64)
        return fail(S4_EGHOST, "box %d: ghost width %d > 64", i, b.ghost);
    if (b.stride[0] != 1)
        return fail(S4_ELAYOUT, "box %d: stride[0] must be 1", i);
    if (b.stride[1] < (int64_t)b.n[0] + 2 * b.ghost)
        return fail(S4_ELAYOUT, "box %d: stride[1] %lld < n[0]+2g", i, (long long)b.stride[1]);
    if (b.stride[2] / b.stride[1] < (int64_t)b.n[1] + 2 * b.ghost)
        return fail(S4_ELAYOUT, "box %d: stride[2] %lld < stride[1]*(n[1]+2g)", i, (long long)b.stride[2]);
    if (b.stride[2] > ((int64_t)1 << 40) || box_elems(b) > ((int64_t)1 << 42))
        return fail(S4_ELAYOUT, "box %d: array too large", i);
    if (op == S4_OP_FILL)
        for (int a = 0; a < 3; ++a)
            if (b.n[a] < b.ghost)
                return fail(S4_EGHOST, "box %d: periodic fill needs n[%d] >= ghost", i, a);
    for (const Cand &c : cands())
        if (items_of(b, c) > 0x3fffffff)
            return fail(S4_EINVAL, "box %d: too many tiles", i);
    return S4_OK;
}

static int check_boxes(const s4_box *b, int nbox, int op)
{
    if (!b)
        return fail(S4_EINVAL, "box array is NULL");
    if (nbox <= 0)
        return fail(S4_EINVAL, "nbox = %d <= 0", nbox);
    if (nbox > (1 << 20))
        return fail(S4_EINVAL, "nbox = %d too large", nbox);
    for (int i = 0; i < nbox; ++i) {
        int r = check_box(b[i], i, op);
        if (r)
            return r;
    }
    return S4_OK;
}

static int check_ptr(const void *p, const char *what, int i, bool may_be_null = false)
{
    if (!p)
        return may_be_null ? S4_OK : fail(S4_EINVAL, "%s[%d] is NULL", what, i);
    if ((uintptr_t)p & 7)
        return fail(S4_ELAYOUT, "%s[%d] is not 8-byte aligned", what, i);
    return S4_OK;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b)
        return false;
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

struct Range {
    const void *p;
    size_t n;
    const char *what;
    int box;
};

// every pair (written, other) must be disjoint
static int check_disjoint(const std::vector<Range> &written, const std::vector<Range> &all)
{
    for (const Range &w : written)
        for (const Range &o : all) {
            if (&w == &o || (w.p == o.p && w.what == o.what && w.box == o.box))
                continue;
            if (overlap(w.p, w.n, o.p, o.n))
                return fail(S4_EALIAS, "%s[%d] overlaps %s[%d]", w.what, w.box, o.what, o.box);
        }
    return S4_OK;
}

// ---------------------------------------------------------------------------
// device boxes

static DevBox devbox(const s4_box &b, const Cand &c)
{
    DevBox D;
    memset(&D, 0, sizeof D);
    for (int a = 0; a < 3; ++a)
        D.n[a] = b.n[a];
    D.g = b.ghost;
    D.sy = b.stride[1];
    D.sz = b.stride[2];
    D.cx = 1.0 / (12.0 * b.dx[0] * b.dx[0]);
    D.cy = 1.0 / (12.0 * b.dx[1] * b.dx[1]);
    D.cz = 1.0 / (12.0 * b.dx[2] * b.dx[2]);
    D.c0 = -30.0 * (D.cx + D.cy + D.cz);
    const int tx = out_tx(c), ty = out_ty(c);
    D.tz = c.tz > 0 ? std::min(c.tz, b.n[2]) : b.n[2];
    D.tiles[0] = (b.n[0] + tx - 1) / tx;
    D.tiles[1] = (b.n[1] + ty - 1) / ty;
    D.tiles[2] = (b.n[2] + D.tz - 1) / D.tz;
    return D;
}

static int64_t dev_items(const DevBox &D)
{
    return (int64_t)D.tiles[0] * D.tiles[1] * D.tiles[2];
}

static int launch_one(s4_ctx *ctx, int op, const Cand &c, const DevBox &D, const StageCoef &K, hipStream_t s,
                      bool ghosted = false)
{
    if (c.variant == 5) {
        // pair-lane tiles need 16-byte aligned interior rows in every field;
        // otherwise the same shape on the one-point tiles (same arithmetic)
        auto al = [&](const double *p) { return !p || ((uintptr_t)(p + D.g) & 15) == 0; };
        if (op == OP_RHS && al(D.in) && al(D.p[0]) && al(D.q[0])) {
            hipError_t e = launch_pairs_rhs(c.tx, c.nw, D, (int)dev_items(D), ctx->nxcd, s);
            return e == hipSuccess ? S4_OK : hip_fail(e, "stencil launch");
        }
        const Cand &c0 = cands()[cand_index(c.tx, c.nw, c.tz)];
        DevBox D0 = D;
        D0.tiles[0] = (D.n[0] + c0.tx - 1) / c0.tx;
        D0.tiles[1] = (D.n[1] + tile_ty(c0) - 1) / tile_ty(c0);
        return launch_one(ctx, op, c0, D0, K, s, ghosted);
    }
    const int64_t items = dev_items(D);
    hipError_t e = c.variant == 2 ? launch_rows_single(op, c.tx / 64, c.ry, D, K, (int)items, ctx->nxcd, s, ghosted)
                                  : launch_tiles_single(op, c.tx, c.nw, D, K, (int)items, ctx->nxcd, s, ghosted);
    if (e != hipSuccess)
        return hip_fail(e, "stencil launch");
    return S4_OK;
}

static int persistent_grid(s4_ctx *ctx, int op, const Cand &c, int64_t nitems, bool ghosted = false)
{
    int per = c.variant == 2 ? max_blocks_rows(op, c.tx / 64, c.ry, ghosted) : max_blocks_per_cu(op, c.tx, c.nw, ghosted);
    if (per <= 0)
        per = 2;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)per * ctx->ncu));
}

// Copy a box table (and its zeroed item counters) into the caller's
// workspace.  Done on every call that needs it: the workspace belongs to the
// caller between calls, so nothing found there is trusted.  The stream is
// synchronised so the host staging bytes may be released.
static int upload_table(void *dst, const std::vector<char> &bytes, hipStream_t s)
{
    S4_HIP(hipMemcpyAsync(dst, bytes.data(), bytes.size(), hipMemcpyHostToDevice, s));
    S4_HIP(hipStreamSynchronize(s));
    return S4_OK;
}

// ---------------------------------------------------------------------------
// workspace layouts

static const int RK4_FIELDS = 6;   // Ua Ub Ra Rb AccU AccR
static const int ADJ_FIELDS = 6;   // U3 R3 KR2 KR1 AccU AccR
static const int TUNE_SETS = 7;    // independent buffer sets the tuner rotates through

static size_t rk4_fields_bytes(const s4_box *b, int nbox)
{
    size_t t = 0;
    for (int i = 0; i < nbox; ++i)
        t += RK4_FIELDS * field_bytes(b[i]);
    return t;
}

// counters of the four work queues of one batched RK4 step (one per stage
// or stage pair, each QUEUE_INTS ints)
static const size_t QUEUE_BYTES = 4 * QUEUE_INTS * sizeof(int);

static size_t rk4_table_bytes(int nbox)
{
    return round256(4 * (size_t)nbox * sizeof(DevBox)) + QUEUE_BYTES; // 4 stage tables + queue counters
}

// work queue `slot` (0..3) of a batched step over nitems items, one range per XCD
static ItemQueue step_queue(const s4_ctx *ctx, int *counters, int slot, int64_t nitems)
{
    return ItemQueue{counters + QUEUE_INTS * slot, (int)nitems, std::max(1, std::min(ctx->nxcd, QUEUE_INTS - 1))};
}

// ---------------------------------------------------------------------------
// API

extern "C" {

const char *s4_last_error(void)
{
    return g_err.c_str();
}

int s4_check_boxes(const s4_box *b, int nbox, int op)
{
    if (op < S4_OP_FILL || op > S4_OP_ADJOINT_STEP)
        return fail(S4_EINVAL, "unknown op %d", op);
    int r = check_boxes(b, nbox, op);
    if (r)
        return r;
    if ((op == S4_OP_ADJOINT_STEP || op == S4_OP_DERIV_MIXED) && nbox != 1)
        return fail(S4_EINVAL, "op %d takes one box", op);
    return S4_OK;
}

int s4_workspace_size(const s4_box *b, int nbox, int op, int mode, size_t *bytes)
{
    if (!bytes)
        return fail(S4_EINVAL, "bytes is NULL");
    int r = s4_check_boxes(b, nbox, op);
    if (r)
        return r;
    if (op == S4_OP_RK4) {
        if (mode < S4_PERBOX || mode > S4_GRAPH)
            return fail(S4_EINVAL, "unknown mode %d", mode);
        *bytes = rk4_fields_bytes(b, nbox) + rk4_table_bytes(nbox);
    } else if (op == S4_OP_ADJOINT_STEP) {
        *bytes = ADJ_FIELDS * field_bytes(b[0]);
    } else {
        *bytes = 0;
    }
    return S4_OK;
}

// fields of tuning scratch per box: the buffers one timed call of the op
// touches, in as many independent sets as the tuner rotates through
static int tune_fields(int op, bool c2 = false)
{
    switch (op) {
    case S4_OP_RK4: return 2 + RK4_FIELDS + (c2 ? 1 : 0); // u, rho + the RK4 workspace (+ c^2)
    case S4_OP_WAVE_RHS: return 2 * TUNE_SETS;           // (u, rho_t) per set
    case S4_OP_ADJOINT_RHS: return 5 * 2;                // (lu, lrho, c2, out_u, out_rho) x 2 sets
    case S4_OP_ADJOINT_STEP: return 6 + ADJ_FIELDS;      // u_n rho_n c2 lam_u lam_rho c2_bar + workspace
    case S4_OP_DERIV_MIXED: return 2 * TUNE_SETS;        // TUNE_SETS fields in, as many out
    default: return 0;
    }
}

int s4_tune_scratch_size(const s4_box *b, int nbox, int op, size_t *bytes)
{
    if (!bytes)
        return fail(S4_EINVAL, "bytes is NULL");
    bool c2 = false;
    int r = split_op(op, c2);
    if (r || (r = s4_check_boxes(b, nbox, op)))
        return r;
    size_t t = 0;
    for (int i = 0; i < nbox; ++i)
        t += (size_t)tune_fields(op, c2) * field_bytes(b[i]);
    *bytes = t + rk4_table_bytes(nbox);
    return S4_OK;
}

static void load_cache(s4_ctx *ctx);

int s4_create(int device, s4_ctx **out)
{
    if (!out)
        return fail(S4_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    S4_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(S4_EINVAL, "device %d out of range (%d devices)", device, ndev);
    S4_HIP(hipSetDevice(device));
    hipDeviceProp_t p;
    S4_HIP(hipGetDeviceProperties(&p, device));
    s4_ctx *c = new s4_ctx;
    c->device = device;
    c->ncu = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
    c->name = p.gcnArchName;
    {
        size_t cut = c->name.find(':');
        if (cut != std::string::npos)
            c->name = c->name.substr(0, cut);
    }
    {
        const int shapes[4][2] = {{32, 8}, {64, 16}, {32, 16}, {68, 16}};
        for (int k = 0; k < 4; ++k) {
            const int per = max_blocks_step4(shapes[k][0], shapes[k][1]);
            if (per > 0)
                c->step4_per[k] = per;
        }
    }
    int nx = 0;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, device) == hipSuccess && nx > 0)
        c->nxcd = nx;
    else
        c->nxcd = (c->name.rfind("gfx94", 0) == 0 || c->name.rfind("gfx95", 0) == 0) ? 8 : 1;
    (void)hipGetLastError();
    {
        // the device address of the no-allocation scratch array, once per device
        hipError_t e = noalloc_scratch(&c->scratch);
        if (e != hipSuccess) {
            c->scratch = nullptr;
            c->scratch_err = hipGetErrorString(e);
            (void)hipGetLastError();
        }
    }
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(S4_EDEVICE, "cannot create the capture stream");
    }
    const char *cp = getenv("S4_TUNE_CACHE");
    if (cp && *cp) {
        c->cache_path = cp;
        load_cache(c);
    }
    const char *tm = getenv("S4_TUNE");
    if (tm && std::string(tm) == "online")
        c->online = true;
    *out = c;
    return S4_OK;
}

int s4_set_online_tuning(s4_ctx *ctx, int enable, double restart_prob, uint64_t seed)
{
    if (!ctx)
        return fail(S4_EINVAL, "ctx is NULL");
    if (!(restart_prob >= 0.0 && restart_prob <= 1.0))
        return fail(S4_EINVAL, "restart_prob must be in [0, 1]");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->online = enable != 0;
    ctx->restart_prob = restart_prob;
    ctx->seed = seed;
    for (auto &kv : ctx->online_state)
        kv.second.hill.restart_prob = restart_prob;
    return S4_OK;
}

int s4_online_simulate(int op, const s4_box *b, int nbox, const double *cost, int ncost, double noise,
                       double restart_prob, uint64_t seed, int lag, int ncalls, int *trace)
{
    int r = s4_check_boxes(b, nbox, op);
    if (r)
        return r;
    if (!cost || !trace || ncalls < 0 || lag < 0 || lag > 64)
        return fail(S4_EINVAL, "bad simulation arguments");
    if (ncost != (int)cands().size())
        return fail(S4_EINVAL, "cost needs one entry per candidate (%d)", (int)cands().size());
    if (!(noise >= 0.0 && noise < 1.0) || !(restart_prob >= 0.0 && restart_prob <= 1.0))
        return fail(S4_EINVAL, "noise in [0, 1) and restart_prob in [0, 1]");
    s4_ctx sim; // host-only: the heuristic needs the CU count only
    Hill h;
    h.allowed = online_allowed(&sim, op, b, nbox, 0);
    h.start = heuristic(&sim, op, b, nbox);
    h.restart_prob = restart_prob;
    h.rng ^= seed * 0xD1342543DE82EF95ull;
    Hill noise_rng;
    noise_rng.rng = seed + 12345;
    std::deque<std::pair<int, double>> inflight; // timings arrive `lag` calls later
    for (int i = 0; i < ncalls; ++i) {
        const int c = h.next();
        trace[i] = c;
        inflight.push_back({c, cost[c] * (1.0 + noise * (2.0 * noise_rng.uniform() - 1.0))});
        if ((int)inflight.size() > lag) {
            h.measured(inflight.front().first, inflight.front().second);
            inflight.pop_front();
        }
    }
    return S4_OK;
}

void s4_destroy(s4_ctx *ctx)
{
    if (!ctx)
        return;
    for (auto &kv : ctx->online_state) {
        for (auto &p : kv.second.pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipEvent_t e : kv.second.pool)
            (void)hipEventDestroy(e);
    }
    for (auto &kv : ctx->graphs)
        graph_free(kv.second);
    if (ctx->cap)
        (void)hipStreamDestroy(ctx->cap);
    delete ctx;
}

static void fill_choice(int op, int nbox, const Choice &ch, int out[8]);
static int level_check(const s4_level *L);

// LEVEL_WIDE when the level's exchange fills the full ghost shell of width
// 4 or more and every box has 4 or more ghost layers and z planes below
// 2 GiB (whole RK4 steps then run on it), else LEVEL_NARROW
static int level_kind(const s4_level *L)
{
    if (L->width < 4 || L->shape != S4_SYNC_FULL)
        return LEVEL_NARROW;
    for (const s4_box &b : L->boxes)
        if (b.ghost < 4 || b.stride[2] * 8 >= (int64_t)0x80000000)
            return LEVEL_NARROW;
    return LEVEL_WIDE;
}

int s4_get_choice(s4_ctx *ctx, int op, const s4_box *b, int nbox, int out[8])
{
    if (!ctx || !out)
        return fail(S4_EINVAL, "NULL argument");
    bool c2 = false;
    int r = split_op(op, c2);
    if (r || (r = s4_check_boxes(b, nbox, op)))
        return r;
    fill_choice(op, nbox, choose(ctx, op, b, nbox, true, false, c2), out);
    return S4_OK;
}

int s4_level_choice(s4_ctx *ctx, const s4_level *L, int out[8])
{
    if (!ctx || !out)
        return fail(S4_EINVAL, "NULL argument");
    int r = level_check(L);
    if (r)
        return r;
    const int nbox = (int)L->boxes.size();
    fill_choice(S4_OP_RK4, nbox, choose(ctx, S4_OP_RK4, L->boxes.data(), nbox, true, level_kind(L)), out);
    return S4_OK;
}

static void fill_choice(int op, int nbox, const Choice &ch, int out[8])
{
    const Cand &c = cands()[ch.cand];
    // 100, 101: RK4 stage pairs (widened tile, per-tap); 102: whole RK4 steps;
    // 200 + op: the op's kernels on the row-register traversal
    out[0] = c.variant == 1   ? 100
             : c.variant == 3 ? 101
             : c.variant == 4 ? 102
             : c.variant == 2 ? 200 + kernel_op(op)
             : c.variant == 5 ? 300 + kernel_op(op)
                              : kernel_op(op);
    out[1] = c.variant == 5 ? out_tx(c) : c.tx;
    out[2] = tile_ty(c);
    out[3] = c.tz;
    out[4] = c.nw * 64;
    out[5] = ch.tuned;
    out[6] = ch.cand;
    int end = 0; // one past the last candidate this op may use on nbox boxes
    for (int i = 0; i < (int)cands().size(); ++i)
        if (cand_allowed(cands()[i], op, nbox))
            end = i + 1;
    out[7] = end;
}

int s4_set_choice(s4_ctx *ctx, int op, const s4_box *b, int nbox, int candidate)
{
    if (!ctx)
        return fail(S4_EINVAL, "ctx is NULL");
    bool c2 = false;
    int r = split_op(op, c2);
    if (r || (r = s4_check_boxes(b, nbox, op)))
        return r;
    if (candidate >= (int)cands().size() || candidate < -1)
        return fail(S4_EINVAL, "candidate %d out of range", candidate);
    if (candidate >= 0 && !cand_allowed(cands()[candidate], op, nbox))
        return fail(S4_ENOTSUP, "candidate %d (kernel set %d) does not apply to op %d on %d boxes", candidate,
                    cands()[candidate].variant, op, nbox);
    if (candidate >= 0 && !cand_fits(cands()[candidate], b, nbox))
        return fail(S4_ENOTSUP,
                    "candidate %d does not fit these boxes (whole RK4 steps: z planes below 2 GiB; pair-lane "
                    "tiles: even n[0] and strides)",
                    candidate);
    std::lock_guard<std::mutex> lk(ctx->mu);
    const std::string key = setup_key(ctx, op, b, nbox, c2);
    if (candidate < 0)
        ctx->forced.erase(key);
    else
        ctx->forced[key] = candidate;
    return S4_OK;
}

int s4_fill_ghosts_periodic(s4_ctx *ctx, const s4_box *b, int nbox, double *const *f, void *stream)
{
    if (!ctx || !f)
        return fail(S4_EINVAL, "NULL argument");
    int r = check_boxes(b, nbox, S4_OP_FILL);
    if (r)
        return r;
    for (int i = 0; i < nbox; ++i)
        if ((r = check_ptr(f[i], "f", i)))
            return r;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < nbox; ++i) {
        DevBox D = devbox(b[i], cands()[0]);
        D.q[0] = f[i];
        hipError_t e = launch_fill(D, s);
        if (e != hipSuccess)
            return hip_fail(e, "ghost fill launch");
    }
    return S4_OK;
}

int s4_wave_rhs(s4_ctx *ctx, const s4_box *b, int nbox, const double *const *u, const double *const *c2,
                double *const *rho_t, void *stream)
{
    if (!ctx || !u || !rho_t)
        return fail(S4_EINVAL, "NULL argument");
    int r = check_boxes(b, nbox, S4_OP_WAVE_RHS);
    if (r)
        return r;
    std::vector<Range> wr, all;
    for (int i = 0; i < nbox; ++i) {
        if ((r = check_ptr(u[i], "u", i)) || (r = check_ptr(rho_t[i], "rho_t", i)) ||
            (r = check_ptr(c2 ? c2[i] : nullptr, "c2", i, true)))
            return r;
        const size_t n = (size_t)box_elems(b[i]) * 8;
        wr.push_back({rho_t[i], n, "rho_t", i});
        all.push_back({u[i], n, "u", i});
        if (c2 && c2[i])
            all.push_back({c2[i], n, "c2", i});
    }
    for (auto &w : wr)
        all.push_back(w);
    if ((r = check_disjoint(wr, all)))
        return r;
    const Choice ch = choose(ctx, S4_OP_WAVE_RHS, b, nbox);
    const Cand &c = cands()[ch.cand];
    OnlineTimer tm(ctx, ch, (hipStream_t)stream);
    StageCoef K{};
    K.scale = 1.0;
    for (int i = 0; i < nbox; ++i) {
        DevBox D = devbox(b[i], c);
        D.in = u[i];
        D.p[0] = c2 ? c2[i] : nullptr;
        D.q[0] = rho_t[i];
        if ((r = launch_one(ctx, OP_RHS, c, D, K, (hipStream_t)stream)))
            return r;
    }
    tm.stop(1.0);
    return S4_OK;
}

static MixArgs mix_args(const s4_box &b, const Cand &c, const double A[9])
{
    MixArgs M;
    memset(&M, 0, sizeof M);
    M.B = devbox(b, c);
    M.items = (int)dev_items(M.B);
    M.a[0] = A[0];
    M.a[1] = A[4];
    M.a[2] = A[8];
    M.a[3] = A[1] + A[3];
    M.a[4] = A[2] + A[6];
    M.a[5] = A[5] + A[7];
    for (int a = 0; a < 3; ++a) {
        M.d1[a] = 1.0 / (12.0 * b.dx[a]);
        M.d2[a] = 1.0 / (12.0 * b.dx[a] * b.dx[a]);
    }
    return M;
}

static int launch_mixed_fields(s4_ctx *ctx, const Cand &c, MixArgs M, int nfield, const double *const *g,
                               double *const *out, hipStream_t s)
{
    for (int f0 = 0; f0 < nfield; f0 += 8) {
        const int nf = std::min(8, nfield - f0);
        for (int k = 0; k < 8; ++k) {
            M.f[k] = k < nf ? g[f0 + k] : nullptr;
            M.out[k] = k < nf ? out[f0 + k] : nullptr;
        }
        hipError_t e = launch_mixed(c.tx, c.nw, M, nf, ctx->nxcd, s);
        if (e != hipSuccess)
            return hip_fail(e, "mixed-derivative launch");
    }
    return S4_OK;
}

int s4_deriv_mixed(s4_ctx *ctx, const s4_box *b, int nfield, const double *const *g, const double A[9],
                   double *const *out, void *stream)
{
    if (!ctx || !g || !out || !A)
        return fail(S4_EINVAL, "NULL argument");
    int r = check_boxes(b, 1, S4_OP_DERIV_MIXED);
    if (r)
        return r;
    if (nfield < 1 || nfield > (1 << 16))
        return fail(S4_EINVAL, "nfield = %d out of range", nfield);
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(A[k]))
            return fail(S4_EINVAL, "A[%d] is not finite", k);
    std::vector<Range> wr, all;
    const size_t n = (size_t)box_elems(b[0]) * 8;
    for (int k = 0; k < nfield; ++k) {
        if ((r = check_ptr(g[k], "g", k)) || (r = check_ptr(out[k], "out", k)))
            return r;
        wr.push_back({out[k], n, "out", k});
        all.push_back({g[k], n, "g", k});
    }
    for (auto &w : wr)
        all.push_back(w);
    if ((r = check_disjoint(wr, all)))
        return r;
    const Choice ch = choose(ctx, S4_OP_DERIV_MIXED, b, 1);
    const Cand &c = cands()[ch.cand];
    const MixArgs M = mix_args(b[0], c, A);
    if ((int64_t)M.items * 8 > 0x7fffffff)
        return fail(S4_EINVAL, "too many work items");
    OnlineTimer tm(ctx, ch, (hipStream_t)stream);
    if ((r = launch_mixed_fields(ctx, c, M, nfield, g, out, (hipStream_t)stream)))
        return r;
    tm.stop((double)nfield);
    return S4_OK;
}

// RK4 stage tables for all boxes: stage s reads u_s (stencil) and writes the
// next stage input; the accumulators hold y_n + sum_{r<=s} b_r k_r.  The
// step reads y_n from (uin, rin) and its last stage writes (uout, rout).
static void rk4_tables_io(const s4_box *b, int nbox, const double *const *uin, const double *const *rin,
                          double *const *uout, double *const *rout, const double *const *c2, char *ws,
                          const Cand &c, std::vector<DevBox> &tab);

static void rk4_tables(const s4_box *b, int nbox, double *const *u, double *const *rho,
                       const double *const *c2, char *ws, const Cand &c, std::vector<DevBox> &tab)
{
    rk4_tables_io(b, nbox, u, rho, u, rho, c2, ws, c, tab);
}

static void rk4_tables_io(const s4_box *b, int nbox, const double *const *uin, const double *const *rin,
                          double *const *uout, double *const *rout, const double *const *c2, char *ws,
                          const Cand &c, std::vector<DevBox> &tab)
{
    tab.assign(4 * (size_t)nbox, DevBox{});
    size_t off = 0;
    int item0 = 0;
    for (int i = 0; i < nbox; ++i) {
        const size_t fb = field_bytes(b[i]);
        double *F[RK4_FIELDS];
        for (int k = 0; k < RK4_FIELDS; ++k)
            F[k] = ws_field(ws + off + k * fb, b[i]);
        off += RK4_FIELDS * fb;
        double *Ua = F[0], *Ub = F[1], *Ra = F[2], *Rb = F[3], *AU = F[4], *AR = F[5];
        const double *in_[4] = {uin[i], Ua, Ub, Ua};
        const double *rs_[4] = {rin[i], Ra, Rb, Ra};
        double *uo_[4] = {Ua, Ub, Ua, uout[i]};
        double *ro_[4] = {Ra, Rb, Ra, rout[i]};
        DevBox D = devbox(b[i], c);
        D.item0 = item0;
        item0 += (int)dev_items(D);
        for (int s = 0; s < 4; ++s) {
            DevBox E = D;
            E.in = in_[s];
            E.p[0] = rs_[s];
            E.p[1] = uin[i];
            E.p[2] = rin[i];
            E.p[3] = AU;
            E.p[4] = AR;
            E.p[5] = c2 ? c2[i] : nullptr;
            E.q[0] = uo_[s];
            E.q[1] = ro_[s];
            E.q[2] = AU;
            E.q[3] = AR;
            tab[(size_t)s * nbox + i] = E;
        }
    }
}

static StageCoef rk4_coef(int s, double dt)
{
    static const double A[4] = {0.5, 0.5, 1.0, 0.0};
    static const double B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    StageCoef K{};
    K.stage = s + 1;
    K.a = A[s] * dt;
    K.b = B[s] * dt;
    K.scale = 1.0;
    return K;
}

// Ghost exchange run before every stage of a level's RK4 step: the device
// piece table and one table of per-box stage-input pointers per stage.
struct SyncArgs {
    const SyncPiece *P;
    const int *W; // piece of each workgroup
    int nblocks;
    double *const *F; // 4 * nbox entries, stage-major
};

// launch the four stages of one RK4 step (batched: nbox > 1 and table in ws);
// with sy, each stage first exchanges its input's ghosts and then reads them
static int rk4_step(s4_ctx *ctx, const Cand &c, const std::vector<DevBox> &tab, int nbox, bool batched,
                    DevBox *dtab, int *counters, int64_t nitems, double dt, hipStream_t s,
                    const SyncArgs *sy = nullptr)
{
    const bool gh = sy != nullptr;
    for (int st = 0; st < 4; ++st) {
        const StageCoef K = rk4_coef(st, dt);
        if (sy) {
            hipError_t e = launch_sync(sy->P, sy->W, sy->F + (size_t)st * nbox, 1, nbox, sy->nblocks, s);
            if (e != hipSuccess)
                return hip_fail(e, "ghost exchange launch");
        }
        if (batched) {
            const int grid = persistent_grid(ctx, OP_STAGE, c, nitems, gh);
            hipError_t e =
                c.variant == 2
                    ? launch_rows_batched(OP_STAGE, c.tx / 64, c.ry, dtab + (size_t)st * nbox, nbox,
                                          step_queue(ctx, counters, st, nitems), grid, K, s, gh)
                    : launch_tiles_batched(OP_STAGE, c.tx, c.nw, dtab + (size_t)st * nbox, nbox,
                                           step_queue(ctx, counters, st, nitems), grid, K, s, gh);
            if (e != hipSuccess)
                return hip_fail(e, "batched stage launch");
        } else {
            for (int i = 0; i < nbox; ++i) {
                int r = launch_one(ctx, OP_STAGE, c, tab[(size_t)st * nbox + i], K, s, gh);
                if (r)
                    return r;
            }
        }
    }
    return S4_OK;
}

// Fused RK4 on one box.  With stage pairs one step is two launches: pair 0
// reads y_n = (ui, ri) and writes y_3 (U3, R3) and the running sum (AU, AR);
// pair 1 reads them and writes y_{n+1} to (uo, ro).  A whole-step kernel
// (variant 4) reads y_n and writes y_{n+1} in one launch.  Steps alternate
// between the caller's state and a ping-pong copy in the workspace, so an
// even number of steps ends in the caller's buffers.
struct PairFields {
    double *U3, *R3, *Up, *Rp, *AU, *AR;
};

static PairFields pair_fields(const s4_box &b, char *ws)
{
    const size_t fb = field_bytes(b);
    auto F = [&](int k) { return ws_field(ws + k * fb, b); };
    return {F(0), F(2), F(1), F(3), F(4), F(5)};
}

// Planes per workgroup of the whole-step kernel.  tz > 0: 0, one workgroup
// per (tile, z chunk) item.  tz = 0 (balanced): step4_run_length.
static int step4_run(const s4_ctx *ctx, const Cand &c, const DevBox &D)
{
    if (c.tz > 0)
        return 0;
    const int64_t total = (int64_t)D.tiles[0] * D.tiles[1] * D.n[2];
    int per = max_blocks_step4(c.tx, c.nw);
    if (per <= 0)
        per = 1;
    return (int)step4_run_length(total, (int64_t)per * ctx->ncu, ctx->ncu);
}

// One RK4 step (ui, ri) -> (uo, ro) with a stage-pair or whole-step kernel
// set.  With u3o and r3o the third stage state y_3 = y_n + dt/2 k_2 is also
// written there (else it stays in the workspace, or on chip).
static int rk4_pair_step(s4_ctx *ctx, const Cand &c, const s4_box &b, const double *ui, const double *ri,
                         double *uo, double *ro, const double *c2, const PairFields &W, double dt, hipStream_t s,
                         double *u3o = nullptr, double *r3o = nullptr)
{
    DevBox D = devbox(b, c);
    const int items = (int)dev_items(D);
    double *const U3 = u3o ? u3o : W.U3, *const R3 = u3o ? r3o : W.R3;
    DevBox A = D;
    A.in = ui;
    A.p[0] = ri;
    A.p[5] = c2;
    A.q[0] = U3;
    A.q[1] = R3;
    A.q[2] = W.AU;
    A.q[3] = W.AR;
    if (c.variant == 4) {
        A.q[0] = uo;
        A.q[1] = ro;
        A.q[2] = u3o;
        A.q[3] = u3o ? r3o : nullptr;
        const StageCoef K[4] = {rk4_coef(0, dt), rk4_coef(1, dt), rk4_coef(2, dt), rk4_coef(3, dt)};
        hipError_t e = launch_rk4_step4(c.tx, c.nw, A, K, step4_run(ctx, c, A), ctx->nxcd, s);
        return e == hipSuccess ? S4_OK : hip_fail(e, "whole-step launch");
    }
    hipError_t e = c.variant == 3
                       ? launch_pair2(0, c.tx, c.nw, A, rk4_coef(0, dt), rk4_coef(1, dt), items, ctx->nxcd, s)
                       : launch_rk4_pair(0, c.tx, c.nw, A, rk4_coef(0, dt), rk4_coef(1, dt), items, ctx->nxcd, s);
    if (e != hipSuccess)
        return hip_fail(e, "stage-pair launch");
    DevBox Bx = D;
    Bx.in = U3;
    Bx.p[0] = R3;
    Bx.p[1] = ui;
    Bx.p[2] = ri;
    Bx.p[3] = W.AU;
    Bx.p[4] = W.AR;
    Bx.p[5] = c2;
    Bx.q[0] = uo;
    Bx.q[1] = ro;
    e = c.variant == 3 ? launch_pair2(1, c.tx, c.nw, Bx, rk4_coef(2, dt), rk4_coef(3, dt), items, ctx->nxcd, s)
                       : launch_rk4_pair(1, c.tx, c.nw, Bx, rk4_coef(2, dt), rk4_coef(3, dt), items, ctx->nxcd, s);
    if (e != hipSuccess)
        return hip_fail(e, "stage-pair launch");
    return S4_OK;
}

// two fused steps: (u, rho) -> ping-pong copy -> (u, rho)
static int rk4_pair_double_step(s4_ctx *ctx, const Cand &c, const s4_box &b, double *u, double *rho,
                                const double *c2, const PairFields &W, double dt, hipStream_t s)
{
    int r = rk4_pair_step(ctx, c, b, u, rho, W.Up, W.Rp, c2, W, dt, s);
    if (r)
        return r;
    return rk4_pair_step(ctx, c, b, W.Up, W.Rp, u, rho, c2, W, dt, s);
}

static std::string graph_key(const s4_box *b, int nbox, double *const *u, double *const *rho,
                             const double *const *c2, double dt, const void *ws, int cand, bool batched)
{
    std::ostringstream o;
    o.precision(17);
    o << "g" << nbox << "|" << dt << "|" << ws << "|" << cand << "|" << batched;
    for (int i = 0; i < nbox; ++i) {
        o << "|" << (const void *)u[i] << "," << (const void *)rho[i] << "," << (const void *)(c2 ? c2[i] : nullptr);
        o << "," << b[i].n[0] << "," << b[i].n[1] << "," << b[i].n[2] << "," << b[i].ghost << "," << b[i].stride[1]
          << "," << b[i].stride[2] << "," << b[i].dx[0] << "," << b[i].dx[1] << "," << b[i].dx[2];
    }
    return o.str();
}

// Replay a captured piece of work nrep times on stream s.  The capture is
// made once per key (recorded on the context's private stream) and cached
// in the context, at most GRAPH_CACHE entries: the least recently used one
// is dropped, once the launches recorded before its event have run.  The
// launches are enqueued with the context's lock held, so no other thread
// drops the entry in between.
static const size_t GRAPH_CACHE = 64;

static int graph_run(s4_ctx *ctx, const std::string &key, const std::function<int(hipStream_t)> &record, int nrep,
                     hipStream_t s)
{
    std::unique_lock<std::mutex> lk(ctx->mu);
    if (ctx->graphs.find(key) == ctx->graphs.end()) {
        lk.unlock();
        GraphEntry ge;
        std::unique_lock<std::mutex> cl(ctx->cap_mu);
        S4_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        int r = record(ctx->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->cap, &g);
        cl.unlock();
        if (r) {
            if (g)
                (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess)
            return hip_fail(e, "hipStreamEndCapture");
        ge.graph = g;
        e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            graph_free(ge);
            return hip_fail(e, "hipGraphInstantiate");
        }
        if (g_timer)
            g_timer->restart();
        lk.lock();
        if (ctx->graphs.find(key) != ctx->graphs.end()) {
            graph_free(ge); // another thread captured the same work meanwhile
        } else {
            while (ctx->graphs.size() >= GRAPH_CACHE) {
                auto lru = ctx->graphs.begin();
                for (auto it = ctx->graphs.begin(); it != ctx->graphs.end(); ++it)
                    if (it->second.used < lru->second.used)
                        lru = it;
                graph_free(lru->second);
                ctx->graphs.erase(lru);
            }
            ctx->graphs[key] = ge;
        }
    }
    GraphEntry &ge = ctx->graphs[key];
    ge.used = ++ctx->graph_tick;
    for (int k = 0; k < nrep; ++k)
        S4_HIP(hipGraphLaunch(ge.exec, s));
    S4_HIP(hipEventRecord(ge.done, s));
    return S4_OK;
}

static int rk4_run(s4_ctx *ctx, const Choice &ch, const s4_box *b, int nbox, double *const *u, double *const *rho,
                   const double *const *c2, double dt, int nsteps, int mode, void *workspace, hipStream_t s);
static int pair_run(s4_ctx *ctx, int ci, const s4_box *b, int nbox, double *const *u, double *const *rho,
                    const double *const *c2, double dt, int nsteps, int mode, void *workspace, hipStream_t s,
                    const s4_level *L);

// argument checks shared by s4_rk4 and s4_level_rk4 (need: workspace bytes)
static int rk4_check(s4_ctx *ctx, const s4_box *b, int nbox, double *const *u, double *const *rho,
                     const double *const *c2, double dt, int nsteps, int mode, void *workspace, size_t ws_bytes,
                     size_t need)
{
    if (!ctx || !u || !rho)
        return fail(S4_EINVAL, "NULL argument");
    int r = check_boxes(b, nbox, S4_OP_RK4);
    if (r)
        return r;
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(S4_EINVAL, "dt must be finite and > 0");
    if (nsteps < 0)
        return fail(S4_EINVAL, "nsteps < 0");
    if (mode < S4_PERBOX || mode > S4_GRAPH)
        return fail(S4_EINVAL, "unknown mode %d", mode);
    std::vector<Range> wr, all;
    for (int i = 0; i < nbox; ++i) {
        if ((r = check_ptr(u[i], "u", i)) || (r = check_ptr(rho[i], "rho", i)) ||
            (r = check_ptr(c2 ? c2[i] : nullptr, "c2", i, true)))
            return r;
        const size_t n = (size_t)box_elems(b[i]) * 8;
        wr.push_back({u[i], n, "u", i});
        wr.push_back({rho[i], n, "rho", i});
        if (c2 && c2[i])
            all.push_back({c2[i], n, "c2", i});
    }
    if (nsteps == 0)
        return S4_OK;
    if (!workspace)
        return fail(S4_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace & 255)
        return fail(S4_ELAYOUT, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(S4_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    wr.push_back({workspace, need, "workspace", 0});
    for (auto &w : wr)
        all.push_back(w);
    return check_disjoint(wr, all);
}

int s4_rk4(s4_ctx *ctx, const s4_box *b, int nbox, double *const *u, double *const *rho, const double *const *c2,
           double dt, int nsteps, int mode, void *workspace, size_t ws_bytes, void *stream)
{
    if (!b || nbox <= 0 || nbox > (1 << 20))
        return check_boxes(b, nbox, S4_OP_RK4);
    const size_t need = rk4_fields_bytes(b, nbox) + rk4_table_bytes(nbox);
    int r = rk4_check(ctx, b, nbox, u, rho, c2, dt, nsteps, mode, workspace, ws_bytes, need);
    if (r || nsteps == 0)
        return r;
    hipStream_t s = (hipStream_t)stream;
    const Choice ch = choose(ctx, S4_OP_RK4, b, nbox, false, false, has_c2(c2, nbox));
    OnlineTimer tm(ctx, ch, s);
    r = rk4_run(ctx, ch, b, nbox, u, rho, c2, dt, nsteps, mode, workspace, s);
    if (r)
        return r;
    tm.stop((double)nsteps);
    return S4_OK;
}

int s4_rk4_noalloc(s4_ctx *ctx, const s4_box *b, int nbox, double *const *u, double *const *rho,
                   const double *const *c2, double dt, int nsteps, int mode, void *stream)
{
    if (!ctx)
        return fail(S4_EINVAL, "ctx is NULL");
    if (!b || nbox <= 0 || nbox > (1 << 20))
        return check_boxes(b, nbox, S4_OP_RK4);
    if (mode == S4_GRAPH)
        return fail(S4_ENOTSUP, "s4_rk4_noalloc runs S4_PERBOX or S4_BATCHED (S4_GRAPH instantiates a graph)");
    if (!ctx->scratch)
        return fail(S4_EDEVICE, "no scratch array address on device %d: %s", ctx->device, ctx->scratch_err.c_str());
    const size_t need = rk4_fields_bytes(b, nbox) + rk4_table_bytes(nbox);
    if (need > (size_t)S4_NOALLOC_SCRATCH_BYTES)
        return fail(S4_ENOMEM, "these boxes need %zu bytes of scratch, s4_rk4_noalloc holds %zu (use s4_rk4)",
                    need, (size_t)S4_NOALLOC_SCRATCH_BYTES);
    int r = rk4_check(ctx, b, nbox, u, rho, c2, dt, nsteps, mode, ctx->scratch, S4_NOALLOC_SCRATCH_BYTES, need);
    if (r || nsteps == 0)
        return r;
    // the loop setup's current choice without an on-line trial (no events)
    const Choice ch = choose(ctx, S4_OP_RK4, b, nbox, true, false, has_c2(c2, nbox));
    return rk4_run(ctx, ch, b, nbox, u, rho, c2, dt, nsteps, mode, ctx->scratch, (hipStream_t)stream);
}

// s4_rk4_step_to and s4_rk4_step_to_y3: one step out of place, optionally
// keeping y_3 (u3o, r3o non-NULL)
static int rk4_step_to(s4_ctx *ctx, const s4_box *b, const double *u_in, const double *rho_in, const double *c2,
                       double dt, double *u_out, double *rho_out, double *u3o, double *r3o, void *workspace,
                       size_t ws_bytes, void *stream)
{
    const bool y3 = u3o || r3o;
    if (!ctx || !u_in || !rho_in || !u_out || !rho_out || (y3 && !(u3o && r3o)))
        return fail(S4_EINVAL, "NULL argument");
    int r = check_boxes(b, 1, S4_OP_RK4);
    if (r)
        return r;
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(S4_EINVAL, "dt must be finite and > 0");
    if ((r = check_ptr(u_in, "u_in", 0)) || (r = check_ptr(rho_in, "rho_in", 0)) ||
        (r = check_ptr(u_out, "u_out", 0)) || (r = check_ptr(rho_out, "rho_out", 0)) ||
        (r = check_ptr(c2, "c2", 0, true)) || (r = check_ptr(u3o, "u3_out", 0, true)) ||
        (r = check_ptr(r3o, "rho3_out", 0, true)))
        return r;
    const size_t need = rk4_fields_bytes(b, 1) + rk4_table_bytes(1);
    if (!workspace)
        return fail(S4_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace & 255)
        return fail(S4_ELAYOUT, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(S4_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    const size_t n = (size_t)box_elems(b[0]) * 8;
    std::vector<Range> wr = {{u_out, n, "u_out", 0}, {rho_out, n, "rho_out", 0}, {workspace, need, "workspace", 0}};
    if (y3) {
        wr.push_back({u3o, n, "u3_out", 0});
        wr.push_back({r3o, n, "rho3_out", 0});
    }
    std::vector<Range> all = wr;
    all.push_back({u_in, n, "u_in", 0});
    all.push_back({rho_in, n, "rho_in", 0});
    if (c2)
        all.push_back({c2, n, "c2", 0});
    if ((r = check_disjoint(wr, all)))
        return r;
    hipStream_t s = (hipStream_t)stream;
    if (y3) {
        // the current choice without a trial of the on-line tuner (these calls
        // are not timed); per-stage kernel sets give way to the stage pairs,
        // whose first pass stores y_3
        int ci = choose(ctx, S4_OP_RK4, b, 1, true, false, c2 != nullptr).cand;
        const int v = cands()[ci].variant;
        if (v != 1 && v != 3 && v != 4)
            ci = heuristic(ctx, S4_OP_RK4, b, 1, true);
        return rk4_pair_step(ctx, cands()[ci], b[0], u_in, rho_in, u_out, rho_out, c2,
                             pair_fields(b[0], (char *)workspace), dt, s, u3o, r3o);
    }
    const Choice ch = choose(ctx, S4_OP_RK4, b, 1, false, false, c2 != nullptr);
    OnlineTimer tm(ctx, ch, s);
    const Cand &c = cands()[ch.cand];
    if (c.variant == 1 || c.variant == 3 || c.variant == 4) {
        r = rk4_pair_step(ctx, c, b[0], u_in, rho_in, u_out, rho_out, c2, pair_fields(b[0], (char *)workspace), dt,
                          s);
    } else {
        std::vector<DevBox> tab;
        double *uo[1] = {u_out}, *ro[1] = {rho_out};
        const double *ui[1] = {u_in}, *ri[1] = {rho_in}, *c2v[1] = {c2};
        rk4_tables_io(b, 1, ui, ri, uo, ro, c2 ? c2v : nullptr, (char *)workspace, c, tab);
        r = rk4_step(ctx, c, tab, 1, false, nullptr, nullptr, dev_items(tab[0]), dt, s);
    }
    if (r)
        return r;
    tm.stop(1.0);
    return S4_OK;
}

int s4_rk4_step_to(s4_ctx *ctx, const s4_box *b, const double *u_in, const double *rho_in, const double *c2,
                   double dt, double *u_out, double *rho_out, void *workspace, size_t ws_bytes, void *stream)
{
    return rk4_step_to(ctx, b, u_in, rho_in, c2, dt, u_out, rho_out, nullptr, nullptr, workspace, ws_bytes, stream);
}

int s4_rk4_step_to_y3(s4_ctx *ctx, const s4_box *b, const double *u_in, const double *rho_in, const double *c2,
                      double dt, double *u_out, double *rho_out, double *u3_out, double *rho3_out, void *workspace,
                      size_t ws_bytes, void *stream)
{
    if (!u3_out || !rho3_out)
        return fail(S4_EINVAL, "NULL argument");
    return rk4_step_to(ctx, b, u_in, rho_in, c2, dt, u_out, rho_out, u3_out, rho3_out, workspace, ws_bytes,
                       stream);
}

// the launches of s4_rk4 for choice ch (arguments already validated)
static int rk4_run(s4_ctx *ctx, const Choice &ch, const s4_box *b, int nbox, double *const *u, double *const *rho,
                   const double *const *c2, double dt, int nsteps, int mode, void *workspace, hipStream_t s)
{
    int r;
    char *ws = (char *)workspace;
    if (cands()[ch.cand].variant == 1 && nbox == 1) {
        // widened-tile stage pairs: pairs of steps, an odd last step with the stage kernels
        const Cand &cp = cands()[ch.cand];
        const PairFields W = pair_fields(b[0], ws);
        const double *c2b = c2 ? c2[0] : nullptr;
        const int pairs = nsteps / 2;
        if (pairs > 0) {
            if (mode != S4_GRAPH) {
                for (int k = 0; k < pairs; ++k)
                    if ((r = rk4_pair_double_step(ctx, cp, b[0], u[0], rho[0], c2b, W, dt, s)))
                        return r;
            } else {
                const std::string key = "pair|" + graph_key(b, nbox, u, rho, c2, dt, workspace, ch.cand, false);
                r = graph_run(
                    ctx, key,
                    [&](hipStream_t cs) { return rk4_pair_double_step(ctx, cp, b[0], u[0], rho[0], c2b, W, dt, cs); },
                    pairs, s);
                if (r)
                    return r;
            }
        }
        if (nsteps % 2 == 0)
            return S4_OK;
        // odd remainder: one step with the per-stage kernels (same arithmetic)
        const Cand &c0 = cands()[tile_heuristic(ctx, b, nbox)];
        std::vector<DevBox> tab0;
        rk4_tables(b, nbox, u, rho, c2, ws, c0, tab0);
        return rk4_step(ctx, c0, tab0, nbox, false, nullptr, nullptr, dev_items(tab0[0]), dt, s);
    }
    if (cands()[ch.cand].variant == 3 || cands()[ch.cand].variant == 4) {
        if ((r = pair_run(ctx, ch.cand, b, nbox, u, rho, c2, dt, nsteps / 2 * 2, mode, workspace, s, nullptr)) ||
            nsteps % 2 == 0)
            return r;
        // an odd last step with the per-stage kernels (same arithmetic)
        const Choice c0{tile_heuristic(ctx, b, nbox), 0, ch.key};
        return rk4_run(ctx, c0, b, nbox, u, rho, c2, dt, 1, mode == S4_GRAPH ? S4_BATCHED : mode, workspace, s);
    }
    const Cand &c = cands()[ch.cand];
    std::vector<DevBox> tab;
    rk4_tables(b, nbox, u, rho, c2, ws, c, tab);
    int64_t nitems = 0;
    for (int i = 0; i < nbox; ++i)
        nitems += dev_items(tab[i]);
    if (nitems > 0x3fffffff)
        return fail(S4_EINVAL, "too many work items");
    const bool batched = nbox > 1 && mode != S4_PERBOX;
    DevBox *dtab = (DevBox *)(ws + rk4_fields_bytes(b, nbox));
    int *counters = (int *)((char *)dtab + round256(4 * (size_t)nbox * sizeof(DevBox)));
    if (batched) {
        // table bytes followed by zeroed queue counters
        std::vector<char> bytes(rk4_table_bytes(nbox), 0);
        memcpy(bytes.data(), tab.data(), tab.size() * sizeof(DevBox));
        if ((r = upload_table(dtab, bytes, s)))
            return r;
    }
    if (mode != S4_GRAPH) {
        for (int step = 0; step < nsteps; ++step)
            if ((r = rk4_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, s)))
                return r;
        return S4_OK;
    }
    const std::string key = graph_key(b, nbox, u, rho, c2, dt, workspace, ch.cand, batched);
    return graph_run(
        ctx, key,
        [&](hipStream_t cs) { return rk4_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, cs); }, nsteps,
        s);
}

int s4_wave_adjoint_rhs(s4_ctx *ctx, const s4_box *b, int nbox, const double *const *lu,
                        const double *const *lrho, const double *const *c2, double *const *out_u,
                        double *const *out_rho, void *stream)
{
    if (!ctx || !lu || !lrho || !out_u || !out_rho)
        return fail(S4_EINVAL, "NULL argument");
    int r = check_boxes(b, nbox, S4_OP_ADJOINT_RHS);
    if (r)
        return r;
    std::vector<Range> wr, all;
    for (int i = 0; i < nbox; ++i) {
        if ((r = check_ptr(lu[i], "lu", i)) || (r = check_ptr(lrho[i], "lrho", i)) ||
            (r = check_ptr(out_u[i], "out_u", i)) || (r = check_ptr(out_rho[i], "out_rho", i)) ||
            (r = check_ptr(c2 ? c2[i] : nullptr, "c2", i, true)))
            return r;
        const size_t n = (size_t)box_elems(b[i]) * 8;
        wr.push_back({out_u[i], n, "out_u", i});
        wr.push_back({out_rho[i], n, "out_rho", i});
        all.push_back({lu[i], n, "lu", i});
        all.push_back({lrho[i], n, "lrho", i});
        if (c2 && c2[i])
            all.push_back({c2[i], n, "c2", i});
    }
    for (auto &w : wr)
        all.push_back(w);
    if ((r = check_disjoint(wr, all)))
        return r;
    const Choice ch = choose(ctx, S4_OP_ADJOINT_RHS, b, nbox);
    const Cand &c = cands()[ch.cand];
    OnlineTimer tm(ctx, ch, (hipStream_t)stream);
    StageCoef K{};
    K.scale = 1.0;
    for (int i = 0; i < nbox; ++i) {
        DevBox D = devbox(b[i], c);
        D.in = lrho[i];
        D.inmul = c2 ? c2[i] : nullptr;
        D.p[0] = lu[i];
        D.q[0] = out_u[i];
        D.q[1] = out_rho[i];
        if ((r = launch_one(ctx, OP_ADJRHS, c, D, K, (hipStream_t)stream)))
            return r;
    }
    tm.stop(1.0);
    return S4_OK;
}

// One backward RK4 step: with c2_bar, the forward stage-pair kernel gives
// u_3 and rho_3 (unless the caller passes them, y3_u and y3_r); then the
// two adjoint passes (stages 4-3, then 2-1).
// Workspace fields: U3 R3 KR2 KR1 ACU ACR.
static int adjoint_step_launch(s4_ctx *ctx, const Cand &c, const s4_box &b, const double *u_n, const double *rho_n,
                               const double *c2, double dt, double *lam_u, double *lam_rho, double *c2_bar,
                               char *ws, hipStream_t s, const double *y3_u = nullptr, const double *y3_r = nullptr)
{
    const size_t fb = field_bytes(b);
    double *F[ADJ_FIELDS];
    for (int k = 0; k < ADJ_FIELDS; ++k)
        F[k] = ws_field(ws + k * fb, b);
    double *KR2 = F[2], *KR1 = F[3], *ACU = F[4], *ACR = F[5];
    const double *U3 = y3_u ? y3_u : F[0], *R3 = y3_u ? y3_r : F[1];
    const bool cb = c2_bar != nullptr;
    hipError_t e;
    if (cb && !y3_u) {
        // the per-tap pair-0 kernel with the stage-pair heuristic's tile (z
        // chunks short enough to give every CU several items)
        const Cand &pc = cands()[heuristic(ctx, S4_OP_RK4, &b, 1, true)];
        DevBox A = devbox(b, pc);
        A.in = u_n;
        A.p[0] = rho_n;
        A.p[5] = c2;
        A.q[0] = F[0];
        A.q[1] = F[1];
        e = launch_pair2(0, pc.tx, pc.nw, A, rk4_coef(0, dt), rk4_coef(1, dt), (int)dev_items(A), ctx->nxcd, s);
        if (e != hipSuccess)
            return hip_fail(e, "forward stage-pair launch");
    }
    StageCoef K{};
    K.a = dt;
    K.b = dt / 6.0;
    K.a_next = dt / 3.0;
    K.b_next = dt / 2.0;
    K.scale = 1.0;
    const DevBox D = devbox(b, c);
    const int items = (int)dev_items(D);
    DevBox E = D;
    E.in = lam_u;
    E.p[0] = lam_rho;
    E.p[1] = U3;
    E.p[2] = u_n;
    E.p[3] = R3;
    E.p[5] = c2;
    E.p[6] = c2_bar;
    E.q[0] = KR2;
    E.q[1] = KR1;
    E.q[2] = ACU;
    E.q[3] = ACR;
    E.q[4] = c2_bar;
    if ((e = launch_adj2(0, c.tx, c.nw, cb, E, K, items, ctx->nxcd, s)) != hipSuccess)
        return hip_fail(e, "adjoint pass launch");
    E = D;
    E.in = KR2;
    E.p[0] = KR1;
    E.p[1] = u_n;
    E.p[2] = rho_n;
    E.p[3] = ACU;
    E.p[4] = ACR;
    E.p[5] = c2;
    E.p[6] = c2_bar;
    E.q[0] = lam_u;
    E.q[1] = lam_rho;
    E.q[4] = c2_bar;
    if ((e = launch_adj2(1, c.tx, c.nw, cb, E, K, items, ctx->nxcd, s)) != hipSuccess)
        return hip_fail(e, "adjoint pass launch");
    return S4_OK;
}

// s4_rk4_adjoint_step and s4_rk4_adjoint_step_y3 (y3_u, y3_r: the step's
// third stage state, or NULL to form it here)
static int rk4_adjoint_step(s4_ctx *ctx, const s4_box *b, const double *u_n, const double *rho_n,
                            const double *y3_u, const double *y3_r, const double *c2, double dt, double *lam_u,
                            double *lam_rho, double *c2_bar, void *workspace, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return fail(S4_EINVAL, "ctx is NULL");
    int r = check_boxes(b, 1, S4_OP_ADJOINT_STEP);
    if (r)
        return r;
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(S4_EINVAL, "dt must be finite and > 0");
    if ((r = check_ptr(u_n, "u_n", 0)) || (r = check_ptr(rho_n, "rho_n", 0)) ||
        (r = check_ptr(lam_u, "lam_u", 0)) || (r = check_ptr(lam_rho, "lam_rho", 0)) ||
        (r = check_ptr(c2, "c2", 0, true)) || (r = check_ptr(c2_bar, "c2_bar", 0, true)) ||
        (r = check_ptr(y3_u, "u3", 0, true)) || (r = check_ptr(y3_r, "rho3", 0, true)))
        return r;
    if (!y3_u != !y3_r)
        return fail(S4_EINVAL, "u3 and rho3 must both be given or both be NULL");
    const size_t fb = field_bytes(b[0]);
    const size_t need = ADJ_FIELDS * fb;
    if (!workspace)
        return fail(S4_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace & 255)
        return fail(S4_ELAYOUT, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(S4_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    const size_t n = (size_t)box_elems(b[0]) * 8;
    std::vector<Range> wr = {{lam_u, n, "lam_u", 0}, {lam_rho, n, "lam_rho", 0}, {workspace, need, "workspace", 0}};
    if (c2_bar)
        wr.push_back({c2_bar, n, "c2_bar", 0});
    std::vector<Range> all = {{u_n, n, "u_n", 0}, {rho_n, n, "rho_n", 0}};
    if (c2)
        all.push_back({c2, n, "c2", 0});
    if (y3_u) {
        all.push_back({y3_u, n, "u3", 0});
        all.push_back({y3_r, n, "rho3", 0});
    }
    for (auto &w : wr)
        all.push_back(w);
    if ((r = check_disjoint(wr, all)))
        return r;

    const Choice ch = choose(ctx, S4_OP_ADJOINT_STEP, b, 1);
    const Cand &c = cands()[ch.cand];
    OnlineTimer tm(ctx, ch, (hipStream_t)stream);
    if ((r = adjoint_step_launch(ctx, c, b[0], u_n, rho_n, c2, dt, lam_u, lam_rho, c2_bar, (char *)workspace,
                                 (hipStream_t)stream, y3_u, y3_r)))
        return r;
    tm.stop(1.0);
    return S4_OK;
}

int s4_rk4_adjoint_step(s4_ctx *ctx, const s4_box *b, const double *u_n, const double *rho_n, const double *c2,
                        double dt, double *lam_u, double *lam_rho, double *c2_bar, void *workspace,
                        size_t ws_bytes, void *stream)
{
    return rk4_adjoint_step(ctx, b, u_n, rho_n, nullptr, nullptr, c2, dt, lam_u, lam_rho, c2_bar, workspace,
                            ws_bytes, stream);
}

int s4_rk4_adjoint_step_y3(s4_ctx *ctx, const s4_box *b, const double *u_n, const double *rho_n,
                           const double *u3, const double *rho3, const double *c2, double dt, double *lam_u,
                           double *lam_rho, double *c2_bar, void *workspace, size_t ws_bytes, void *stream)
{
    if (c2_bar && (!u3 || !rho3))
        return fail(S4_EINVAL, "u3 and rho3 are needed with c2_bar");
    return rk4_adjoint_step(ctx, b, u_n, rho_n, c2_bar ? u3 : nullptr, c2_bar ? rho3 : nullptr, c2, dt, lam_u,
                            lam_rho, c2_bar, workspace, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// level: ghost exchange between the boxes of one refinement level

static int64_t sync_blocks(const s4_level *L)
{
    int64_t blk = 0;
    for (const LevelPiece &P : L->pieces)
        blk += (P.n[0] * P.n[1] * P.n[2] + 255) / 256;
    return blk;
}

// bytes of the device schedule: the pieces, then one piece index per workgroup
static size_t sync_pieces_bytes(const s4_level *L)
{
    return round256(std::max<size_t>(1, L->pieces.size()) * sizeof(SyncPiece)) +
           round256((size_t)std::max<int64_t>(1, sync_blocks(L)) * sizeof(int));
}

static size_t ptr_table_bytes(int nbox, int ntab)
{
    return round256((size_t)ntab * nbox * sizeof(double *));
}

// the device schedule's bytes (sync_pieces_bytes long) at dst
static void sync_table(const s4_level *L, char *dst)
{
    SyncPiece *out = (SyncPiece *)dst;
    int *W = (int *)(dst + round256(std::max<size_t>(1, L->pieces.size()) * sizeof(SyncPiece)));
    int64_t blk = 0;
    for (size_t p = 0; p < L->pieces.size(); ++p) {
        const LevelPiece &P = L->pieces[p];
        const s4_box &d = L->boxes[(size_t)P.dst], &sb = L->boxes[(size_t)P.src];
        SyncPiece q;
        memset(&q, 0, sizeof q);
        q.dst = P.dst;
        q.src = P.src;
        for (int a = 0; a < 3; ++a)
            q.n[a] = (int32_t)P.n[a];
        q.blk0 = (int32_t)blk;
        q.doff = (P.d0[0] + d.ghost) + (P.d0[1] + d.ghost) * d.stride[1] + (P.d0[2] + d.ghost) * d.stride[2];
        q.soff = (P.s0[0] + sb.ghost) + (P.s0[1] + sb.ghost) * sb.stride[1] + (P.s0[2] + sb.ghost) * sb.stride[2];
        q.dsy = d.stride[1];
        q.dsz = d.stride[2];
        q.ssy = sb.stride[1];
        q.ssz = sb.stride[2];
        out[p] = q;
        const int64_t nb = (P.n[0] * P.n[1] * P.n[2] + 255) / 256;
        for (int64_t k = 0; k < nb; ++k)
            W[blk + k] = (int)p;
        blk += nb;
    }
}

static const int *sync_block_table(const s4_level *L, const void *dev)
{
    return (const int *)((const char *)dev + round256(std::max<size_t>(1, L->pieces.size()) * sizeof(SyncPiece)));
}

static int level_check(const s4_level *L)
{
    if (!L)
        return fail(S4_EINVAL, "level is NULL");
    int r = check_boxes(L->boxes.data(), (int)L->boxes.size(), S4_OP_RK4);
    if (r)
        return r;
    if (sync_blocks(L) > 0x7fffffff)
        return fail(S4_EINVAL, "ghost exchange too large for one launch");
    for (const LevelPiece &P : L->pieces)
        if (P.n[0] * P.n[1] * P.n[2] >= ((int64_t)1 << 31))
            return fail(S4_EINVAL, "ghost exchange piece of %lld points is too large",
                        (long long)(P.n[0] * P.n[1] * P.n[2]));
    return S4_OK;
}

int s4_level_workspace_size(const s4_level *L, int op, size_t *bytes)
{
    if (!bytes)
        return fail(S4_EINVAL, "NULL argument");
    int r = level_check(L);
    if (r)
        return r;
    const int nbox = (int)L->boxes.size();
    if (op == S4_OP_LEVEL_SYNC)
        *bytes = sync_pieces_bytes(L) + ptr_table_bytes(nbox, 1);
    else if (op == S4_OP_RK4)
        *bytes = rk4_fields_bytes(L->boxes.data(), nbox) + rk4_table_bytes(nbox) + sync_pieces_bytes(L) +
                 ptr_table_bytes(nbox, 8);
    else
        return fail(S4_EINVAL, "op %d has no level workspace", op);
    return S4_OK;
}

int s4_level_sync(s4_ctx *ctx, const s4_level *L, double *const *f, void *workspace, size_t ws_bytes, void *stream)
{
    if (!ctx || !f)
        return fail(S4_EINVAL, "NULL argument");
    int r = level_check(L);
    if (r)
        return r;
    const int nbox = (int)L->boxes.size();
    std::vector<Range> wr;
    for (int i = 0; i < nbox; ++i) {
        if ((r = check_ptr(f[i], "f", i)))
            return r;
        wr.push_back({f[i], (size_t)box_elems(L->boxes[(size_t)i]) * 8, "f", i});
    }
    const size_t need = sync_pieces_bytes(L) + ptr_table_bytes(nbox, 1);
    if (!workspace)
        return fail(S4_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace & 255)
        return fail(S4_ELAYOUT, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(S4_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    std::vector<Range> all = wr;
    all.push_back({workspace, need, "workspace", 0});
    wr.push_back(all.back());
    if ((r = check_disjoint(wr, all)))
        return r;
    const int64_t nblocks = sync_blocks(L);
    if (nblocks == 0)
        return S4_OK;
    hipStream_t s = (hipStream_t)stream;
    std::vector<char> bytes(need, 0);
    sync_table(L, bytes.data());
    memcpy(bytes.data() + sync_pieces_bytes(L), f, (size_t)nbox * sizeof(double *));
    if ((r = upload_table(workspace, bytes, s)))
        return r;
    const SyncPiece *P = (const SyncPiece *)workspace;
    double *const *F = (double *const *)((char *)workspace + sync_pieces_bytes(L));
    hipError_t e = launch_sync(P, sync_block_table(L, workspace), F, 1, nbox, (int)nblocks, s);
    if (e != hipSuccess)
        return hip_fail(e, "ghost exchange launch");
    return S4_OK;
}

// Per-stage RK4 on a level (candidate ci of variant 0 or 2): exchange the
// stage input, then the ghost-addressed stage kernels, four times a step.
static int level_stage_run(s4_ctx *ctx, const s4_level *L, int ci, double *const *u, double *const *rho,
                           const double *const *c2, double dt, int nsteps, int mode, void *workspace, hipStream_t s)
{
    const s4_box *b = L->boxes.data();
    const int nbox = (int)L->boxes.size();
    const Cand &c = cands()[ci];
    char *ws = (char *)workspace;
    std::vector<DevBox> tab;
    rk4_tables(b, nbox, u, rho, c2, ws, c, tab);
    int64_t nitems = 0;
    for (int i = 0; i < nbox; ++i)
        nitems += dev_items(tab[i]);
    if (nitems > 0x3fffffff)
        return fail(S4_EINVAL, "too many work items");
    const int64_t nblocks = sync_blocks(L);

    // [stage tables | item counters | exchange schedule | stage-input pointers], uploaded at once
    const size_t tb = rk4_table_bytes(nbox), pb = sync_pieces_bytes(L), fb = ptr_table_bytes(nbox, 8);
    char *dbase = ws + rk4_fields_bytes(b, nbox);
    std::vector<char> bytes(tb + pb + fb, 0);
    memcpy(bytes.data(), tab.data(), tab.size() * sizeof(DevBox));
    sync_table(L, bytes.data() + tb);
    double **F = (double **)(bytes.data() + tb + pb);
    for (int st = 0; st < 4; ++st)
        for (int i = 0; i < nbox; ++i)
            F[(size_t)st * nbox + i] = const_cast<double *>(tab[(size_t)st * nbox + i].in);
    int r = upload_table(dbase, bytes, s);
    if (r)
        return r;
    DevBox *dtab = (DevBox *)dbase;
    int *counters = (int *)(dbase + round256(4 * (size_t)nbox * sizeof(DevBox)));
    const SyncArgs sy{(const SyncPiece *)(dbase + tb), sync_block_table(L, dbase + tb), (int)nblocks,
                      (double *const *)(dbase + tb + pb)};
    const bool batched = nbox > 1 && mode != S4_PERBOX;
    if (mode != S4_GRAPH) {
        for (int step = 0; step < nsteps; ++step)
            if ((r = rk4_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, s, &sy)))
                return r;
        return S4_OK;
    }
    const std::string key = "level|" + std::to_string(L->serial) + "|" +
                            graph_key(b, nbox, u, rho, c2, dt, workspace, ci, batched);
    return graph_run(
        ctx, key,
        [&](hipStream_t cs) { return rk4_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, cs, &sy); },
        nsteps, s);
}

// Stage-pair RK4 (variant 3) over any set of boxes, on their own (periodic
// addressing) or as a level (ghost addressing with exchanges).  A step of
// parity 0 reads y from (u, rho) and writes the workspace copy (Up, Rp); a
// step of parity 1 goes back, so an even number of steps ends in the
// caller's buffers.  Tables: [parity][pair][box].  On a level, pair 0 needs
// the ghosts of its input u and rho, pair 1 those of u_3 and rho_3 (its u_n
// ghosts are still those exchanged before pair 0).
static void pair_tables(const s4_box *b, int nbox, double *const *u, double *const *rho, const double *const *c2,
                        const std::vector<char *> &wsb, const Cand &c, std::vector<DevBox> &tab,
                        std::vector<PairFields> &pf)
{
    tab.assign(4 * (size_t)nbox, DevBox{});
    pf.resize((size_t)nbox);
    int item0 = 0;
    for (int i = 0; i < nbox; ++i) {
        const PairFields W = pair_fields(b[i], wsb[(size_t)i]);
        pf[(size_t)i] = W;
        DevBox D = devbox(b[i], c);
        D.item0 = item0;
        item0 += (int)dev_items(D);
        for (int p = 0; p < 2; ++p) {
            const double *ui = p ? W.Up : u[i], *ri = p ? W.Rp : rho[i];
            double *uo = p ? u[i] : W.Up, *ro = p ? rho[i] : W.Rp;
            DevBox A = D;
            A.in = ui;
            A.p[0] = ri;
            A.p[5] = c2 ? c2[i] : nullptr;
            if (c.variant == 4) { // one whole step: y_n -> y_{n+1} (table 2p; 2p+1 unused)
                A.q[0] = uo;
                A.q[1] = ro;
                tab[(size_t)(2 * p) * nbox + i] = A;
                tab[(size_t)(2 * p + 1) * nbox + i] = A;
                continue;
            }
            A.q[0] = W.U3;
            A.q[1] = W.R3;
            A.q[2] = W.AU;
            A.q[3] = W.AR;
            DevBox Bx = D;
            Bx.in = W.U3;
            Bx.p[0] = W.R3;
            Bx.p[1] = ui;
            Bx.p[2] = ri;
            Bx.p[3] = W.AU;
            Bx.p[4] = W.AR;
            Bx.p[5] = c2 ? c2[i] : nullptr;
            Bx.q[0] = uo;
            Bx.q[1] = ro;
            tab[(size_t)(2 * p) * nbox + i] = A;
            tab[(size_t)(2 * p + 1) * nbox + i] = Bx;
        }
    }
}

static int pair_step(s4_ctx *ctx, const Cand &c, const std::vector<DevBox> &tab, int nbox, bool batched,
                     DevBox *dtab, int *counters, int64_t nitems, double dt, int parity, hipStream_t s,
                     const SyncArgs *sy)
{
    const bool gh = sy != nullptr;
    if (c.variant == 4) {
        // one whole-step launch: periodic boxes, or a wide level after one
        // exchange of (u, rho) of width 4 or more
        const StageCoef K[4] = {rk4_coef(0, dt), rk4_coef(1, dt), rk4_coef(2, dt), rk4_coef(3, dt)};
        const DevBox *T = tab.data() + (size_t)(2 * parity) * nbox;
        bool hasc2 = false;
        for (int i = 0; i < nbox; ++i) {
            if (T[i].sz * 8 >= (int64_t)0x80000000)
                return fail(S4_ENOTSUP, "whole RK4 steps need z planes below 2 GiB (box %d)", i);
            if (gh && T[i].g < 4)
                return fail(S4_ENOTSUP, "whole RK4 steps on a level need 4 ghost layers (box %d)", i);
            hasc2 = hasc2 || T[i].p[5] != nullptr;
        }
        hipError_t e = hipSuccess;
        if (gh) {
            e = launch_sync(sy->P, sy->W, sy->F + (size_t)(2 * parity) * 2 * nbox, 2, nbox, sy->nblocks, s);
            if (e != hipSuccess)
                return hip_fail(e, "ghost exchange launch");
        }
        if (batched) {
            int per = max_blocks_step4(c.tx, c.nw);
            if (per <= 0)
                per = 1;
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)per * ctx->ncu));
            e = launch_rk4_step4_batched(c.tx, c.nw, hasc2, dtab + (size_t)(2 * parity) * nbox, nbox,
                                         step_queue(ctx, counters, parity, nitems), grid, K, s, gh);
        } else {
            for (int i = 0; i < nbox && e == hipSuccess; ++i)
                e = launch_rk4_step4(c.tx, c.nw, T[i], K, step4_run(ctx, c, T[i]), ctx->nxcd, s, gh);
        }
        return e == hipSuccess ? S4_OK : hip_fail(e, "whole-step launch");
    }
    for (int k = 0; k < 2; ++k) {
        const StageCoef K1 = rk4_coef(2 * k, dt), K2 = rk4_coef(2 * k + 1, dt);
        const int t = 2 * parity + k;
        if (sy) {
            hipError_t e = launch_sync(sy->P, sy->W, sy->F + (size_t)t * 2 * nbox, 2, nbox, sy->nblocks, s);
            if (e != hipSuccess)
                return hip_fail(e, "ghost exchange launch");
        }
        if (batched) {
            int per = max_blocks_pair2(k, c.tx, c.nw, gh);
            if (per <= 0)
                per = 2;
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nitems, (int64_t)per * ctx->ncu));
            hipError_t e = launch_pair2_batched(k, c.tx, c.nw, dtab + (size_t)t * nbox, nbox,
                                                step_queue(ctx, counters, t, nitems), grid, K1, K2, s, gh);
            if (e != hipSuccess)
                return hip_fail(e, "batched stage-pair launch");
        } else {
            for (int i = 0; i < nbox; ++i) {
                const DevBox &D = tab[(size_t)t * nbox + i];
                hipError_t e = launch_pair2(k, c.tx, c.nw, D, K1, K2, (int)dev_items(D), ctx->nxcd, s, gh);
                if (e != hipSuccess)
                    return hip_fail(e, "stage-pair launch");
            }
        }
    }
    return S4_OK;
}

// nsteps (even) stage-pair steps; L != NULL: the boxes form that level
static int pair_run(s4_ctx *ctx, int ci, const s4_box *b, int nbox, double *const *u, double *const *rho,
                    const double *const *c2, double dt, int nsteps, int mode, void *workspace, hipStream_t s,
                    const s4_level *L)
{
    if (nsteps <= 0)
        return S4_OK;
    const Cand &c = cands()[ci];
    char *ws = (char *)workspace;
    std::vector<DevBox> tab;
    std::vector<PairFields> pf;
    std::vector<char *> wsb((size_t)nbox);
    size_t off = 0;
    for (int i = 0; i < nbox; ++i) {
        wsb[(size_t)i] = ws + off;
        off += RK4_FIELDS * field_bytes(b[i]);
    }
    pair_tables(b, nbox, u, rho, c2, wsb, c, tab, pf);
    int64_t nitems = 0;
    for (int i = 0; i < nbox; ++i)
        nitems += dev_items(tab[i]);
    if (nitems > 0x3fffffff)
        return fail(S4_EINVAL, "too many work items");
    const bool batched = nbox > 1 && mode != S4_PERBOX;
    char *dbase = ws + rk4_fields_bytes(b, nbox);
    const size_t tb = rk4_table_bytes(nbox);
    const size_t pb = L ? sync_pieces_bytes(L) : 0, fb = L ? ptr_table_bytes(nbox, 8) : 0;
    int r;
    if (batched || L) {
        std::vector<char> bytes(tb + pb + fb, 0);
        memcpy(bytes.data(), tab.data(), tab.size() * sizeof(DevBox));
        if (L) {
            sync_table(L, bytes.data() + tb);
            double **F = (double **)(bytes.data() + tb + pb);
            for (int i = 0; i < nbox; ++i) {
                const PairFields &W = pf[(size_t)i];
                double *fl[4][2] = {{u[i], rho[i]}, {W.U3, W.R3}, {W.Up, W.Rp}, {W.U3, W.R3}};
                for (int t = 0; t < 4; ++t)
                    for (int f = 0; f < 2; ++f)
                        F[(size_t)(2 * t + f) * nbox + i] = fl[t][f];
            }
        }
        if ((r = upload_table(dbase, bytes, s)))
            return r;
    }
    DevBox *dtab = (DevBox *)dbase;
    int *counters = (int *)(dbase + round256(4 * (size_t)nbox * sizeof(DevBox)));
    SyncArgs sy{nullptr, nullptr, 0, nullptr};
    if (L)
        sy = SyncArgs{(const SyncPiece *)(dbase + tb), sync_block_table(L, dbase + tb), (int)sync_blocks(L),
                      (double *const *)(dbase + tb + pb)};
    const SyncArgs *syp = L ? &sy : nullptr;
    auto two = [&](hipStream_t cs) -> int {
        int rr = pair_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, 0, cs, syp);
        return rr ? rr : pair_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, 1, cs, syp);
    };
    if (mode != S4_GRAPH) {
        for (int k = 0; k < nsteps / 2; ++k)
            if ((r = two(s)))
                return r;
        return S4_OK;
    }
    const std::string key = "pair2|" + (L ? std::to_string(L->serial) : std::string("-")) + "|" +
                            graph_key(b, nbox, u, rho, c2, dt, workspace, ci, batched);
    return graph_run(ctx, key, two, nsteps / 2, s);
}

int s4_level_rk4(s4_ctx *ctx, const s4_level *L, double *const *u, double *const *rho, const double *const *c2,
                 double dt, int nsteps, int mode, void *workspace, size_t ws_bytes, void *stream)
{
    int r = level_check(L);
    if (r)
        return r;
    const s4_box *b = L->boxes.data();
    const int nbox = (int)L->boxes.size();
    if (L->width < 2)
        return fail(S4_EGHOST, "level exchange width %d < 2 (stencil radius)", L->width);
    if (L->uncovered > 0)
        return fail(S4_EGHOST, "%lld ghost points of the level are not covered by any box",
                    (long long)L->uncovered);
    size_t need = 0;
    if ((r = s4_level_workspace_size(L, S4_OP_RK4, &need)))
        return r;
    if ((r = rk4_check(ctx, b, nbox, u, rho, c2, dt, nsteps, mode, workspace, ws_bytes, need)) || nsteps == 0)
        return r;
    hipStream_t s = (hipStream_t)stream;
    const int ci = choose(ctx, S4_OP_RK4, b, nbox, true, level_kind(L)).cand;
    if (cands()[ci].variant != 3 && cands()[ci].variant != 4)
        return level_stage_run(ctx, L, ci, u, rho, c2, dt, nsteps, mode, workspace, s);
    if ((r = pair_run(ctx, ci, b, nbox, u, rho, c2, dt, nsteps / 2 * 2, mode, workspace, s, L)) || nsteps % 2 == 0)
        return r;
    // an odd last step with the per-stage kernels (same arithmetic)
    return level_stage_run(ctx, L, tile_heuristic(ctx, b, nbox), u, rho, c2, dt, 1,
                           mode == S4_GRAPH ? S4_BATCHED : mode, workspace, s);
}

int s4_copy(s4_ctx *ctx, void *dst, const void *src, size_t bytes, void *stream)
{
    if (!ctx || !dst || !src)
        return fail(S4_EINVAL, "NULL argument");
    if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return fail(S4_ELAYOUT, "copy needs 16-byte aligned pointers and size");
    if (overlap(dst, bytes, src, bytes))
        return fail(S4_EALIAS, "copy source and destination overlap");
    if (bytes == 0)
        return S4_OK;
    // one lane per 16 bytes; a launch holds fewer than 2^32 lanes
    if (bytes / 16 > (size_t)0xffffff00u)
        return fail(S4_EINVAL, "copy of %zu bytes exceeds one launch (64 GiB)", bytes);
    hipError_t e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "copy launch");
    return S4_OK;
}

// ---------------------------------------------------------------------------
// tuning

static void save_cache(s4_ctx *ctx);

int s4_tune(s4_ctx *ctx, int op, const s4_box *b, int nbox, int flags, void *scratch, size_t scratch_bytes,
            void *stream)
{
    if (!ctx)
        return fail(S4_EINVAL, "ctx is NULL");
    size_t need = 0;
    int r = s4_tune_scratch_size(b, nbox, op, &need);
    if (r)
        return r;
    bool with_c2 = false;
    split_op(op, with_c2);
    const int kop = kernel_op(op);
    if (kop < 0)
        return fail(S4_EINVAL, "op %d has no tunable kernel", op);
    if (!scratch || ((uintptr_t)scratch & 255))
        return fail(S4_ELAYOUT, "scratch must be non-NULL and 256-byte aligned");
    if (scratch_bytes < need)
        return fail(S4_ENOMEM, "scratch %zu bytes < %zu needed", scratch_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    S4_HIP(hipMemsetAsync(scratch, 0, need, s));
    const int nf = tune_fields(op, with_c2);
    std::vector<std::vector<double *>> F(nbox);
    size_t off = 0;
    for (int i = 0; i < nbox; ++i) {
        const size_t fb = field_bytes(b[i]);
        for (int k = 0; k < nf; ++k)
            F[i].push_back(ws_field((char *)scratch + off + k * fb, b[i]));
        off += (size_t)nf * fb;
    }
    char *tail = (char *)scratch + off; // box tables and counters (batched RK4)
    const double dt = 1e-9 * std::min({b[0].dx[0], b[0].dx[1], b[0].dx[2]});
    const int reps = flags & 1 ? 15 : 5;
    hipEvent_t e0, e1;
    S4_HIP(hipEventCreate(&e0));
    S4_HIP(hipEventCreate(&e1));
    // time candidate ci: the median of nrep timed calls after two warm-up calls
    auto time_cand = [&](int ci, int nrep, float &med) -> int {
        int r = S4_OK;
        const Cand &c = cands()[ci];
        // per candidate: what one call of the op launches, on scratch buffers
        std::vector<DevBox> tab;
        int64_t nitems = 0;
        DevBox *dtab = (DevBox *)tail;
        int *counters = (int *)(tail + round256(4 * (size_t)nbox * sizeof(DevBox)));
        const bool batched = op == S4_OP_RK4 && nbox > 1;
        if (op == S4_OP_RK4) {
            std::vector<double *> us(nbox), rs(nbox);
            std::vector<const double *> cs(nbox, nullptr);
            for (int i = 0; i < nbox; ++i) {
                us[i] = F[i][0];
                rs[i] = F[i][1];
                if (with_c2)
                    cs[i] = F[i][(size_t)nf - 1];
            }
            const double *const *c2a = with_c2 ? cs.data() : nullptr;
            // the RK4 workspace of box i is its fields 2..7, contiguous per box
            std::vector<char *> wsb(nbox);
            for (int i = 0; i < nbox; ++i)
                wsb[i] = (char *)F[i][2] - field_shift(b[i]);
            if (c.variant == 3 || c.variant == 4) {
                std::vector<PairFields> pfs;
                pair_tables(b, nbox, us.data(), rs.data(), c2a, wsb, c, tab, pfs);
                for (int i = 0; i < nbox; ++i)
                    nitems += dev_items(tab[(size_t)i]);
            } else {
                tab.assign(4 * (size_t)nbox, DevBox{});
                for (int i = 0; i < nbox; ++i) {
                    std::vector<DevBox> one;
                    double *ui[1] = {us[i]}, *ri[1] = {rs[i]};
                    const double *ci1[1] = {cs[i]};
                    rk4_tables(&b[i], 1, ui, ri, with_c2 ? ci1 : nullptr, wsb[i], c, one);
                    for (int st = 0; st < 4; ++st) {
                        one[st].item0 = (int)nitems;
                        tab[(size_t)st * nbox + i] = one[st];
                    }
                    nitems += dev_items(one[0]);
                }
            }
            if (batched) {
                std::vector<char> bytes(rk4_table_bytes(nbox), 0);
                memcpy(bytes.data(), tab.data(), tab.size() * sizeof(DevBox));
                if ((r = upload_table(dtab, bytes, s)))
                    return r;
            }
        }
        int rot = 0;
        const PairFields pf = op == S4_OP_RK4 ? pair_fields(b[0], (char *)F[0][2] - field_shift(b[0])) : PairFields{};
        auto run = [&]() -> int {
            const int set = rot++ % TUNE_SETS;
            switch (op) {
            case S4_OP_RK4:
                if (c.variant == 3 || c.variant == 4) // one step, alternating between (u, rho) and the ping-pong copy
                    return pair_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, set & 1, s, nullptr);
                if (c.variant == 1) // one fused step: (u, rho) -> ping-pong buffers, alternating
                    return rk4_pair_step(ctx, c, b[0], set & 1 ? pf.Up : F[0][0], set & 1 ? pf.Rp : F[0][1],
                                         set & 1 ? F[0][0] : pf.Up, set & 1 ? F[0][1] : pf.Rp,
                                         with_c2 ? F[0][(size_t)nf - 1] : nullptr, pf, dt, s);
                return rk4_step(ctx, c, tab, nbox, batched, dtab, counters, nitems, dt, s);
            case S4_OP_WAVE_RHS: {
                StageCoef K{};
                K.scale = 1.0;
                for (int i = 0; i < nbox; ++i) {
                    DevBox D = devbox(b[i], c);
                    D.in = F[i][2 * set];
                    D.q[0] = F[i][2 * set + 1];
                    int rr = launch_one(ctx, OP_RHS, c, D, K, s);
                    if (rr)
                        return rr;
                }
                return S4_OK;
            }
            case S4_OP_ADJOINT_RHS: {
                StageCoef K{};
                K.scale = 1.0;
                const int o = 5 * (set % 2);
                for (int i = 0; i < nbox; ++i) {
                    DevBox D = devbox(b[i], c);
                    D.in = F[i][o + 1];
                    D.inmul = F[i][o + 2];
                    D.p[0] = F[i][o];
                    D.q[0] = F[i][o + 3];
                    D.q[1] = F[i][o + 4];
                    int rr = launch_one(ctx, OP_ADJRHS, c, D, K, s);
                    if (rr)
                        return rr;
                }
                return S4_OK;
            }
            case S4_OP_ADJOINT_STEP: {
                const std::vector<double *> &G = F[0];
                return adjoint_step_launch(ctx, c, b[0], G[0], G[1], G[2], 1.0, G[3], G[4], G[5],
                                           (char *)G[6] - field_shift(b[0]), s);
            }
            case S4_OP_DERIV_MIXED: {
                const double A[9] = {1, 0.5, 0.25, 0.5, 1, 0.5, 0.25, 0.5, 1};
                MixArgs M = mix_args(b[0], c, A);
                const double *gin[TUNE_SETS];
                double *gout[TUNE_SETS];
                for (int k = 0; k < TUNE_SETS; ++k) {
                    gin[k] = F[0][k];
                    gout[k] = F[0][TUNE_SETS + k];
                }
                return launch_mixed_fields(ctx, c, M, TUNE_SETS, gin, gout, s);
            }
            default:
                return fail(S4_EINVAL, "op %d has no tunable kernel", op);
            }
        };
        for (int w = 0; w < 2 && !r; ++w)
            r = run();
        std::vector<float> ts;
        for (int k = 0; k < nrep && !r; ++k) {
            if (hipEventRecord(e0, s) != hipSuccess) {
                r = fail(S4_EDEVICE, "event record");
                break;
            }
            r = run();
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                r = r ? r : fail(S4_EDEVICE, "event sync");
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ts.push_back(ms);
        }
        if (r)
            return r;
        std::sort(ts.begin(), ts.end());
        med = ts[ts.size() / 2];
        return S4_OK;
    };
    std::vector<float> t(cands().size(), -1.0f);
    for (int ci = 0; ci < (int)cands().size() && !r; ++ci)
        if (cand_allowed(cands()[ci], op, nbox) && cand_fits(cands()[ci], b, nbox))
            r = time_cand(ci, reps, t[(size_t)ci]);
    // The candidates within 3 % of the fastest are timed again, interleaved,
    // in three rounds, each keeping its best median: settings a few per cent
    // apart are then not ranked by when in the sweep they ran (clocks and
    // temperature drift over it).
    if (!r) {
        float t0 = -1.0f;
        for (float x : t)
            if (x >= 0 && (t0 < 0 || x < t0))
                t0 = x;
        std::vector<int> close;
        for (int ci = 0; ci < (int)t.size(); ++ci)
            if (t[(size_t)ci] >= 0 && t[(size_t)ci] <= 1.03f * t0)
                close.push_back(ci);
        if (close.size() > 1)
            for (int round = 0; round < 3 && !r; ++round)
                for (int ci : close) {
                    float m = 0;
                    if ((r = time_cand(ci, reps, m)))
                        break;
                    t[(size_t)ci] = round == 0 ? m : std::min(t[(size_t)ci], m);
                }
    }
    int best = -1, best_level = -1;
    for (int ci = 0; ci < (int)t.size() && !r; ++ci) {
        if (t[(size_t)ci] < 0)
            continue;
        if (best < 0 || t[(size_t)ci] < t[(size_t)best])
            best = ci;
        if (level_capable(cands()[ci], LEVEL_NARROW) && (best_level < 0 || t[(size_t)ci] < t[(size_t)best_level]))
            best_level = ci;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r)
        return r;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        const std::string key = setup_key(ctx, op, b, nbox, with_c2);
        ctx->tuned[key] = best;
        // the same boxes as a level run the best level-capable setting
        if (op == S4_OP_RK4 && !with_c2 && nbox > 1 && best_level >= 0)
            ctx->tuned[key + LEVEL_SUFFIX] = best_level;
    }
    save_cache(ctx);
    return S4_OK;
}

// JSON cache: {"<setup key>": candidate index, ...}; keys contain no quotes.
// A candidate in the cache file: its parameters, "v<variant> x<tx> w<waves>
// z<chunk> r<rows>", so an entry keeps its meaning when the candidate list
// changes between builds.
static std::string cand_tag(const Cand &c)
{
    std::ostringstream o;
    o << "v" << c.variant << " x" << c.tx << " w" << c.nw << " z" << c.tz << " r" << c.ry;
    return o.str();
}

// index of the candidate with this tag, -1 if none
static int cand_from_tag(const std::string &tag)
{
    for (size_t i = 0; i < cands().size(); ++i)
        if (cand_tag(cands()[i]) == tag)
            return (int)i;
    return -1;
}

// Entries "key": "tag" of a cache file, mapped to candidate indices; entries
// whose value is not a string naming a current candidate (an index written
// by an older build, a candidate no longer built) are left out.
static std::map<std::string, int> parse_cache(const std::string &t)
{
    std::map<std::string, int> out;
    size_t p = 0;
    while ((p = t.find('"', p)) != std::string::npos) {
        const size_t q = t.find('"', p + 1);
        if (q == std::string::npos)
            break;
        const std::string key = t.substr(p + 1, q - p - 1);
        size_t v = t.find_first_not_of(" \t\r\n:", q + 1);
        if (v == std::string::npos)
            break;
        if (t[v] != '"') { // not a tag: skip to the next entry
            const size_t comma = t.find_first_of(",}", v);
            if (comma == std::string::npos)
                break;
            p = comma + 1;
            continue;
        }
        const size_t ve = t.find('"', v + 1);
        if (ve == std::string::npos)
            break;
        const int ci = cand_from_tag(t.substr(v + 1, ve - v - 1));
        if (ci >= 0)
            out[key] = ci;
        p = ve + 1;
    }
    return out;
}

static bool read_file(const std::string &path, std::string &out)
{
    std::ifstream f(path);
    if (!f)
        return false;
    std::stringstream ss;
    ss << f.rdbuf();
    out = ss.str();
    return true;
}

static void load_cache(s4_ctx *ctx)
{
    std::string t;
    if (!read_file(ctx->cache_path, t))
        return;
    for (auto &kv : parse_cache(t))
        ctx->tuned[kv.first] = kv.second;
}

static void save_cache(s4_ctx *ctx)
{
    if (ctx->cache_path.empty())
        return;
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::ofstream f(ctx->cache_path + ".tmp");
    f << "{\n";
    size_t k = 0;
    for (auto &kv : ctx->tuned)
        f << "  \"" << kv.first << "\": \"" << cand_tag(cands()[(size_t)kv.second]) << "\""
          << (++k < ctx->tuned.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    std::rename((ctx->cache_path + ".tmp").c_str(), ctx->cache_path.c_str());
}

int s4_tune_cache_lookup(const char *path, const char *device, int op, const s4_box *b, int nbox, int level,
                         int *candidate)
{
    if (!path || !device || !candidate)
        return fail(S4_EINVAL, "NULL argument");
    *candidate = -1;
    bool c2 = false;
    int r = split_op(op, c2);
    if (r)
        return r;
    if (kernel_op(op) < 0)
        return fail(S4_EINVAL, "op %d has no tunable kernel", op);
    if ((r = check_boxes(b, nbox, op)))
        return r;
    if (level && op != S4_OP_RK4)
        return fail(S4_EINVAL, "levels keep RK4 choices only");
    if (level < 0 || level > LEVEL_WIDE)
        return fail(S4_EINVAL, "level %d is not 0, 1 or 2", level);
    std::string t;
    if (!read_file(path, t))
        return fail(S4_EINVAL, "cannot read %s", path);
    const auto m = parse_cache(t);
    const std::string key = level_key(setup_key_on(device, op, b, nbox, c2), level);
    auto it = m.find(key);
    if (it != m.end() && cand_valid(it->second, op, b, nbox, level))
        *candidate = it->second;
    return S4_OK;
}

} // extern "C"
