/*
 * sten4.h -- C ABI of libsten4.so: FP64 4th-order finite-difference stencils,
 * classical RK4 and its discrete adjoint over the boxes of one refinement
 * level of a block-structured AMR grid, as hand-written HIP kernels for
 * gfx950 (MI355X).
 *
 * What the library models (Schnetter, "Performance and Optimization
 * Abstractions for Large Scale Heterogeneous Systems in the Cactus/Chemora
 * Framework"):
 *   - a refinement level is a set of non-overlapping boxes ("bboxset") on a
 *     uniform grid, each point at x0 + n*dx with integer n, and each box maps
 *     directly to an array in memory (Sec. II);
 *   - stencil loop kernels run over every box, reading ghost zones that hold
 *     copies of neighbouring points (Sec. II, II-A);
 *   - the loop over a box's index space declares its array alignment and
 *     padding, and is split into tiles, threads and vector lanes, with edge
 *     masks only at the box boundary (Sec. III-A, Sec. IV-C4 "Iterators").
 * The discrete operators are the textbook ones the paper leaves to the
 * application: 4th-order centred five-point differences, the classical RK4
 * tableau, and reverse-mode differentiation of that RK4 step.
 *
 * ---------------------------------------------------------------------------
 * Layout.  A field of a box is FP64, C order [z][y][x], x unit stride.  The
 * field pointer points at the ghost corner (-g,-g,-g); interior point
 * (i,j,k), 0 <= i < n[0] etc., lives at
 *     ptr + (i+g) + (j+g)*stride[1] + (k+g)*stride[2].
 * stride[0] must be 1, stride[1] >= n[0]+2g, stride[2] >= stride[1]*(n[1]+2g)
 * (padding allowed).  All fields of one box share its strides.  A row whose
 * interior start (ptr + g) is 128-byte aligned and whose stride[1] is a
 * multiple of 16 gives the fastest loads; any 8-byte aligned layout is valid.
 *
 * Memory ownership.  Every field, output and workspace buffer is device
 * memory owned by the caller; the library never allocates device memory for
 * data and never frees caller memory.  s4_box arrays and the 3x3 matrix A are
 * host memory, read during the call.  A context owns host-side tuning and
 * graph caches only.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Every call
 * is asynchronous and ordered on that stream, except that an s4_rk4 call on
 * more than one box in S4_BATCHED or S4_GRAPH mode copies its box table into
 * the caller's workspace and synchronises `stream` once before launching.
 *
 * Errors.  Each call returns S4_OK (0) or a negative code; the message of the
 * last failure on the calling thread is in s4_last_error().  Arguments are
 * validated on the host before anything is launched, so a failed call has
 * not touched device memory.  Device faults surface as S4_EDEVICE on a later
 * call.  No C++ exception crosses this ABI.
 * ---------------------------------------------------------------------------
 */
#ifndef STEN4_H
#define STEN4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define S4_OK 0
#define S4_EINVAL (-1)  /* null pointer, nbox <= 0, n < 1, dx <= 0, dt <= 0, nsteps < 0, bad op/mode */
#define S4_EGHOST (-2)  /* ghost width < 2 (the stencil radius), or periodic fill with n < g */
#define S4_ELAYOUT (-3) /* stride[0] != 1, strides too small, pointer not 8-byte aligned */
#define S4_EALIAS (-4)  /* an output overlaps an input that is read by a stencil */
#define S4_EDEVICE (-5) /* HIP runtime error (message in s4_last_error) */
#define S4_ENOMEM (-6)  /* workspace too small */
#define S4_ENOTSUP (-7) /* unsupported combination */

/* RK4 execution modes */
#define S4_PERBOX 0  /* per box and stage: one stage-kernel launch over that box's tiles */
#define S4_BATCHED 1 /* per stage: one persistent stage kernel over a (box, tile) queue of all boxes */
#define S4_GRAPH 2   /* S4_BATCHED with one RK4 step captured in a hipGraph, replayed nsteps times */

/* operation ids (workspace sizing, tuning, tile choice) */
#define S4_OP_FILL 1
#define S4_OP_WAVE_RHS 2
#define S4_OP_RK4 3
#define S4_OP_DERIV_MIXED 4
#define S4_OP_ADJOINT_RHS 5
#define S4_OP_ADJOINT_STEP 6
#define S4_OP_LEVEL_SYNC 7

/* ORed into S4_OP_RK4 for s4_tune, s4_tune_scratch_size, s4_get_choice and
 * s4_set_choice: the loop setup of RK4 calls that pass a variable c^2
 * (s4_rk4 with any c2[i] non-NULL, s4_rk4_step_to and s4_rk4_step_to_y3 with
 * c2 non-NULL).  It reads one more field per point and needs more registers,
 * so its tile choice is kept and tuned apart from that of the same boxes
 * without c^2 (Sec. III-B keys the tuning on the loop setup).  A choice
 * forced without this bit applies to both; a tuned one only to its own.
 * Levels (s4_level_rk4) keep one setup.  Any other op with it: S4_EINVAL. */
#define S4_WITH_C2 0x100

/* bboxset operations (s4_bset_op) */
#define S4_SET_UNION 0
#define S4_SET_INTERSECTION 1
#define S4_SET_DIFFERENCE 2
#define S4_SET_SYMDIFF 3

/* ghost-exchange shapes (s4_level_create) */
#define S4_SYNC_FULL 0  /* the whole ghost shell of the given width: faces, edges, corners */
#define S4_SYNC_FACES 1 /* only points beside a face (what axis-aligned stencils read) */

typedef struct s4_ctx s4_ctx;

/* One box: a bbox of one refinement level with its ghost zones (Sec. II). */
typedef struct {
    int32_t n[3];      /* interior points along x, y, z (>= 1) */
    int32_t ghost;     /* ghost width g on every face (>= 2) */
    int64_t stride[3]; /* element strides along x, y, z; stride[0] == 1 */
    double dx[3];      /* grid spacing along x, y, z (> 0) */
    int32_t level;     /* refinement level (informational only) */
    int32_t reserved;  /* set to 0 */
} s4_box;

/* Create a context bound to HIP device `device`.  Reads the device's
 * properties (CU count, XCD count, name), which seed the default tile
 * choice.  The environment variable S4_TUNE_CACHE names a JSON file of tuned
 * choices that is read here and rewritten by s4_tune: one object mapping a
 * loop-setup key to the parameters of the chosen candidate,
 *   "op<op>|<device>|<nbox>|<nx>,<ny>,<nz>,g<ghost>,s<stride1>,<stride2>
 *    (one such group per box)[|c2][|level or |level4]": "v<variant> x<tx> w<waves>
 *    z<z chunk> r<rows>".
 * Entries that name no candidate of this build, or a candidate the setup's
 * op cannot run on its boxes, are ignored (the heuristic applies). */
int s4_create(int device, s4_ctx **out);

/* Free the context's host caches and captured graphs.  NULL is ignored. */
void s4_destroy(s4_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *s4_last_error(void);

/* Validate box descriptors for `op` on the host; no device call is made.
 * Returns S4_OK or the code the corresponding entry point would return. */
int s4_check_boxes(const s4_box *b, int nbox, int op);

/* Bytes of workspace that `op` (S4_OP_RK4 or S4_OP_ADJOINT_STEP) in `mode`
 * needs for these boxes; 0 for operations that need none. */
int s4_workspace_size(const s4_box *b, int nbox, int op, int mode, size_t *bytes);

/* Periodic ghost fill (each box is its own periodic neighbour).  For every
 * ghost point (i,j,k) of box b, f = f(i mod n0, j mod n1, k mod n2): the
 * result of copying faces along x, then y (over the full x extent), then z
 * (over the full x and y extents), so edges and corners are filled.  The
 * paper fills ghost zones by communication between the boxes of a level
 * (Sec. II); one self-periodic box is the degenerate case.  f[i] is the
 * field of box i; requires n >= g on every axis (S4_EGHOST otherwise). */
int s4_fill_ghosts_periodic(s4_ctx *ctx, const s4_box *b, int nbox, double *const *f, void *stream);

/* Wave-equation right-hand side in first-order form, y = (u, rho):
 *   u_t = rho (returned as an alias: nothing is written),
 *   rho_t = c^2 (L u),  L = D2_x + D2_y + D2_z,
 *   D2 f_i = (-f_{i-2} + 16 f_{i-1} - 30 f_i + 16 f_{i+1} - f_{i+2}) / (12 h^2).
 * u's ghosts must be filled (they are read, never written).  c2 == NULL, or
 * c2[i] == NULL, means c = 1 for that box; c2 is read at interior points only
 * and uses the box layout.  rho_t[i] is written at interior points only and
 * must not overlap u[i] (S4_EALIAS).  The stencil follows the paper's loop
 * kernels over a box with ghost zones (Sec. III-A, IV-C4). */
int s4_wave_rhs(s4_ctx *ctx, const s4_box *b, int nbox, const double *const *u,
                const double *const *c2, double *const *rho_t, void *stream);

/* Multi-field derivative kernel on one box, for each field f = g[k]:
 *   out[k] = sum_a D2_a f + sum_{a<b} D_ab f + sum_{a,b} A[3a+b] (D1_a f)(D1_b f),
 *   D1 f_i = (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 h),
 *   D_ab f = sum_{p,q=-2..2} w_p w_q f(x + p e_a + q e_b) / (144 h_a h_b),
 *   w = (1, -8, 0, 8, -1)  (the tensor product of two D1 stencils).
 * Axes a, b in {x, y, z} = {0, 1, 2}; A is host memory, row major, used as
 * given.  Ghosts of every g[k] must be filled including edges (the mixed
 * terms read them).  out[k] is written at interior points only and must not
 * overlap any g[j].  Definition: the textbook 4th-order centred first and
 * second differences (the paper leaves the discretisation to the
 * application code; it prints only a 2nd-order example loop in Sec. IV-C4),
 * with the mixed derivative read as the tensor product of two first
 * differences.  The loop over the box is the tiled traversal of Sec. III-A
 * with the aligned, padded iteration of Sec. IV-C4. */
int s4_deriv_mixed(s4_ctx *ctx, const s4_box *b, int nfield, const double *const *g,
                   const double A[9], double *const *out, void *stream);

/* Advance the wave equation on every box by nsteps classical RK4 steps:
 *   k1 = F(y_n), k2 = F(y_n + dt/2 k1), k3 = F(y_n + dt/2 k2), k4 = F(y_n + dt k3),
 *   y_{n+1} = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4),
 * with F the RHS above and a periodic ghost fill of the stage u before every
 * F.  The box is its own periodic neighbour: the stage kernels read stencil
 * neighbours at wrapped indices, which equals a periodic ghost fill before
 * every F without the fill's launches.  u[i], rho[i] are updated in place at
 * interior points; their ghosts are neither read nor written.  The kernel
 * set (one kernel per stage, two stages per pass, or a whole step per pass
 * on a tile widened by 2 points each side) is the context's choice for the
 * loop setup (s4_get_choice); all give the same values bit for bit.
 * c2 as in s4_wave_rhs.  `workspace` is device memory of at least
 * s4_workspace_size(b, nbox, S4_OP_RK4, mode) bytes, 256-byte aligned, owned
 * by the caller and not used by anything else while the call's work runs.
 * Definition: Kutta's classical RK4 tableau (textbook; the paper names no
 * time integrator) over the wave RHS above.  The stage kernels are the
 * traversal of Sec. III-A; the stage-pair and whole-step sets fuse stages
 * into one loop, the loop fusion the paper proposes as future work
 * (Sec. III-C); S4_BATCHED runs every box of the set in one launch that
 * hands out work items at run time, as LoopControl assigns loop regions to
 * threads on the fly to balance uneven cost (Sec. III).
 * mode: S4_PERBOX, S4_BATCHED or S4_GRAPH.  S4_GRAPH caches one captured
 * step per (boxes, pointers, dt, workspace) in the context; the cache entry
 * is invalid once any of those buffers is freed (s4_destroy drops it). */
int s4_rk4(s4_ctx *ctx, const s4_box *b, int nbox, double *const *u, double *const *rho,
           const double *const *c2, double dt, int nsteps, int mode, void *workspace,
           size_t ws_bytes, void *stream);

/* Bytes of the device scratch array behind s4_rk4_noalloc (one per device,
 * held from the library's first use on that device until the process ends). */
#define S4_NOALLOC_SCRATCH_BYTES (128u << 20)

/* s4_rk4 for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is the library's own static scratch array of
 * S4_NOALLOC_SCRATCH_BYTES on the context's device instead of a caller
 * buffer, and the call allocates nothing (no hipMalloc, hipFree, graph
 * instantiation or timing events).  Same arguments, results and kernel sets
 * as s4_rk4 with mode S4_PERBOX or S4_BATCHED; S4_GRAPH gives S4_ENOTSUP.
 * Boxes whose s4_workspace_size exceeds S4_NOALLOC_SCRATCH_BYTES give
 * S4_ENOMEM before anything is launched (one box of up to 128^3 interior
 * points with 2 ghosts fits).  Every call on one device shares that
 * device's array: calls that overlap on one device, on any streams or
 * contexts, race and give undefined results; the array keeps the last
 * call's contents, and everything a call needs zeroed it clears itself.
 * The on-line tuner is not advanced (the current choice of the loop setup
 * runs). */
int s4_rk4_noalloc(s4_ctx *ctx, const s4_box *b, int nbox, double *const *u, double *const *rho,
                   const double *const *c2, double dt, int nsteps, int mode, void *stream);

/* One RK4 step of s4_rk4 on one periodic box, out of place: reads
 * (u_in, rho_in), writes (u_out, rho_out) at interior points; the inputs are
 * not modified and must not overlap the outputs (S4_EALIAS).  Gives the same
 * values as s4_rk4 on a copy of the inputs.  For recomputing the states of a
 * checkpointed segment during backpropagation.  c2 and the workspace as for
 * s4_rk4 (S4_OP_RK4 on this machine).  Definition: one step of the classical RK4
 * tableau of s4_rk4 (textbook); traversal Sec. III-A, fused as Sec. III-C. */
int s4_rk4_step_to(s4_ctx *ctx, const s4_box *b, const double *u_in, const double *rho_in, const double *c2,
                   double dt, double *u_out, double *rho_out, void *workspace, size_t ws_bytes, void *stream);

/* s4_rk4_step_to that also returns the step's third stage state
 * y_3 = y_n + dt/2 k_2 of classical RK4 (u3_out, rho3_out: interior points,
 * in the box's layout, ghosts not written), the forward state the backward
 * step reads (s4_rk4_adjoint_step_y3).  (u_out, rho_out) are bit for bit
 * those of s4_rk4_step_to, and y_3 bit for bit the value every RK4 kernel
 * set forms.  u3_out and rho3_out must not be NULL (S4_EINVAL) and must not
 * overlap the inputs, the other outputs or the workspace (S4_EALIAS).
 * Runs the current tile choice for S4_OP_RK4 on this machine when it is a
 * stage-pair or whole-step set (the per-stage sets give way to the stage
 * pairs), without a trial or timing of the on-line tuner.  Workspace as for
 * s4_rk4_step_to. */
int s4_rk4_step_to_y3(s4_ctx *ctx, const s4_box *b, const double *u_in, const double *rho_in, const double *c2,
                      double dt, double *u_out, double *rho_out, double *u3_out, double *rho3_out,
                      void *workspace, size_t ws_bytes, void *stream);

/* Adjoint (transpose) of the wave RHS as a linear map of interior values,
 * for periodic boxes:
 *   F^T(lu, lrho) = (L_p(c^2 lrho), lu),
 * where L_p is "periodic ghost fill, then L", a symmetric operator.  out_u
 * receives L_p(c^2 lrho): the kernel forms c^2*lrho at each interior point and
 * reads lrho (and c2) at periodically wrapped indices, so lrho's ghosts are
 * not read.  out_rho receives a copy of lu.  Interior points only.
 * Definition: the transpose of the linear map of s4_wave_rhs on periodic
 * boxes (textbook linear algebra; the paper has no adjoint), in which the
 * periodic 4th-order Laplacian is symmetric.  Traversal as Sec. III-A. */
int s4_wave_adjoint_rhs(s4_ctx *ctx, const s4_box *b, int nbox, const double *const *lu,
                        const double *const *lrho, const double *const *c2,
                        double *const *out_u, double *const *out_rho, void *stream);

/* One backward RK4 step on one periodic box (reverse-mode differentiation
 * of s4_rk4's step):
 *   kb4 = dt/6 ybar;              yb4 = F^T kb4
 *   kb3 = dt/3 ybar + dt   yb4;   yb3 = F^T kb3
 *   kb2 = dt/3 ybar + dt/2 yb3;   yb2 = F^T kb2
 *   kb1 = dt/6 ybar + dt/2 yb2;   yb1 = F^T kb1
 *   ybar_n = ybar + yb1 + yb2 + yb3 + yb4
 *   c2_bar += sum_s (kb_s)_rho * (L_p u_s)
 * u_n, rho_n: the forward state at the start of the step (with c2_bar, the
 * stage states u_3, rho_3 are recomputed from it and u_2, u_4 are formed at
 * each stencil tap, with periodic addressing; ghosts of u_n are not read and
 * u_n, rho_n are not modified).  The step runs as two passes: adjoint stages
 * 4 and 3, then 2 and 1, each stencilling c^2 kb_rho formed at every tap.  lam_u, lam_rho: on entry
 * ybar = dJ/dy_{n+1}, on return dJ/dy_n (interior).  c2_bar, if not NULL,
 * is accumulated into at interior points; c2 == NULL means c = 1.
 * Workspace as for s4_rk4 with S4_OP_ADJOINT_STEP.  Definition: reverse-mode
 * differentiation of one classical RK4 step (textbook; the paper has no
 * adjoint): the step is linear in y, so its transpose is the same tableau
 * applied with the transposed RHS of s4_wave_adjoint_rhs in reverse stage
 * order.  Traversal Sec. III-A; two stages per pass as Sec. III-C's fusion. */
int s4_rk4_adjoint_step(s4_ctx *ctx, const s4_box *b, const double *u_n, const double *rho_n,
                        const double *c2, double dt, double *lam_u, double *lam_rho,
                        double *c2_bar, void *workspace, size_t ws_bytes, void *stream);

/* s4_rk4_adjoint_step given the step's third stage state (u3, rho3), as
 * s4_rk4_step_to_y3 returns it, instead of recomputing it: with c2_bar the
 * step then runs its two adjoint passes only.  Results are bit for bit
 * those of s4_rk4_adjoint_step when (u3, rho3) came from s4_rk4_step_to_y3
 * on (u_n, rho_n) with the same c2 and dt.  u3 and rho3 are read (interior
 * points, with periodic addressing) only when c2_bar is not NULL; they are
 * required then (S4_EINVAL) and may be NULL otherwise.  They must not
 * overlap lam_u, lam_rho, c2_bar or the workspace (S4_EALIAS).  Workspace
 * as for s4_rk4_adjoint_step. */
int s4_rk4_adjoint_step_y3(s4_ctx *ctx, const s4_box *b, const double *u_n, const double *rho_n,
                           const double *u3, const double *rho3, const double *c2, double dt,
                           double *lam_u, double *lam_rho, double *c2_bar, void *workspace,
                           size_t ws_bytes, void *stream);

/* Time the candidate tile shapes and kernel variants of `op` on these boxes
 * (median of hipEvent timings after warm-up; the candidates within 3 % of
 * the fastest are timed again, interleaved, in three rounds, each keeping
 * its best median; ties to the lowest candidate index) and keep the
 * fastest for this "loop setup": the op, box sizes,
 * ghost width, strides and alignment, and device (the key the paper's
 * LoopControl tunes per loop setup, Sec. III-B).  Scratch buffers are
 * taken from `scratch` (device memory of at least s4_tune_scratch_size
 * bytes); the caller's data are not touched.  flags: 0 = quick sweep,
 * 1 = full sweep.  op S4_OP_RK4 | S4_WITH_C2 times the step with a c^2
 * field in scratch and keeps the choice for calls that pass c^2.
 * Persists to S4_TUNE_CACHE when set.  For RK4 on several
 * boxes it also keeps the fastest candidate that can run on a level
 * (s4_level_choice), for the same boxes coupled as a level. */
int s4_tune(s4_ctx *ctx, int op, const s4_box *b, int nbox, int flags, void *scratch,
            size_t scratch_bytes, void *stream);

/* Host-only reading of a tuning cache file in the S4_TUNE_CACHE format:
 * *candidate = the candidate index a context on device `device` (its
 * architecture name, e.g. "gfx950") would take from that file for `op`
 * (with S4_WITH_C2 for RK4 calls that pass c^2) on these boxes, as a level
 * (level 1; level 2: a wide level, see s4_level_rk4) or not (level 0), or
 * -1 when the file holds no usable entry for that setup.  S4_EINVAL if the
 * file cannot be read.  No device call. */
int s4_tune_cache_lookup(const char *path, const char *device, int op, const s4_box *b, int nbox, int level,
                         int *candidate);

/* Scratch bytes s4_tune needs for these boxes. */
int s4_tune_scratch_size(const s4_box *b, int nbox, int op, size_t *bytes);

/* The tile choice the library would use for `op` on box b (or on the set):
 * out[0] variant id, out[1] tile x, out[2] tile y, out[3] z chunk,
 * out[4] threads per workgroup, out[5] 1 if it came from s4_tune, 2 if
 * on-line tuning is active,
 * out[6] candidate index (with on-line tuning: the best setting so far),
 * out[7] one past the last candidate index this op may use on these boxes
 * (the op uses those of 0 .. out[7]-1 that s4_set_choice accepts; RK4 uses
 * all of them, the wave RHS skips the RK4-only sets).  out[0] is 100 or 101 when the
 * choice is one of RK4's two fused stage-pair kernel sets (widened tile,
 * per-tap second stage), 102 when it is the whole-step kernel set (one
 * launch per RK4 step on a tile widened by 4 points in total along x and y),
 * 200 + the kernel op when it is
 * the row-register kernel set (out[1] is then the item's x extent, 64 per
 * wavefront along x, and out[2] its y extent), and 300 + the kernel op when
 * it is the pair-lane tile set of the wave RHS (two x points per lane;
 * out[1] is the tile's x extent in points; boxes with an even n[0] and even
 * strides; a call whose fields' interior rows are not 16-byte aligned runs
 * the same shape on the one-point tiles). */
int s4_get_choice(s4_ctx *ctx, int op, const s4_box *b, int nbox, int out[8]);

/* Force a candidate (index into the op's candidate list) for this loop
 * setup, or -1 to drop the forced choice.  For tests that compare
 * candidates bit for bit, and for benchmark sweeps.  S4_ENOTSUP for a
 * candidate the op cannot use on these boxes (out[7] of s4_get_choice
 * bounds them; the whole-step kernels also need z planes below 2 GiB, the
 * pair-lane tiles an even n[0] and even strides). */
int s4_set_choice(s4_ctx *ctx, int op, const s4_box *b, int nbox, int candidate);

/* On-line tuning: the paper's run-time random-restart hill climbing
 * (Sec. III-B).  With enable != 0 every call of an op times its own launches
 * with HIP events (read back at a later call, never waited for) and the tile
 * choice of its loop setup moves: the neighbourhood of the best setting so
 * far is tried one setting per call, the best moves to any faster
 * neighbour, and once no neighbour is left a random setting is tried with
 * probability restart_prob per call (then its neighbourhood), abandoned after
 * one call if it is more than 1.5x slower than the best.  seed seeds the
 * random restarts.  A forced choice (s4_set_choice) is never changed; a
 * tuned one (s4_tune) is the starting point.  S4_TUNE=online in the
 * environment enables it at s4_create with restart_prob 0.02. */
int s4_set_online_tuning(s4_ctx *ctx, int enable, double restart_prob, uint64_t seed);

/* Host-only simulation of the on-line tuner for one loop setup of `op` on
 * these boxes, for testing its search: cost[i] is the time of candidate i
 * (ncost = the number of candidates), each timing is perturbed by a factor
 * in [1 - noise, 1 + noise] from a seeded generator and reaches the tuner
 * `lag` calls after the call it times (as device timings do).  Writes the
 * candidate used at each of the ncalls calls to trace.  No device call. */
int s4_online_simulate(int op, const s4_box *b, int nbox, const double *cost, int ncost, double noise,
                       double restart_prob, uint64_t seed, int lag, int ncalls, int *trace);

/* ---------------------------------------------------------------------------
 * bboxsets (Sec. II-B, II-C).  A bboxset is a set of points of the integer
 * grid Z^dim, dim = 1, 2 or 3, held on the host as its discrete derivative:
 * along the last axis, the coordinates where the (dim-1)-dimensional
 * cross-section changes and each change (the xor of the sections on both
 * sides), recursively down to single booleans.  The derivative is the
 * leftward mod-2 difference d_a R(p) = R(p) xor R(p - e_a); the set is
 * recovered by xor-scanning each axis from low to high coordinates.  The
 * fully unrolled derivative d_0 d_1 ... R of one bbox is its 2^dim corners
 * (8 for a cuboid); an L-shaped 2D region has 6.  These "key points" are
 * what is stored.  Set operations sweep the last axis as in the paper's
 * traversal algorithm (Fig. 2) and recurse on cross-sections.
 *
 * Boxes are half-open: box k of an array spans lo[k*dim + a] <= p[a] <
 * hi[k*dim + a]; a box with hi <= lo on any axis is empty.  Coordinates must
 * satisfy |c| <= 2^40.  Handles are owned by the caller and freed with
 * s4_bset_free; every function leaves its inputs unchanged and returns
 * S4_OK or S4_EINVAL (NULL argument, bad dim/op/axis, coordinate out of
 * range, mismatched dims, a point count beyond int64).  No device call. */
typedef struct s4_bset s4_bset;

/* The union of nbox boxes (nbox == 0: the empty set). */
int s4_bset_from_boxes(int dim, const int64_t *lo, const int64_t *hi, int64_t nbox, s4_bset **out);

/* Free a set; NULL is ignored. */
void s4_bset_free(s4_bset *s);

/* out = a op b, op one of S4_SET_UNION, S4_SET_INTERSECTION,
 * S4_SET_DIFFERENCE (a minus b), S4_SET_SYMDIFF. */
int s4_bset_op(int op, const s4_bset *a, const s4_bset *b, s4_bset **out);

/* out = a moved by the vector v (dim entries): p in out iff p - v in a. */
int s4_bset_shift(const s4_bset *a, const int64_t *v, s4_bset **out);

/* out = every point of a grown by lo[k] points downward and hi[k] upward
 * along axis k (lo, hi >= 0, <= 2^20): the Minkowski sum with [-lo, hi]. */
int s4_bset_expand(const s4_bset *a, const int64_t *lo, const int64_t *hi, s4_bset **out);

/* out = d_axis a = a xor (a moved by +e_axis). */
int s4_bset_derivative(const s4_bset *a, int axis, s4_bset **out);

/* info[0] dim, info[1] number of points, info[2] number of key points (of
 * the full derivative), info[3] number of boxes s4_bset_boxes returns. */
int s4_bset_info(const s4_bset *a, int64_t info[4]);

/* The key points, dim coordinates each, in lexicographic order of
 * (last axis, ..., axis 0); writes min(count, max) points to out and the
 * total to *count. */
int s4_bset_keys(const s4_bset *a, int64_t *out, int64_t max, int64_t *count);

/* Pairwise disjoint boxes whose union is a (one run of boxes per interval
 * of constant cross-section along the last axis, recursively); writes
 * min(count, max) boxes to lo/hi (dim entries each) and the total to *count. */
int s4_bset_boxes(const s4_bset *a, int64_t *lo, int64_t *hi, int64_t max, int64_t *count);

/* *out = 1 if point p (dim entries) is in a, else 0. */
int s4_bset_contains(const s4_bset *a, const int64_t *p, int *out);

/* *out = 1 if a and b hold the same points (same dim), else 0. */
int s4_bset_equal(const s4_bset *a, const s4_bset *b, int *out);

/* ---------------------------------------------------------------------------
 * One refinement level as a set of boxes that fill each other's ghost zones
 * (Sec. II: ghost zones hold copies of neighbouring points; on one level
 * they come from the boxes beside them).  Box i's interior occupies the
 * global index range [lo[3i+a], lo[3i+a] + b[i].n[a]) on axis a; interiors
 * must not overlap and all boxes share one grid spacing.  domain[a] > 0
 * makes axis a periodic with that extent (every box then lies inside
 * [0, domain[a]) and a point p stands for p mod domain[a]); domain[a] == 0
 * leaves it open (ghost points beyond the level stay uncovered, for the
 * physical boundary or a coarser level to fill).
 *
 * s4_level_create builds, on the host, the exchange schedule of `width`
 * ghost layers (1 <= width <= every box's ghost) in shape S4_SYNC_FULL or
 * S4_SYNC_FACES with the bboxset algebra: per box, the ghost region it needs
 * (the grown interior minus the interior), intersected with every other
 * box's interior and its periodic images, cut into disjoint copy pieces.
 * Returns S4_EINVAL for inconsistent boxes (overlap, outside the periodic
 * domain, spacings differ, width > a periodic extent), S4_EGHOST for a
 * width outside [1, ghost], and the codes of s4_check_boxes.  The level is
 * a host object owned by the caller (s4_level_destroy); it keeps copies of
 * the boxes and origins. */
typedef struct s4_level s4_level;

int s4_level_create(const s4_box *b, const int64_t *lo, int nbox, const int64_t domain[3], int width, int shape,
                    s4_level **out);

void s4_level_destroy(s4_level *L);

/* info[0] boxes, info[1] copy pieces, info[2] ghost points the exchange
 * fills, info[3] ghost points of the requested shape that no box covers,
 * info[4] interior points of the level, info[5] width, info[6] shape. */
int s4_level_info(const s4_level *L, int64_t info[7]);

/* The copy pieces: 11 int64 each, (dst box, src box, dst start x y z, src
 * start x y z, extent x y z), starts in box-local interior coordinates
 * (negative = ghost).  Writes min(count, max) pieces and the total to *count. */
int s4_level_pieces(const s4_level *L, int64_t *out, int64_t max, int64_t *count);

/* Workspace bytes of s4_level_sync (op S4_OP_LEVEL_SYNC) or s4_level_rk4
 * (op S4_OP_RK4, any mode). */
int s4_level_workspace_size(const s4_level *L, int op, size_t *bytes);

/* Fill the ghost points of field f[i] of every box i by the level's
 * schedule: each gets the value at the same grid point (periodically
 * wrapped) in the interior of the box that owns it; ghost points no box
 * covers are left as they are.  One kernel launch; interiors are only read.
 * f[i] use box i's layout and must not overlap each other.  The schedule
 * is copied into the caller's workspace (>= s4_level_workspace_size bytes,
 * 256-byte aligned) and `stream` is synchronised once before the launch. */
int s4_level_sync(s4_ctx *ctx, const s4_level *L, double *const *f, void *workspace, size_t ws_bytes,
                  void *stream);

/* s4_rk4 on a level whose boxes are coupled through their ghost zones:
 * before every evaluation of F the stage's u is exchanged by the level's
 * schedule (which must cover every ghost point of its shape: S4_EGHOST
 * otherwise, and have width >= 2), then the stage kernels read stencil
 * neighbours from the ghost zones.  On a periodic level that tiles its
 * domain the result equals s4_rk4 on one box spanning the domain.  The
 * ghost points of u and rho are overwritten by the exchanges (the stage-pair
 * kernel set exchanges both before its first pass); everything else as for
 * s4_rk4 (modes, c2, in-place update, graph cache keyed additionally by
 * the schedule).  On a wide level -- a schedule of shape S4_SYNC_FULL and
 * width >= 4 over boxes with ghost >= 4 -- the whole-step kernel set also
 * runs: one exchange of u and rho per step fills the ghost shell, from
 * which a step reads its radius-4 neighbourhood (ghost zones deep enough to
 * skip the exchanges between stages; Sec. II fills ghost zones by
 * communication within a level, Sec. III-C proposes the loop fusion). */
int s4_level_rk4(s4_ctx *ctx, const s4_level *L, double *const *u, double *const *rho, const double *const *c2,
                 double dt, int nsteps, int mode, void *workspace, size_t ws_bytes, void *stream);

/* The tile choice s4_level_rk4 uses on this level, laid out as
 * s4_get_choice's out[] (out[7]: the candidates RK4 may use on these
 * boxes).  A level runs only kernel sets whose stencils read what its
 * exchange fills: radius-2 ghost zones, or on a wide level (see
 * s4_level_rk4) the radius-4 neighbourhood of the whole steps.  A forced or
 * tuned choice for the boxes that needs more (the widened-tile stage pairs,
 * out[0] 100, always; the whole steps, 102, on other levels) is replaced by
 * the fastest level-capable candidate s4_tune found, else by the heuristic
 * start, which is the whole steps on a wide level.  Sec. III-B (a loop
 * setup's execution parameters). */
int s4_level_choice(s4_ctx *ctx, const s4_level *L, int out[8]);

/* Plain device copy of `bytes` bytes (a multiple of 16, 16-byte aligned,
 * at most 64 GiB: S4_EINVAL beyond): the streaming-copy probe that
 * calibrates achievable HBM bandwidth and the byte counters against a
 * kernel of known traffic.  One lane per 16 bytes, in a single pass over
 * the buffers (non-temporal loads and stores). */
int s4_copy(s4_ctx *ctx, void *dst, const void *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* STEN4_H */
