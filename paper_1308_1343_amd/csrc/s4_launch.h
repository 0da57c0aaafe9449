// s4_launch.h -- launchers exported by s4_kernels.hip to the host side.
#pragma once

#include <hip/hip_runtime.h>

#include "s4_internal.h"

namespace s4 {

// One box, one workgroup per work item (grid = nitems); nxcd > 1 spreads
// contiguous item ranges over the XCDs.  ghosted: OP_STAGE reads stencil
// neighbours from the stencil input's ghost zones instead of wrapping.
hipError_t launch_tiles_single(int op, int tx, int nw, const DevBox &B, const StageCoef &K, int nitems,
                               int nxcd, hipStream_t s, bool ghosted = false);

// All boxes of a device table in one persistent launch of `grid` workgroups
// over the per-XCD work queue Q (its 1 + Q.nq counters must be zero before
// the first launch; each launch leaves them zero).
hipError_t launch_tiles_batched(int op, int tx, int nw, const DevBox *tab, int nbox, const ItemQueue &Q,
                                int grid, const StageCoef &K, hipStream_t s, bool ghosted = false);

// Resident workgroups per CU of the batched kernel for this shape (0 if unknown).
int max_blocks_per_cu(int op, int tx, int nw, bool ghosted = false);

// Row-register kernels (4 wavefronts: wx along x times 4/wx along y, ry rows
// each) for OP_RHS and OP_STAGE, single box and persistent batched forms.
hipError_t launch_rows_single(int op, int wx, int ry, const DevBox &B, const StageCoef &K, int nitems, int nxcd,
                              hipStream_t s, bool ghosted = false);
hipError_t launch_rows_batched(int op, int wx, int ry, const DevBox *tab, int nbox, const ItemQueue &Q,
                               int grid, const StageCoef &K, hipStream_t s, bool ghosted = false);
int max_blocks_rows(int op, int wx, int ry, bool ghosted = false);

// Wave RHS (OP_RHS, ghosts read) on pair-lane tiles: txl lanes of two x
// points each along x, nw wavefronts.  Needs an even n[0], even strides and
// 16-byte aligned interior row starts of every field.
hipError_t launch_pairs_rhs(int txl, int nw, const DevBox &B, int nitems, int nxcd, hipStream_t s);

// Multi-field mixed-derivative kernel over fields [0, nfield) of M (nfield <= 8);
// one workgroup per (field, tile) item.
hipError_t launch_mixed(int tx, int nw, const MixArgs &M, int nfield, int nxcd, hipStream_t s);

// One fused pair of RK4 stages (pair 0: stages 1-2, pair 1: stages 3-4) on box
// B: workgroups of txe x (nw*64/txe) lanes, output tiles of (txe-4) x (tye-4).
hipError_t launch_rk4_pair(int pair, int txe, int nw, const DevBox &B, const StageCoef &K1, const StageCoef &K2,
                           int nitems, int nxcd, hipStream_t s);

// One whole RK4 step on box B in one pass (periodic addressing): workgroups
// of txe x (nw*64/txe) lanes, output tiles of (txe-4) x (tye-4) (B.tiles[0..1]
// counts them).  run = 0: one workgroup per work item (tile, z chunk of
// B.tz planes); run > 0: each workgroup runs `run` planes of the box's
// tile-plane sequence (run_piece).  B.in, p[0], p[5]: u_n, rho_n, c^2
// (optional); q[0], q[1]: u_{n+1}, rho_{n+1}, which must not alias the
// inputs.  K: the coefficients of stages 1..4.  hipErrorInvalidValue for
// z planes of 2 GiB or more.  ghosted: stencil neighbours from the ghost
// zones (a level after an exchange of width 4; needs B.g >= 4, no y_3)
// instead of wrapped indices.
hipError_t launch_rk4_step4(int txe, int nw, const DevBox &B, const StageCoef K[4], int run, int nxcd,
                            hipStream_t s, bool ghosted = false);
// persistent form over a table of boxes (queue as launch_tiles_batched);
// hasc2: some box may have c^2 (p[5], null for the others).  The caller
// checks that no box has a z plane of 2 GiB or more, and with ghosted that
// every box has ghost width 4 or more.
hipError_t launch_rk4_step4_batched(int txe, int nw, bool hasc2, const DevBox *tab, int nbox, const ItemQueue &Q,
                                    int grid, const StageCoef K[4], hipStream_t s, bool ghosted = false);
// resident workgroups per CU of the whole-step kernels (0 if unknown)
int max_blocks_step4(int txe, int nw);

// Two RK4 stages per pass on the plain tile (pair 0: stages 1-2, pair 1:
// stages 3-4), workgroups of tx x (nw*64/tx) lanes, one output point each;
// periodic addressing, or ghost addressing when ghosted.
hipError_t launch_pair2(int pair, int tx, int nw, const DevBox &B, const StageCoef &K1, const StageCoef &K2,
                        int nitems, int nxcd, hipStream_t s, bool ghosted = false);
// persistent form over a table of boxes (queue as launch_tiles_batched)
hipError_t launch_pair2_batched(int pair, int tx, int nw, const DevBox *tab, int nbox, const ItemQueue &Q,
                                int grid, const StageCoef &K1, const StageCoef &K2, hipStream_t s,
                                bool ghosted = false);
int max_blocks_pair2(int pair, int tx, int nw, bool ghosted = false);

// One pass (0: adjoint stages 4-3, 1: stages 2-1) of the two-pass backward
// RK4 step on one periodic box; c2bar: accumulate dJ/dc^2.
hipError_t launch_adj2(int pass, int tx, int nw, bool c2bar, const DevBox &B, const StageCoef &K, int nitems,
                       int nxcd, hipStream_t s);

// Periodic ghost fill of the field q[0] of box B (one thread per ghost point).
hipError_t launch_fill(const DevBox &B, hipStream_t s);

// Level ghost exchange over nblocks workgroups of 256 threads: W[b] is the
// piece (in device table P) that workgroup b copies; F is a device table of
// nf x nbox field pointers (field-major), every field exchanged alike.
hipError_t launch_sync(const SyncPiece *P, const int *W, double *const *F, int nf, int nbox, int nblocks,
                       hipStream_t s);

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

// Device address, on the current device, of the scratch array of
// s4_rk4_noalloc (S4_NOALLOC_SCRATCH_BYTES, 256-byte aligned); looked up once
// per device.
hipError_t noalloc_scratch(void **ptr);

} // namespace s4
