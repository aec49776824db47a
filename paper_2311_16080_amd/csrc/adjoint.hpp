// adjoint.hpp -- internal interface of the adjoint kernels (not public ABI).
#pragma once
#include "batch.hpp"

namespace lbm {

enum : int { ADJ_STEP = 0, ADJ_SEED = 1, ADJ_MATERIALIZE = 2, ADJ_DS_OUT = 3, ADJ_WALLS = 4, ADJ_DF_OUT = 5 };

// Tiles of moving-wall face cells: tile k = cells [start[k], start[k] + block)
// (face-local order) of face face[k] of domain dom[k].
struct WallTiles {
    const int *dom;
    const int *face;
    const int *start;
    int n;
    int block;
};

// One adjoint-path launch.  batch == null: a single domain described by
// params (Params<CT>), one workgroup per Z-row chunk; otherwise the batch's
// tile list (workgroup k = tile k) and per-domain parameters.
struct AdjLaunch {
    int op;
    int lattice;
    int storage;
    const void *params;     // Params<CT> (single domain)
    const BatchDev *batch;  // batch tile list, or null
    const void *F;          // natural state f(t) (ADJ_STEP / ADJ_SEED) or in-place state (ADJ_MATERIALIZE)
    const void *An;         // a(t+1)
    void *Ao;               // a(t)
    void *D;                // materialized natural state
    void *ds;               // dL/ds accumulator (CT) or null
    float *ds_out;          // ADJ_DS_OUT destination
    double *acc;            // one row per workgroup: sum lambda (f - feq)
    double *accw;           // 3 rows per wall tile
    WallTiles walls;
    const void *grho, *gu;
    int force;              // ADJ_STEP: the body force is on
    int reg;                // ADJ_STEP: a face is regularized (its closure transpose needs the pre-closure state)
    int kbc;                // ADJ_STEP: the KBC collision (D2Q9, D3Q27; no body force, no regularized face)
    void *dF;               // dL/dF accumulators (CT, 3 planes of N, internal axes) or null
    void *df_out;           // ADJ_DF_OUT destination (D planes of N, caller axes, in_f64 ? double : float) or null
    double eps;             // ADJ_DF_OUT: scale of the force (rows in acc: D FP64 sums per 256 cells)
    int in_f64;
    int pending;            // batch: the state read needs the Zou-He closure
    int64_t N;
    unsigned grid, block;
    hipStream_t stream;
};

hipError_t launch_adjoint(const AdjLaunch &g);

}  // namespace lbm
