// adjoint.hpp -- internal interface of the adjoint kernels (not public ABI).
#pragma once
#include "batch.hpp"

namespace lbm {

// per-block accumulator row: [0] dL/dtau, [1 + 3 f + a] dL/du_w of face f, axis a (internal)
constexpr int kAdjSlots = 19;

enum : int { ADJ_STEP = 0, ADJ_SEED = 1, ADJ_MATERIALIZE = 2, ADJ_DS_OUT = 3 };

struct AdjLaunch {
    int op;
    int lattice;
    int storage;
    const void *params;   // Params<CT>
    const void *F;        // natural state f(t) (ADJ_STEP / ADJ_SEED) or in-place state (ADJ_MATERIALIZE)
    const void *An;       // a(t+1)
    void *Ao;             // a(t)
    void *D;              // materialized natural state
    void *ds;             // dL/ds accumulator (CT) or null
    float *ds_out;        // ADJ_DS_OUT destination
    double *acc;          // per-block accumulator rows
    const void *grho, *gu;
    int in_f64;
    double inv_tau2;
    int64_t N;
    unsigned grid, block;
    hipStream_t stream;
};

hipError_t launch_adjoint(const AdjLaunch &g);

// Batch variants: the same ops over a tile list (workgroup k = tile k); the
// adjoint buffers use the state's per-domain offsets; acc holds one row per
// tile.  ADJ_REDUCE sums the rows [rbeg[d], rend[d]) of each domain d into
// out[d * kAdjSlots ...] in a fixed order.
enum : int { ADJ_REDUCE = 4 };

struct BatchAdjLaunch {
    int op;
    int lattice;
    int storage;
    BatchDev b;
    const void *F;
    const void *An;
    void *Ao;
    void *D;
    double *acc;
    const double *inv_tau2;   // [ndom] 1 / tau_d^2
    const void *grho, *gu;
    int in_f64;
    int pending;
    const int64_t *rbeg, *rend;
    double *out;
    unsigned grid, block;
    hipStream_t stream;
};

hipError_t launch_adjoint_batch(const BatchAdjLaunch &g);
hipError_t launch_adj_reduce(const double *acc, int64_t rows, double *out, hipStream_t s);

}  // namespace lbm
