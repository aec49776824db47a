// ctx.hpp -- the context object behind the opaque lbm_ctx handle (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/lbm.h"
#include "batch.hpp"

namespace lbm {

// One domain of a batch context.
struct Domain {
    int nx, ny, nz;       // caller axes
    int nX, nY, nZ;       // internal axes
    int64_t cell0;        // first packed cell
    int64_t N;
    int64_t block0;       // first block of this domain in a batch launch
    int64_t nblocks;
    int zblocks;
    double tau;
    lbm_face iface[6];    // internal faces
};

struct TapeState;
struct BatchState;

}  // namespace lbm

struct lbm_ctx {
    // shape
    int lattice = 0, Q = 0, D = 0;
    int nx = 0, ny = 0, nz = 0;      // caller axes
    int nX = 0, nY = 0, nZ = 0;      // internal axes (Z contiguous)
    int64_t N = 0;                   // cells
    int64_t plane = 0;               // elements per direction plane
    double tau = 1.0;
    lbm_bc bc{};                     // faces as given
    lbm_face iface[6]{};             // faces in internal axes
    lbm_options opt{};
    int block = 256, zblocks = 1;
    int64_t grid = 1;
    int nt = -1;                     // step kernel memory hints (LBM_NT = 0..4; -1: per storage type)
    int xcd_remap = 0;               // LBM_XCD_REMAP = 0 / 1 (measured: off is faster)
    int zrot = 0;                    // LBM_ZROT = 0 / 1: rotate lanes within a Z row by 32
    int pair = 1;                    // LBM_PAIR = 0 / 1 / 2: two cells per lane for FP16 / BF16 storage (0 never, 1 even steps, 2 all in-place steps)
    int block_req = 0;               // LBM_BLOCK = 64 / 128 / 192 / 256 (threads per block, along Z); 0: by row length
    int flat = 0;                    // blocks cover consecutive cells of the grid (rows not a multiple of 64 cells)
    int flat_req = -1;               // LBM_FLAT = 0 / 1 forces the row / flat mapping (measurement); -1: by row length
    int split = 0;                   // 2-byte storage in split pairs (core.hpp, sidx)
    int split_req = -1;              // LBM_SPLIT = 0 / 1: split pairs off / on where possible (default on)

    // device
    int device = -1;
    hipStream_t stream = nullptr;
    void *A = nullptr, *B = nullptr;  // population buffers
    uint8_t *flags = nullptr;
    uint32_t *nbm = nullptr;
    float *s = nullptr;
    double *partial = nullptr, *sums_dev = nullptr;
    double *frows = nullptr;         // force sums: grid rows + 1 result row of 21
    int64_t *rbeg = nullptr, *rend = nullptr;
    lbm::Params<double> pd{};
    lbm::Params<float> pf{};
    lbm::FaceTab<double> *ftd = nullptr;   // device face tables
    lbm::FaceTab<float> *ftf = nullptr;

    // curved-wall links (interpolated bounce-back)
    std::vector<uint8_t> solid_host;       // host copy of the solid mask (N bytes), empty without solids
    int64_t nlinks = 0;
    int link_order = 1;
    void *links = nullptr;                 // device block: q, dlt (compute type), cell, cff, cfff (int32), dir, kind
    lbm::LinkTab<double> ltd{};            // views of that block
    lbm::LinkTab<float> ltf{};

    int collision = 0;                     // LBM_BGK / LBM_KBC
    int walls_only = 1;                    // LBM_WALLS_ONLY = 0 / 1

    // body force (exact-difference method)
    bool force_on = false;
    double force_u[3] = {0.0, 0.0, 0.0};   // uniform part, scale applied (caller axes)
    const void *force_field = nullptr;     // device: D planes of N values (CT of the storage)
    double force_eps = 1.0;

    // time
    int64_t t = 0;

    // batch
    bool batch = false;
    int ndomains = 1;
    std::vector<lbm::Domain> dom;
    int64_t bgrid = 0;
    lbm::BatchState *bs = nullptr;

    // tape (adjoint)
    lbm::TapeState *tape = nullptr;
    bool tape_recording = false;
    bool moved_since_tape = true;
    int64_t tape_serial = 0;         // id of the most recent tape (lbm_tape_id)

    // captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_steps = 0;
    int64_t graph_t0 = 0;
    void *graph_A = nullptr;
    int graph_persistent = 0;
};

namespace lbm {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate_domain(int lattice, int nx, int ny, int nz, double tau, const lbm_bc *bc);
void refresh_params(lbm_ctx *c);
size_t storage_size(int storage);
int dev_alloc(void **p, size_t bytes, const char *what);
void dev_free(void *&p);
void free_all(lbm_ctx *c);
Launch make_launch(lbm_ctx *c);
hipError_t forward_step(lbm_ctx *c);

// Kernel mode of the step taken from time t: 0 / 1 the in-place even / odd
// step, 2 the push step, 3 the pull step (LBM_PULL starts from a natural state
// with the local even step).
inline int step_mode_at(const lbm_ctx *c, int64_t t) {
    if (c->opt.pattern == LBM_INPLACE) return (int)(t & 1);
    if (c->opt.pattern == LBM_PULL) return t > 0 ? 3 : 0;
    return 2;
}
inline int step_mode(const lbm_ctx *c) { return step_mode_at(c, c->t); }
// The state at time t holds f*_i(x) in slot opp(i) of x (what the in-place
// even step and the pull step leave) rather than the natural f_i(x) in slot i.
inline bool swapped_at(const lbm_ctx *c, int64_t t) {
    return (c->opt.pattern == LBM_INPLACE && (t & 1)) || (c->opt.pattern == LBM_PULL && t > 0);
}

// graph.hip
void drop_graph(lbm_ctx *c);

// tape.hip
int tape_after_step(lbm_ctx *c);
void tape_release(lbm_ctx *c);
// a parameter of the recorded steps changed: the tape no longer describes them
void tape_invalidate(lbm_ctx *c);

// batch.hip
int batch_upload(lbm_ctx *c);
void batch_layout(lbm_ctx *c);   // per-domain state offsets
void batch_release(lbm_ctx *c);
hipError_t batch_init(lbm_ctx *c, const void *rho, const void *u, bool f64);
hipError_t batch_step(lbm_ctx *c);
hipError_t batch_moments(lbm_ctx *c, bool odd, void *rho, void *u, bool f64, double *partial);
hipError_t batch_persistent_steps(lbm_ctx *c, int n);
bool batch_uses_persistent(const lbm_ctx *c);
BatchLaunch batch_launch_of(lbm_ctx *c);   // tile-list launch over the current state
int batch_autotune(lbm_ctx *c);

}  // namespace lbm
