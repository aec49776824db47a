// kernels.hpp -- internal interface between the C-ABI host code and the
// kernel launchers (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "core.hpp"

namespace lbm {

enum : int { LAT_D2Q9 = 0, LAT_D3Q19 = 1, LAT_D3Q27 = 2 };
enum : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };
enum : int { OP_STEP = 0, OP_INIT = 1, OP_MOMENTS = 2, OP_FORCES = 3, OP_BOUZIDI = 4, OP_LINK_FORCES = 5 };

// One launch: lattice, storage, a Params<CT> block, buffers, shape.
struct Launch {
    int lattice;
    int storage;
    const void *params;  // Params<double> for F64 storage, Params<float> otherwise
    void *A;             // state buffer
    void *B;             // second buffer (double-buffer pattern)
    unsigned grid;
    unsigned block;
    hipStream_t stream;
    int nt;              // step kernel memory hints: 0 plain, 1 non-temporal, 2 non-temporal stores
    int pair;            // 2-byte storage: two cells per lane (k_step_pair) for 1: even steps, 2: all in-place steps
    unsigned pgrid;      // launch shape of k_step_pair
    unsigned pblock;
    int force;           // body force on (params carry it)
    int kbc;             // KBC collision
    int walls_only;      // allow the walls-only step variant (LBM_WALLS_ONLY = 0 disables it, for measurement)
    int nt_push = -1;    // memory hints for push steps (mode 2); -1: as nt
};

hipError_t launch_step(const Launch &g, int mode, bool has_s);
hipError_t launch_init(const Launch &g, const void *rho, const void *u, int in_f64, int64_t N);
hipError_t launch_moments(const Launch &g, bool odd, void *rho, void *u, int out_f64, double *partial, int64_t N);
hipError_t launch_reduce(const double *partial, const int64_t *begin, const int64_t *end, double *out, int rows,
                         hipStream_t s);
hipError_t launch_solid(int lattice, const Launch &g, const uint8_t *solid, uint8_t *flags, uint32_t *nbm);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// momentum-exchange force rows (one row of 21 FP64 per step-kernel workgroup)
// of the current state for workgroups [b0, b0 + nb) (nb = 0: b0 to the end;
// b0, nb < 2^31), written from rows[0]; then their fixed-order sum into out[21]
hipError_t launch_forces(const Launch &g, double *rows, int64_t b0 = 0, int64_t nb = 0);
hipError_t launch_rows_reduce(const double *rows, int64_t nrows, int slots, double *out, hipStream_t s);
// interpolated bounce-back on the curved links after a step (links: LinkTab<CT>
// of the storage's compute type; natural: the state is in natural slot order,
// i.e. after an odd in-place step or a push step)
hipError_t launch_bouzidi(const Launch &g, const void *links, bool natural);
// one row of 21 FP64 sums per 256 links (slots 0..2: the curved links' share of
// the force on the solids) for row blocks [r0, r0 + nr) (nr = 0: to the end),
// written from rows[0]
hipError_t launch_link_forces(const Launch &g, const void *links, double *rows, int64_t r0 = 0, int64_t nr = 0);

}  // namespace lbm
