// batch.hpp -- internal interface of the batched-domain kernels (not public ABI).
//
// A batch holds many independent domains of one lattice.  Each domain keeps
// its own Q planes (padded to 64 cells) back to back in one allocation, and
// its own parameter block (Params) and face table in device memory.  The work
// list is a list of tiles: B consecutive cells (in the domain's linear cell
// order) of one domain, one workgroup per tile, so ragged domain sizes leave
// at most one partial tile per domain.
#pragma once
#include "kernels.hpp"

namespace lbm {

struct BatchDev {
    const void *P;              // Params<CT>[ndom]
    const int *tile_dom;        // [ntiles] domain of the tile
    const int *tile_start;      // [ntiles] first local cell of the tile
    const int64_t *stoff;       // [ndom] state offset of the domain (elements)
    const int64_t *cell0;       // [ndom] first packed cell of the domain (caller fields)
    int ntiles;
    int ndom;
    int64_t ncells;             // total packed cells
};

struct BatchLaunch {
    int lattice;
    int storage;
    BatchDev b;
    void *A;
    unsigned block;             // tile size (threads per workgroup)
    unsigned grid;              // tiles, or resident workgroups for the persistent kernel
    hipStream_t stream;
};

hipError_t batch_launch_step(const BatchLaunch &g, int mode, int pending);
hipError_t batch_launch_persistent(const BatchLaunch &g, int nsteps, int64_t t0);
hipError_t batch_launch_init(const BatchLaunch &g, const void *rho, const void *u, int in_f64);
hipError_t batch_launch_moments(const BatchLaunch &g, bool odd, int pending, void *rho, void *u, int out_f64,
                                double *partial);
// resident workgroups per CU for the persistent kernel (occupancy query)
int batch_persistent_occupancy(int lattice, int storage, int block);

}  // namespace lbm
