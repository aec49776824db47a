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

// local cell c of a domain -> (X, Y, Z); c < 2^24 (small domains), so the
// float reciprocal quotient is off by at most one and is corrected
__device__ __forceinline__ void split_cell(int c, int nY, int nZ, int &X, int &Y, int &Z) {
    const float rz = 1.0f / (float)nZ, ry = 1.0f / (float)nY;
    int r = (int)((float)c * rz);
    int z = c - r * nZ;
    if (z < 0) { r -= 1; z += nZ; } else if (z >= nZ) { r += 1; z -= nZ; }
    int x = (int)((float)r * ry);
    int y = r - x * nY;
    if (y < 0) { x -= 1; y += nY; } else if (y >= nY) { x += 1; y -= nY; }
    X = x;
    Y = y;
    Z = z;
}

template <class CT>
__device__ __forceinline__ const Params<CT> &dom_params(const BatchDev &b, int d) {
    return static_cast<const Params<CT> *>(b.P)[d];
}

hipError_t batch_launch_step(const BatchLaunch &g, int mode, int pending);
// natural-order push step A -> B (the recompute step of the backward pass)
hipError_t batch_launch_push(const BatchLaunch &g, void *B, int pending);
hipError_t batch_launch_persistent(const BatchLaunch &g, int nsteps, int64_t t0);
hipError_t batch_launch_init(const BatchLaunch &g, const void *rho, const void *u, int in_f64);
hipError_t batch_launch_moments(const BatchLaunch &g, bool odd, int pending, void *rho, void *u, int out_f64,
                                double *partial);
// resident workgroups per CU for the persistent kernel (occupancy query)
int batch_persistent_occupancy(int lattice, int storage, int block);

}  // namespace lbm
