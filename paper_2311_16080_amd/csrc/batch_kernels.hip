// batch_kernels.hip -- kernels of batched small domains (gfx950).
//
// Same per-cell arithmetic as the single-domain path (step_cell,
// moments_cell), driven by a tile list: workgroup k processes tile k = B
// consecutive cells of one domain.  The persistent variant keeps one grid of
// resident workgroups for n steps, striding over the tile list, with a grid
// barrier between steps (cooperative launch, so all workgroups are resident).
#include <hip/hip_cooperative_groups.h>

#include "batch.hpp"
#include "kernels_impl.hpp"

namespace lbm {

template <class L, class ST, int MODE, int NT>
__device__ __forceinline__ void batch_tile(const BatchDev &b, ST *A, int tile, int pending, ST *B = nullptr) {
    using CT = typename Store<ST>::CT;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    const int n = p.nX * p.nY * p.nZ;
    if (c >= n) return;
    int X, Y, Z;
    split_cell(c, p.nY, p.nZ, X, Y, Z);
    step_cell<L, ST, MODE, false, NT>(p, A + b.stoff[d], MODE == 2 ? B + b.stoff[d] : nullptr, X, Y, Z, pending);
}

template <class L, class ST, int MODE, int NT>
__global__ void __launch_bounds__(kMaxBlock) k_step_batch(const BatchDev b, ST *__restrict__ A, int pending) {
    batch_tile<L, ST, MODE, NT>(b, A, (int)blockIdx.x, pending);
}

template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_push_batch(const BatchDev b, const ST *__restrict__ A,
                                                          ST *__restrict__ B, int pending) {
    batch_tile<L, ST, 2, 1>(b, const_cast<ST *>(A), (int)blockIdx.x, pending, B);
}

// n steps in one launch: resident workgroups stride over the tiles; a grid
// barrier separates the steps (every workgroup reaches every barrier).
template <class L, class ST, int NT>
__global__ void __launch_bounds__(kMaxBlock) k_step_batch_persistent(const BatchDev b, ST *__restrict__ A, int nsteps,
                                                                     long long t0) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int k = 0; k < nsteps; ++k) {
        const long long t = t0 + k;
        const int pending = t > 0 ? 1 : 0;
        if (t & 1) {
            for (int tile = (int)blockIdx.x; tile < b.ntiles; tile += (int)gridDim.x)
                batch_tile<L, ST, 1, NT>(b, A, tile, pending);
        } else {
            for (int tile = (int)blockIdx.x; tile < b.ntiles; tile += (int)gridDim.x)
                batch_tile<L, ST, 0, NT>(b, A, tile, pending);
        }
        grid.sync();
    }
}

template <class L, class ST, class IT>
__global__ void __launch_bounds__(kMaxBlock) k_init_batch(const BatchDev b, ST *__restrict__ A,
                                                          const IT *__restrict__ rho_in, const IT *__restrict__ u_in) {
    using CT = typename Store<ST>::CT;
    const int tile = (int)blockIdx.x;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    if (c >= p.nX * p.nY * p.nZ) return;
    const int64_t g = b.cell0[d] + c;
    const int64_t N = b.ncells;
    CT rho = rho_in ? (CT)rho_in[g] : p.rho0;
    CT u[3] = {0, 0, 0};
    if (u_in) {
        if constexpr (L::D == 2) {
            u[1] = (CT)u_in[g];
            u[2] = (CT)u_in[N + g];
        } else {
            u[0] = (CT)u_in[g];
            u[1] = (CT)u_in[N + g];
            u[2] = (CT)u_in[2 * N + g];
        }
    }
    const CT usq15 = (CT)1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    ST *Ad = A + b.stoff[d];
    unroll<L::Q>([&](auto I) { sth<L, ST, I>(Ad, c, heq<L, I>(rho - p.rho0, rho, u[0], u[1], u[2], usq15)); });
}

template <class L, class ST, class OT, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_moments_batch(const BatchDev b, const ST *__restrict__ A, int pending,
                                                             OT *__restrict__ rho_out, OT *__restrict__ u_out,
                                                             double *__restrict__ partial) {
    using CT = typename Store<ST>::CT;
    const int tile = (int)blockIdx.x;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    double m[5] = {0, 0, 0, 0, 0};
    if (c < p.nX * p.nY * p.nZ) {
        int X, Y, Z;
        split_cell(c, p.nY, p.nZ, X, Y, Z);
        CT rho, ux, uy, uz;
        if (moments_cell<L, ST, ODD>(p, A + b.stoff[d], X, Y, Z, pending, rho, ux, uy, uz)) {
            const double r = (double)rho, vx = (double)ux, vy = (double)uy, vz = (double)uz;
            m[0] = r;
            m[1] = r * vx;
            m[2] = r * vy;
            m[3] = r * vz;
            m[4] = 0.5 * r * (vx * vx + vy * vy + vz * vz);
        }
        store_moments<L>(rho_out, u_out, b.cell0[d] + c, b.ncells, rho, ux, uy, uz);
    }
    if (partial) block_sums(m, partial, tile);
}

// ---------------------------------------------------------------------------
template <class L, class ST>
static hipError_t b_step(const BatchLaunch &g, int mode, int pending) {
    ST *A = static_cast<ST *>(g.A);
    if (mode == 0)
        hipLaunchKernelGGL((k_step_batch<L, ST, 0, 1>), dim3(g.grid), dim3(g.block), 0, g.stream, g.b, A, pending);
    else
        hipLaunchKernelGGL((k_step_batch<L, ST, 1, 1>), dim3(g.grid), dim3(g.block), 0, g.stream, g.b, A, pending);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t b_push(const BatchLaunch &g, void *B, int pending) {
    hipLaunchKernelGGL((k_push_batch<L, ST>), dim3(g.grid), dim3(g.block), 0, g.stream, g.b,
                       static_cast<const ST *>(g.A), static_cast<ST *>(B), pending);
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t b_persistent(const BatchLaunch &g, int nsteps, int64_t t0) {
    ST *A = static_cast<ST *>(g.A);
    long long tt = (long long)t0;
    BatchDev b = g.b;
    void *args[] = {(void *)&b, (void *)&A, (void *)&nsteps, (void *)&tt};
    return hipLaunchCooperativeKernel((const void *)k_step_batch_persistent<L, ST, 1>, dim3(g.grid), dim3(g.block),
                                      args, 0, g.stream);
}

template <class L, class ST>
static int b_occupancy(int block) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_step_batch_persistent<L, ST, 1>, block, 0) !=
        hipSuccess)
        return 0;
    return n;
}

template <class L, class ST>
static hipError_t b_init(const BatchLaunch &g, const void *rho, const void *u, int in_f64) {
    ST *A = static_cast<ST *>(g.A);
    if (in_f64)
        hipLaunchKernelGGL((k_init_batch<L, ST, double>), dim3(g.grid), dim3(g.block), 0, g.stream, g.b, A,
                           static_cast<const double *>(rho), static_cast<const double *>(u));
    else
        hipLaunchKernelGGL((k_init_batch<L, ST, float>), dim3(g.grid), dim3(g.block), 0, g.stream, g.b, A,
                           static_cast<const float *>(rho), static_cast<const float *>(u));
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t b_moments(const BatchLaunch &g, bool odd, int pending, void *rho, void *u, int out_f64,
                            double *partial) {
    const ST *A = static_cast<const ST *>(g.A);
#define LBM_BM(OT, ODD)                                                                                            \
    hipLaunchKernelGGL((k_moments_batch<L, ST, OT, ODD>), dim3(g.grid), dim3(g.block), 0, g.stream, g.b, A, pending, \
                       static_cast<OT *>(rho), static_cast<OT *>(u), partial);
    if (out_f64) {
        if (odd) { LBM_BM(double, true) } else { LBM_BM(double, false) }
    } else {
        if (odd) { LBM_BM(float, true) } else { LBM_BM(float, false) }
    }
#undef LBM_BM
    return hipGetLastError();
}

template <class L, class ST>
static hipError_t b_dispatch(const BatchLaunch &g, int op, int a, int c, int64_t t0, const void *p0, const void *p1,
                             void *q0, void *q1, double *partial, int *occ) {
    switch (op) {
        case 0: return b_step<L, ST>(g, a, c);
        case 1: return b_persistent<L, ST>(g, a, t0);
        case 2: return b_init<L, ST>(g, p0, p1, a);
        case 3: return b_moments<L, ST>(g, a != 0, c, q0, q1, (int)t0, partial);
        case 4: *occ = b_occupancy<L, ST>((int)g.block); return hipSuccess;
        case 5: return b_push<L, ST>(g, q0, c);
    }
    return hipErrorInvalidValue;
}

template <class L>
static hipError_t b_storage(const BatchLaunch &g, int op, int a, int c, int64_t t0, const void *p0, const void *p1,
                            void *q0, void *q1, double *partial, int *occ) {
    switch (g.storage) {
        case ST_F64: return b_dispatch<L, double>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
        case ST_F32: return b_dispatch<L, float>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
        case ST_F16: return b_dispatch<L, _Float16>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
        case ST_BF16: return b_dispatch<L, bf16_t>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
    }
    return hipErrorInvalidValue;
}

static hipError_t b_all(const BatchLaunch &g, int op, int a, int c, int64_t t0, const void *p0 = nullptr,
                        const void *p1 = nullptr, void *q0 = nullptr, void *q1 = nullptr, double *partial = nullptr,
                        int *occ = nullptr) {
    switch (g.lattice) {
        case LAT_D2Q9: return b_storage<D2Q9>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
        case LAT_D3Q19: return b_storage<D3Q19>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
        case LAT_D3Q27: return b_storage<D3Q27>(g, op, a, c, t0, p0, p1, q0, q1, partial, occ);
    }
    return hipErrorInvalidValue;
}

hipError_t batch_launch_step(const BatchLaunch &g, int mode, int pending) { return b_all(g, 0, mode, pending, 0); }

hipError_t batch_launch_push(const BatchLaunch &g, void *B, int pending) {
    return b_all(g, 5, 0, pending, 0, nullptr, nullptr, B);
}

hipError_t batch_launch_persistent(const BatchLaunch &g, int nsteps, int64_t t0) { return b_all(g, 1, nsteps, 0, t0); }

hipError_t batch_launch_init(const BatchLaunch &g, const void *rho, const void *u, int in_f64) {
    return b_all(g, 2, in_f64, 0, 0, rho, u);
}

hipError_t batch_launch_moments(const BatchLaunch &g, bool odd, int pending, void *rho, void *u, int out_f64,
                                double *partial) {
    return b_all(g, 3, odd ? 1 : 0, pending, out_f64, nullptr, nullptr, rho, u, partial);
}

int batch_persistent_occupancy(int lattice, int storage, int block) {
    BatchLaunch g{};
    g.lattice = lattice;
    g.storage = storage;
    g.block = (unsigned)block;
    int occ = 0;
    if (b_all(g, 4, 0, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, &occ) != hipSuccess) return 0;
    return occ;
}

}  // namespace lbm
