// kernels.hip -- non-templated kernels and the lattice dispatch of the
// single-domain forward path (gfx950).  The templated kernels live in
// kernels_impl.hpp and are instantiated per lattice in kernels_d*.hip.
#include "kernels.hpp"

namespace lbm {

template <class L, class ST>
hipError_t dispatch_one(const Launch &g, int op, int a0, bool b0, const void *p0, const void *p1, void *q0, void *q1,
                        double *partial, int64_t N);

template <class L>
static hipError_t dispatch_storage(const Launch &g, int op, int a0, bool b0, const void *p0, const void *p1, void *q0,
                                   void *q1, double *partial, int64_t N) {
    switch (g.storage) {
        case ST_F64: return dispatch_one<L, double>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
        case ST_F32: return dispatch_one<L, float>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
        case ST_F16: return dispatch_one<L, _Float16>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
        case ST_BF16: return dispatch_one<L, bf16_t>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
    }
    return hipErrorInvalidValue;
}
template <class L>
hipError_t solid_t(const Launch &g, const uint8_t *solid, uint8_t *flags, uint32_t *nbm);

// Sum rows [begin[d], end[d]) of the partials into out[d*5 .. d*5+4], one
// block per output row, in a fixed order.
__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ partial, const int64_t *__restrict__ begin,
                                                const int64_t *__restrict__ end, double *__restrict__ out) {
    __shared__ double red[5][256];
    const int d = (int)blockIdx.x;
    const int t = (int)threadIdx.x;
    double m[5] = {0, 0, 0, 0, 0};
    for (int64_t b = begin[d] + t; b < end[d]; b += 256)
        for (int k = 0; k < 5; ++k) m[k] += partial[b * 5 + k];
    for (int k = 0; k < 5; ++k) red[k][t] = m[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 5; ++k) red[k][t] += red[k][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < 5; ++k) out[d * 5 + k] = red[k][0];
}

// One 16-byte non-temporal load and store per lane: the fastest plain copy
// measured on gfx950, used as the achievable-bandwidth reference.
typedef float lbm_v4f __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy(lbm_v4f *__restrict__ dst, const lbm_v4f *__restrict__ src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

static hipError_t dispatch(const Launch &g, int op, int a0, bool b0, const void *p0, const void *p1, void *q0,
                           void *q1, double *partial, int64_t N) {
    switch (g.lattice) {
        case LAT_D2Q9: return dispatch_storage<D2Q9>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
        case LAT_D3Q19: return dispatch_storage<D3Q19>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
        case LAT_D3Q27: return dispatch_storage<D3Q27>(g, op, a0, b0, p0, p1, q0, q1, partial, N);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(const Launch &g, int mode, bool has_s) {
    if (mode == 2 && g.nt_push >= 0 && g.nt_push != g.nt) {
        Launch h = g;
        h.nt = g.nt_push;
        return dispatch(h, OP_STEP, mode, has_s, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
    }
    return dispatch(g, OP_STEP, mode, has_s, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
}

hipError_t launch_init(const Launch &g, const void *rho, const void *u, int in_f64, int64_t N) {
    return dispatch(g, OP_INIT, in_f64, false, rho, u, nullptr, nullptr, nullptr, N);
}

hipError_t launch_moments(const Launch &g, bool odd, void *rho, void *u, int out_f64, double *partial, int64_t N) {
    return dispatch(g, OP_MOMENTS, out_f64, odd, nullptr, nullptr, rho, u, partial, N);
}

hipError_t launch_reduce(const double *partial, const int64_t *begin, const int64_t *end, double *out, int rows,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(rows), dim3(256), 0, s, partial, begin, end, out);
    return hipGetLastError();
}

hipError_t launch_forces(const Launch &g, double *rows, int64_t b0, int64_t nb) {
    return dispatch(g, OP_FORCES, 0, false, nullptr, nullptr, nullptr, nullptr, rows, (b0 << 32) | nb);
}

hipError_t launch_bouzidi(const Launch &g, const void *links, bool natural) {
    return dispatch(g, OP_BOUZIDI, natural ? 1 : 0, false, links, nullptr, nullptr, nullptr, nullptr, 0);
}

hipError_t launch_link_forces(const Launch &g, const void *links, double *rows, int64_t r0, int64_t nr) {
    return dispatch(g, OP_LINK_FORCES, 0, false, links, nullptr, nullptr, nullptr, rows, (r0 << 32) | nr);
}

// out[k] = sum of rows[r * slots + k] over r, one block per slot, fixed order
__global__ void __launch_bounds__(256) k_rows_reduce(const double *__restrict__ rows, int64_t nrows, int slots,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    const int k = (int)blockIdx.x;
    double v = 0.0;
    for (int64_t r = threadIdx.x; r < nrows; r += 256) v += rows[r * slots + k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

hipError_t launch_rows_reduce(const double *rows, int64_t nrows, int slots, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_reduce, dim3(slots), dim3(256), 0, s, rows, nrows, slots, out);
    return hipGetLastError();
}

hipError_t launch_solid(int lattice, const Launch &g, const uint8_t *solid, uint8_t *flags, uint32_t *nbm) {
    switch (lattice) {
        case LAT_D2Q9: return solid_t<D2Q9>(g, solid, flags, nbm);
        case LAT_D3Q19: return solid_t<D3Q19>(g, solid, flags, nbm);
        default: return solid_t<D3Q27>(g, solid, flags, nbm);
    }
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    // one element per lane; split launches keep each grid below 2^31 lanes
    const int64_t per = (int64_t)1 << 30;
    for (int64_t o = 0; o < n; o += per) {
        const int64_t m = (n - o < per) ? (n - o) : per;
        const int64_t blocks = (m + 255) / 256;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<lbm_v4f *>(dst) + o,
                           static_cast<const lbm_v4f *>(src) + o, m);
    }
    return hipGetLastError();
}

}  // namespace lbm
