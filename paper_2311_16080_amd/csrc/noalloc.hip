// noalloc.hip -- lbm_forces_noalloc: the momentum-exchange force of the last
// step without any allocation or synchronisation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).  Its scratch
// is one file-scope device array per GPU; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace lbm;

namespace {
constexpr int kSlots = 21;
// rows of one pass (one row per step-kernel workgroup or per 256 curved links)
constexpr int64_t kChunkRows = 16384;
// passes of one call
constexpr int64_t kMaxChunks = 4096;
constexpr size_t kScratchDoubles = (size_t)(kChunkRows + kMaxChunks + 1) * kSlots;   // 3.4 MB
}  // namespace

// Layout: [kChunkRows rows][kMaxChunks pass sums][1 total], 21 FP64 each.
// Each GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch array (looked up once per device,
// with that device current).
int scratch_of(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return fail(LBM_EUNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_ptr[device] = static_cast<double *>(p);
    }
    *out = g_ptr[device];
    return LBM_OK;
}

// internal faces / axes -> caller faces / axes (2-D: internal (Y, Z) are the
// caller's (x, y), internal faces 2..5 the caller's -x, +x, -y, +y)
__global__ void k_forces_to_caller(const double *__restrict__ m, double *__restrict__ out, int D) {
    const int k = (int)threadIdx.x;
    if (k >= kSlots) return;
    if (D == 3) {
        out[k] = m[k];
        return;
    }
    double v = 0.0;
    if (k < 3) {
        v = (k < 2) ? m[k + 1] : 0.0;
    } else {
        const int f = (k - 3) / 3, a = (k - 3) % 3;
        if (f < 4 && a < 2) v = m[3 + 3 * (f + 2) + (a + 1)];
    }
    out[k] = v;
}

}  // namespace

extern "C" int lbm_forces_noalloc(lbm_ctx *c, double *out_dev) {
    if (!c || !out_dev) return fail(LBM_EINVAL, "null argument");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "lbm_forces_noalloc takes a single-domain context");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised (call lbm_init_equilibrium)");
    if (c->t < 1) return fail(LBM_ESTATE, "no step taken since the last init / load");
    const int64_t lrows = (c->nlinks + 255) / 256;
    const int64_t rows = c->grid + lrows;
    const int64_t chunks = (rows + kChunkRows - 1) / kChunkRows;
    if (chunks > kMaxChunks)
        return fail(LBM_EINVAL, "%lld force rows exceed the %lld this entry point's scratch holds (use lbm_forces)",
                    (long long)rows, (long long)(kChunkRows * kMaxChunks));
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    double *base = nullptr;
    int rc = scratch_of(c->device, &base);
    if (rc) return rc;
    double *rowbuf = base;
    double *passes = base + (size_t)kChunkRows * kSlots;
    double *total = passes + (size_t)kMaxChunks * kSlots;
    refresh_params(c);
    const Launch g = make_launch(c);
    const void *lt = (c->opt.storage == LBM_F64) ? (const void *)&c->ltd : (const void *)&c->ltf;
    // pass k covers rows [k R, (k + 1) R) of [step-grid rows | curved-link rows]
    for (int64_t k = 0; k < chunks && e == hipSuccess; ++k) {
        const int64_t r0 = k * kChunkRows;
        const int64_t r1 = (r0 + kChunkRows < rows) ? r0 + kChunkRows : rows;
        if (r0 < c->grid) {
            const int64_t b1 = (r1 < c->grid) ? r1 : c->grid;
            e = launch_forces(g, rowbuf, r0, b1 - r0);
        }
        if (e == hipSuccess && r1 > c->grid) {
            const int64_t l0 = (r0 > c->grid) ? r0 - c->grid : 0;
            e = launch_link_forces(g, lt, rowbuf + (size_t)((c->grid > r0) ? c->grid - r0 : 0) * kSlots, l0,
                                   r1 - c->grid - l0);
        }
        if (e == hipSuccess) e = launch_rows_reduce(rowbuf, r1 - r0, kSlots, passes + (size_t)k * kSlots, c->stream);
    }
    if (e == hipSuccess) e = launch_rows_reduce(passes, chunks, kSlots, total, c->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_forces_to_caller, dim3(1), dim3(64), 0, c->stream, total, out_dev, c->D);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_fail(e, "lbm_forces_noalloc");
    return LBM_OK;
}
