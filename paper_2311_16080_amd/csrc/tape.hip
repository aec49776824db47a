// tape.hip -- checkpoint tape and the backward (discrete adjoint) driver.
//
// Recording keeps a bit-exact copy of the state every K steps (the paper's
// gradient checkpointing for unrolled training, Sec. 6.1).  The backward pass
// walks the segments from last to first: it rebuilds the segment's K states in
// natural order with the double-buffer push step (the same per-cell arithmetic
// as the in-place step, so the recomputed states equal the originals bit for
// bit), then runs the adjoint step backwards through them.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "adjoint.hpp"
#include "ctx.hpp"

using namespace lbm;

namespace lbm {
struct TapeState {
    int K = 0;
    int max_steps = 0;
    int64_t t_begin = 0, t_end = 0;
    size_t sbytes = 0;        // one state image (Q planes, storage type)
    size_t abytes = 0;        // one adjoint image (Q planes, compute type)
    int nck = 0;
    std::vector<int64_t> ck_t;
    void *ck = nullptr;       // nck state images
    void *ring = nullptr;     // K natural states
    void *abuf[2] = {nullptr, nullptr};
    void *ds = nullptr;       // N compute-type accumulators
    double *acc = nullptr;    // grid x kAdjSlots
    double *out = nullptr;    // kAdjSlots per domain
    double *itau2 = nullptr;  // batch: 1 / tau_d^2 per domain
    int64_t rows = 0;         // accumulator rows
};
}  // namespace lbm

static size_t state_bytes_of(const lbm_ctx *c) { return (size_t)c->Q * (size_t)c->plane * storage_size(c->opt.storage); }
static size_t compute_size(const lbm_ctx *c) { return c->opt.storage == LBM_F64 ? 8 : 4; }

void lbm::tape_release(lbm_ctx *c) {
    if (c->tape) {
        TapeState *T = c->tape;
        dev_free(T->ck);
        dev_free(T->ring);
        dev_free(T->abuf[0]);
        dev_free(T->abuf[1]);
        dev_free(T->ds);
        dev_free((void *&)T->acc);
        dev_free((void *&)T->out);
        dev_free((void *&)T->itau2);
        delete T;
    }
    c->tape = nullptr;
    c->tape_recording = false;
}

static hipError_t checkpoint(lbm_ctx *c, int slot) {
    TapeState *T = c->tape;
    return hipMemcpyAsync(static_cast<char *>(T->ck) + (size_t)slot * T->sbytes, c->A, T->sbytes,
                          hipMemcpyDeviceToDevice, c->stream);
}

int lbm::tape_after_step(lbm_ctx *c) {
    if (!c->tape_recording) return LBM_OK;
    TapeState *T = c->tape;
    const int64_t k = c->t - T->t_begin;
    if (k > T->max_steps) {
        c->tape_recording = false;
        return fail(LBM_ESTATE, "tape full: more than max_steps = %d steps recorded", T->max_steps);
    }
    if (k % T->K == 0) {
        const int slot = (int)(k / T->K);
        hipError_t e = checkpoint(c, slot);
        if (e != hipSuccess) return hip_fail(e, "tape checkpoint");
        T->ck_t[slot] = c->t;
    }
    return LBM_OK;
}

extern "C" int lbm_tape_begin(lbm_ctx *c, int K, int max_steps) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (K < 1 || max_steps < 1) return fail(LBM_EINVAL, "K and max_steps must be >= 1");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised");
    if (c->tape_recording) return fail(LBM_ESTATE, "a tape is already recording");
    tape_release(c);
    (void)hipSetDevice(c->device);
    TapeState *T = new (std::nothrow) TapeState();
    if (!T) return fail(LBM_ENOMEM, "host allocation failed");
    c->tape = T;
    T->K = K;
    T->max_steps = max_steps;
    T->sbytes = state_bytes_of(c);
    T->abytes = (size_t)c->Q * (size_t)c->plane * compute_size(c);
    T->nck = max_steps / K + 1;
    T->ck_t.assign(T->nck, -1);
    int rc = dev_alloc(&T->ck, (size_t)T->nck * T->sbytes, "tape checkpoints");
    if (!rc) rc = dev_alloc(&T->ring, (size_t)K * T->sbytes, "tape recompute ring");
    if (!rc) rc = dev_alloc(&T->abuf[0], T->abytes, "adjoint state");
    if (!rc) rc = dev_alloc(&T->abuf[1], T->abytes, "adjoint state");
    // batch: one accumulator row per tile of the smallest tile size (any tuning fits)
    T->rows = c->batch ? c->bgrid : c->grid;
    if (!rc && !c->batch) rc = dev_alloc(&T->ds, (size_t)c->N * compute_size(c), "dL/ds accumulator");
    if (!rc) rc = dev_alloc((void **)&T->acc, (size_t)T->rows * kAdjSlots * sizeof(double), "adjoint sums");
    if (!rc) rc = dev_alloc((void **)&T->out, (size_t)c->ndomains * kAdjSlots * sizeof(double), "adjoint sums");
    if (!rc && c->batch) {
        rc = dev_alloc((void **)&T->itau2, (size_t)c->ndomains * sizeof(double), "batch 1/tau^2");
        if (!rc) {
            std::vector<double> v(c->ndomains);
            for (int d = 0; d < c->ndomains; ++d) v[d] = 1.0 / (c->dom[d].tau * c->dom[d].tau);
            if (hipMemcpy(T->itau2, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(LBM_EDEVICE, "batch 1/tau^2 upload");
        }
    }
    if (rc) {
        tape_release(c);
        return fail(LBM_ENOMEM, "tape for K = %d, max_steps = %d does not fit in device memory (%s)", K, max_steps,
                    lbm_last_error());
    }
    T->t_begin = c->t;
    hipError_t e = checkpoint(c, 0);
    if (e != hipSuccess) {
        tape_release(c);
        return hip_fail(e, "tape checkpoint");
    }
    T->ck_t[0] = c->t;
    c->tape_recording = true;
    return LBM_OK;
}

extern "C" int lbm_tape_end(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->tape && c->tape_recording) {
        c->tape->t_end = c->t;
        c->moved_since_tape = false;
    }
    c->tape_recording = false;
    return LBM_OK;
}

extern "C" int lbm_tape_free(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    tape_release(c);
    return LBM_OK;
}

static AdjLaunch adj_launch(lbm_ctx *c, int op) {
    AdjLaunch g;
    std::memset(&g, 0, sizeof g);
    g.op = op;
    g.lattice = c->lattice;
    g.storage = c->opt.storage;
    g.params = (c->opt.storage == LBM_F64) ? (const void *)&c->pd : (const void *)&c->pf;
    g.N = c->N;
    g.grid = (unsigned)c->grid;
    g.block = (unsigned)c->block;
    g.stream = c->stream;
    return g;
}

static void set_pending(lbm_ctx *c, int64_t t) { c->pd.zh_pending = c->pf.zh_pending = (t > 0) ? 1 : 0; }

static BatchAdjLaunch badj_launch(lbm_ctx *c, int op, int64_t t) {
    const BatchLaunch bl = batch_launch_of(c);
    BatchAdjLaunch g;
    std::memset(&g, 0, sizeof g);
    g.op = op;
    g.lattice = bl.lattice;
    g.storage = bl.storage;
    g.b = bl.b;
    g.grid = bl.grid;
    g.block = bl.block;
    g.stream = bl.stream;
    g.pending = (t > 0) ? 1 : 0;
    return g;
}

// natural-order copy of a stored state image taken at time t into dst
static hipError_t restore_natural(lbm_ctx *c, const void *img, int64_t t, void *dst) {
    TapeState *T = c->tape;
    if (c->batch && (t & 1)) {
        BatchAdjLaunch g = badj_launch(c, ADJ_MATERIALIZE, t);
        g.F = img;
        g.D = dst;
        hipError_t e = hipMemsetAsync(dst, 0, T->sbytes, c->stream);  // padding slots stay defined
        if (e != hipSuccess) return e;
        return launch_adjoint_batch(g);
    }
    if (c->opt.pattern == LBM_INPLACE && (t & 1)) {
        AdjLaunch g = adj_launch(c, ADJ_MATERIALIZE);
        g.F = img;
        g.D = dst;
        hipError_t e = hipMemsetAsync(dst, 0, T->sbytes, c->stream);  // solid slots stay defined
        if (e != hipSuccess) return e;
        return launch_adjoint(g);
    }
    return hipMemcpyAsync(dst, img, T->sbytes, hipMemcpyDeviceToDevice, c->stream);
}

extern "C" int lbm_backward(lbm_ctx *c, const void *dL_drho, const void *dL_du, int dtype, float *dL_ds,
                            double *dL_dtau, double *dL_duw) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if ((dL_drho || dL_du) && dtype != LBM_F64 && dtype != LBM_F32)
        return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
    if (!c->tape) return fail(LBM_ESTATE, "no tape recorded");
    if (c->tape_recording) lbm_tape_end(c);
    TapeState *T = c->tape;
    if (c->moved_since_tape || c->t != T->t_end) return fail(LBM_ESTATE, "the state moved since the tape ended");
    (void)hipSetDevice(c->device);
    refresh_params(c);
    const int64_t n = T->t_end - T->t_begin;
    char *ring = static_cast<char *>(T->ring);
    hipError_t e = hipSuccess;
    int cur = 0;

    // seed a(t_end) from the final state
    e = restore_natural(c, c->A, c->t, ring);
    if (e == hipSuccess && c->batch) {
        BatchAdjLaunch g = badj_launch(c, ADJ_SEED, c->t);
        g.F = ring;
        g.grho = dL_drho;
        g.gu = dL_du;
        g.in_f64 = dtype == LBM_F64;
        g.Ao = T->abuf[cur];
        e = launch_adjoint_batch(g);
    } else if (e == hipSuccess) {
        set_pending(c, c->t);
        AdjLaunch g = adj_launch(c, ADJ_SEED);
        g.F = ring;
        g.grho = dL_drho;
        g.gu = dL_du;
        g.in_f64 = dtype == LBM_F64;
        g.Ao = T->abuf[cur];
        e = launch_adjoint(g);
    }
    if (e == hipSuccess) e = hipMemsetAsync(T->acc, 0, (size_t)T->rows * kAdjSlots * sizeof(double), c->stream);
    if (e == hipSuccess && T->ds) e = hipMemsetAsync(T->ds, 0, (size_t)c->N * compute_size(c), c->stream);

    const int nseg = (int)((n + T->K - 1) / T->K);
    void *A0 = c->A, *B0 = c->B;
    const int64_t t_now = c->t;
    for (int seg = nseg - 1; seg >= 0 && e == hipSuccess; --seg) {
        const int64_t t0 = T->t_begin + (int64_t)seg * T->K;
        const int64_t t1 = (t0 + T->K < T->t_end) ? t0 + T->K : T->t_end;
        e = restore_natural(c, static_cast<char *>(T->ck) + (size_t)seg * T->sbytes, t0, ring);
        // recompute f(t0 + 1) .. f(t1 - 1) into the ring with the push step
        for (int64_t k = 1; k < t1 - t0 && e == hipSuccess; ++k) {
            if (c->batch) {
                BatchLaunch g = batch_launch_of(c);
                g.A = ring + (size_t)(k - 1) * T->sbytes;
                e = batch_launch_push(g, ring + (size_t)k * T->sbytes, (t0 + k - 1 > 0) ? 1 : 0);
                continue;
            }
            set_pending(c, t0 + k - 1);
            Launch g = make_launch(c);
            g.A = ring + (size_t)(k - 1) * T->sbytes;
            g.B = ring + (size_t)k * T->sbytes;
            e = launch_step(g, 2, c->s != nullptr);
        }
        // adjoint steps backwards
        for (int64_t t = t1 - 1; t >= t0 && e == hipSuccess; --t) {
            if (c->batch) {
                BatchAdjLaunch g = badj_launch(c, ADJ_STEP, t);
                g.F = ring + (size_t)(t - t0) * T->sbytes;
                g.An = T->abuf[cur];
                g.Ao = T->abuf[1 - cur];
                g.acc = T->acc;
                g.inv_tau2 = T->itau2;
                e = launch_adjoint_batch(g);
                cur = 1 - cur;
                continue;
            }
            set_pending(c, t);
            AdjLaunch g = adj_launch(c, ADJ_STEP);
            g.F = ring + (size_t)(t - t0) * T->sbytes;
            g.An = T->abuf[cur];
            g.Ao = T->abuf[1 - cur];
            g.ds = c->s ? T->ds : nullptr;
            g.acc = T->acc;
            g.inv_tau2 = 1.0 / (c->tau * c->tau);
            e = launch_adjoint(g);
            cur = 1 - cur;
        }
    }
    c->A = A0;
    c->B = B0;
    c->t = t_now;
    set_pending(c, c->t);

    if (e == hipSuccess && dL_ds) {
        if (c->s) {
            AdjLaunch g = adj_launch(c, ADJ_DS_OUT);
            g.ds = T->ds;
            g.ds_out = dL_ds;
            e = launch_adjoint(g);
        } else {
            e = hipMemsetAsync(dL_ds, 0, (size_t)c->N * sizeof(float), c->stream);
        }
    }
    const int nd = c->ndomains;
    std::vector<double> sums((size_t)nd * kAdjSlots);
    if (e == hipSuccess) {
        if (c->batch) {
            BatchAdjLaunch g = badj_launch(c, ADJ_REDUCE, c->t);
            g.acc = T->acc;
            g.rbeg = c->rbeg;
            g.rend = c->rend;
            g.out = T->out;
            e = launch_adjoint_batch(g);
        } else {
            e = launch_adj_reduce(T->acc, c->grid, T->out, c->stream);
        }
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(sums.data(), T->out, sums.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_backward");
    for (int d = 0; d < nd; ++d) {
        const double *S = sums.data() + (size_t)d * kAdjSlots;
        if (dL_dtau) dL_dtau[d] = S[0];
        if (dL_duw) {
            // internal faces / axes -> caller faces / axes
            double *o = dL_duw + (size_t)d * 18;
            for (int k = 0; k < 18; ++k) o[k] = 0.0;
            for (int f = 0; f < 6; ++f)
                for (int a = 0; a < 3; ++a) {
                    const double v = S[1 + 3 * f + a];
                    if (c->D == 3) o[3 * f + a] = v;
                    else if (f >= 2 && a >= 1) o[3 * (f - 2) + (a - 1)] = v;
                }
        }
    }
    return LBM_OK;
}
