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
    int64_t id = 0;           // lbm_tape_id of this tape
    bool stale = false;       // a parameter changed after the tape began
    bool had_s = false;       // a partial bounce-back field was set when it began
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
    double *acc = nullptr;    // one row per workgroup of the adjoint step
    int64_t rows = 0;
    // moving-wall face tiles (dL/du_w)
    std::vector<int> wdom, wface, wstart;
    int *wt = nullptr;        // device: dom[nwt], face[nwt], start[nwt]
    int nwt = 0;
    double *accw = nullptr;   // 3 rows per wall tile
    // body-force gradient (allocated by the first backward that asks for it)
    void *dF = nullptr;       // 3 planes of N compute-type accumulators
    double *frows = nullptr;  // D FP64 sums per 256 cells, then D totals
};
}  // namespace lbm

static constexpr int kWallBlock = 256;

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
        dev_free((void *&)T->wt);
        dev_free((void *&)T->accw);
        dev_free(T->dF);
        dev_free((void *&)T->frows);
        delete T;
    }
    c->tape = nullptr;
    c->tape_recording = false;
}

void lbm::tape_invalidate(lbm_ctx *c) {
    c->moved_since_tape = true;
    if (c->tape) c->tape->stale = true;
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

// tiles over the cells of every moving-wall face (internal axes) of every domain
static void build_wall_tiles(const lbm_ctx *c, TapeState *T) {
    T->wdom.clear();
    T->wface.clear();
    T->wstart.clear();
    for (int d = 0; d < c->ndomains; ++d) {
        const int nX = c->batch ? c->dom[d].nX : c->nX;
        const int nY = c->batch ? c->dom[d].nY : c->nY;
        const int nZ = c->batch ? c->dom[d].nZ : c->nZ;
        const lbm_face *fc = c->batch ? c->dom[d].iface : c->iface;
        for (int f = 0; f < 6; ++f) {
            const lbm_face &F = fc[f];
            if (F.type != LBM_WALL || (F.u[0] == 0.0 && F.u[1] == 0.0 && F.u[2] == 0.0)) continue;
            const int ax = f >> 1;
            const int64_t cells = (int64_t)(ax == 0 ? nY : nX) * (ax == 2 ? nY : nZ);
            for (int64_t s = 0; s < cells; s += kWallBlock) {
                T->wdom.push_back(d);
                T->wface.push_back(f);
                T->wstart.push_back((int)s);
            }
        }
    }
    T->nwt = (int)T->wdom.size();
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
    T->id = ++c->tape_serial;
    T->had_s = c->s != nullptr;
    T->K = K;
    T->max_steps = max_steps;
    T->sbytes = state_bytes_of(c);
    T->abytes = (size_t)c->Q * (size_t)c->plane * compute_size(c);
    T->nck = max_steps / K + 1;
    T->ck_t.assign(T->nck, -1);
    build_wall_tiles(c, T);
    // batch: one accumulator row per tile of the smallest tile size (any tuning fits)
    T->rows = c->batch ? c->bgrid : c->grid;
    int rc = dev_alloc(&T->ck, (size_t)T->nck * T->sbytes, "tape checkpoints");
    // the first state of a segment is read from its checkpoint when that is in natural order
    if (!rc && K > 1) rc = dev_alloc(&T->ring, (size_t)K * T->sbytes, "tape recompute ring");
    if (!rc && K == 1) rc = dev_alloc(&T->ring, T->sbytes, "tape recompute ring");
    if (!rc) rc = dev_alloc(&T->abuf[0], T->abytes, "adjoint state");
    if (!rc) rc = dev_alloc(&T->abuf[1], T->abytes, "adjoint state");
    if (!rc && c->s) rc = dev_alloc(&T->ds, (size_t)c->N * compute_size(c), "dL/ds accumulator");
    if (!rc) rc = dev_alloc((void **)&T->acc, (size_t)T->rows * sizeof(double), "adjoint sums");
    if (!rc && T->nwt) {
        rc = dev_alloc((void **)&T->wt, (size_t)3 * T->nwt * sizeof(int), "wall tiles");
        if (!rc) rc = dev_alloc((void **)&T->accw, (size_t)3 * T->nwt * sizeof(double), "wall sums");
        if (!rc) {
            std::vector<int> all(T->wdom);
            all.insert(all.end(), T->wface.begin(), T->wface.end());
            all.insert(all.end(), T->wstart.begin(), T->wstart.end());
            if (hipMemcpy(T->wt, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(LBM_EDEVICE, "wall tile upload");
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

extern "C" int64_t lbm_tape_id(const lbm_ctx *c) {
    if (!c) return -1;
    return c->tape ? c->tape->id : 0;
}

extern "C" int lbm_tape_free(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    tape_release(c);
    return LBM_OK;
}

// Regularized faces: their closure's transpose (adjoint.hip) runs on single
// domains without a body force.
static bool has_regularized_face(const lbm_ctx *c) {
    for (int d = 0; d < c->ndomains; ++d) {
        const lbm_face *fc = c->batch ? c->dom[d].iface : c->iface;
        for (int f = 0; f < 6; ++f)
            if (fc[f].type == LBM_REG_VELOCITY || fc[f].type == LBM_REG_PRESSURE) return true;
    }
    return false;
}

namespace {
struct Backward {
    lbm_ctx *c;
    TapeState *T;
    BatchLaunch bl{};

    AdjLaunch launch(int op, int64_t t) {
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
        g.pending = (t > 0) ? 1 : 0;
        g.reg = has_regularized_face(c) ? 1 : 0;
        g.kbc = (c->collision == LBM_KBC) ? 1 : 0;
        if (c->batch) {
            g.batch = &bl.b;
            g.grid = bl.grid;
            g.block = bl.block;
        } else {
            c->pd.zh_pending = c->pf.zh_pending = g.pending;
        }
        g.walls.dom = T->wt;
        g.walls.face = T->wt ? T->wt + T->nwt : nullptr;
        g.walls.start = T->wt ? T->wt + 2 * T->nwt : nullptr;
        g.walls.n = T->nwt;
        g.walls.block = kWallBlock;
        return g;
    }

    // a natural-order view of a state image taken at time t: the image itself
    // when it is in natural order, else materialized into dst
    hipError_t natural(const void *img, int64_t t, void *dst, const void **out) {
        if (swapped_at(c, t)) {
            AdjLaunch g = launch(ADJ_MATERIALIZE, t);
            g.F = img;
            g.D = dst;
            hipError_t e = hipMemsetAsync(dst, 0, T->sbytes, c->stream);  // slots of solid cells stay defined
            if (e != hipSuccess) return e;
            *out = dst;
            return launch_adjoint(g);
        }
        *out = img;
        return hipSuccess;
    }

    // natural-order push step src -> dst from time t
    hipError_t push(const void *src, void *dst, int64_t t) {
        if (c->batch) {
            BatchLaunch g = bl;
            g.A = const_cast<void *>(src);
            return batch_launch_push(g, dst, (t > 0) ? 1 : 0);
        }
        c->pd.zh_pending = c->pf.zh_pending = (t > 0) ? 1 : 0;
        Launch g = make_launch(c);
        g.A = const_cast<void *>(src);
        g.B = dst;
        return launch_step(g, 2, c->s != nullptr);
    }
};
}  // namespace

static int backward_impl(lbm_ctx *c, const void *dL_drho, const void *dL_du, int dtype, float *dL_ds,
                         double *dL_dtau, double *dL_duw, void *dL_dfield, double *dL_dforce) {
    if (!c) return fail(LBM_EINVAL, "null context");
    const bool want_force = dL_dfield || dL_dforce;
    if ((dL_drho || dL_du || dL_dfield) && dtype != LBM_F64 && dtype != LBM_F32)
        return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
    if (!c->tape) return fail(LBM_ESTATE, "no tape recorded");
    if (has_regularized_face(c) && (c->batch || c->force_on || want_force))
        return fail(LBM_EUNSUPPORTED, "the adjoint of regularized faces covers single domains without a body force");
    if (c->nlinks) return fail(LBM_EUNSUPPORTED, "the adjoint of interpolated bounce-back is not implemented");
    if (c->collision == LBM_KBC && (c->force_on || want_force || c->batch || has_regularized_face(c)))
        return fail(LBM_EUNSUPPORTED, "the adjoint of the KBC collision covers single domains without a body force "
                                      "or regularized faces");
    if (c->collision != LBM_BGK && c->collision != LBM_KBC)
        return fail(LBM_EUNSUPPORTED, "the adjoint covers the BGK and KBC collisions");
    if (want_force && c->batch) return fail(LBM_EUNSUPPORTED, "body forces are not supported on batch contexts");
    if (c->tape_recording) lbm_tape_end(c);
    TapeState *T = c->tape;
    if (T->stale || T->had_s != (c->s != nullptr))
        return fail(LBM_ESTATE, "tau, a face, the solid cells, the solid fraction, the body force or the collision "
                                "changed after the tape began; record a new tape");
    if (c->moved_since_tape || c->t != T->t_end) return fail(LBM_ESTATE, "the state moved since the tape ended");
    (void)hipSetDevice(c->device);
    const int64_t fblocks = (c->N + 255) / 256;
    if (want_force && !T->dF) {
        int rc = dev_alloc(&T->dF, (size_t)3 * (size_t)c->N * compute_size(c), "dL/dF accumulator");
        if (!rc) rc = dev_alloc((void **)&T->frows, ((size_t)fblocks + 1) * 3 * sizeof(double), "dL/dF sums");
        if (rc) {
            dev_free(T->dF);
            dev_free((void *&)T->frows);
            return rc;
        }
    }
    refresh_params(c);
    Backward bw{c, T};
    if (c->batch) bw.bl = batch_launch_of(c);
    const int64_t n = T->t_end - T->t_begin;
    char *ring = static_cast<char *>(T->ring);
    hipError_t e = hipSuccess;
    int cur = 0;

    // seed a(t_end) from the final state
    const void *Fn = nullptr;
    e = bw.natural(c->A, c->t, ring, &Fn);
    if (e == hipSuccess) {
        AdjLaunch g = bw.launch(ADJ_SEED, c->t);
        g.F = Fn;
        g.grho = dL_drho;
        g.gu = dL_du;
        g.in_f64 = dtype == LBM_F64;
        g.Ao = T->abuf[cur];
        e = launch_adjoint(g);
    }
    if (e == hipSuccess) e = hipMemsetAsync(T->acc, 0, (size_t)T->rows * sizeof(double), c->stream);
    if (e == hipSuccess && T->nwt) e = hipMemsetAsync(T->accw, 0, (size_t)3 * T->nwt * sizeof(double), c->stream);
    if (e == hipSuccess && T->ds) e = hipMemsetAsync(T->ds, 0, (size_t)c->N * compute_size(c), c->stream);
    if (e == hipSuccess && want_force) e = hipMemsetAsync(T->dF, 0, (size_t)3 * (size_t)c->N * compute_size(c), c->stream);

    const int nseg = (int)((n + T->K - 1) / T->K);
    std::vector<const void *> S((size_t)T->K);
    for (int seg = nseg - 1; seg >= 0 && e == hipSuccess; --seg) {
        const int64_t t0 = T->t_begin + (int64_t)seg * T->K;
        const int64_t t1 = (t0 + T->K < T->t_end) ? t0 + T->K : T->t_end;
        // f(t0) .. f(t1 - 1) in natural order: the checkpoint, then push steps into the ring
        e = bw.natural(static_cast<char *>(T->ck) + (size_t)seg * T->sbytes, t0, ring, &S[0]);
        for (int64_t k = 1; k < t1 - t0 && e == hipSuccess; ++k) {
            void *dst = ring + (size_t)k * T->sbytes;
            e = bw.push(S[k - 1], dst, t0 + k - 1);
            S[k] = dst;
        }
        // adjoint steps backwards
        for (int64_t t = t1 - 1; t >= t0 && e == hipSuccess; --t) {
            AdjLaunch w = bw.launch(ADJ_WALLS, t);
            w.An = T->abuf[cur];
            w.accw = T->accw;
            e = launch_adjoint(w);
            if (e != hipSuccess) break;
            AdjLaunch g = bw.launch(ADJ_STEP, t);
            g.F = S[t - t0];
            g.An = T->abuf[cur];
            g.Ao = T->abuf[1 - cur];
            g.ds = c->s ? T->ds : nullptr;
            g.acc = T->acc;
            g.force = (c->force_on || want_force) ? 1 : 0;
            g.dF = want_force ? T->dF : nullptr;
            e = launch_adjoint(g);
            cur = 1 - cur;
        }
    }
    refresh_params(c);

    if (e == hipSuccess && dL_ds) {
        if (T->ds) {
            AdjLaunch g = bw.launch(ADJ_DS_OUT, c->t);
            g.ds = T->ds;
            g.ds_out = dL_ds;
            e = launch_adjoint(g);
        } else {
            e = hipMemsetAsync(dL_ds, 0, (size_t)c->N * sizeof(float), c->stream);
        }
    }
    // body-force gradient: the field's (scaled by eps), and its fixed-order sum
    double fsum[3] = {0.0, 0.0, 0.0};
    if (e == hipSuccess && want_force) {
        AdjLaunch g = bw.launch(ADJ_DF_OUT, c->t);
        g.dF = T->dF;
        g.df_out = dL_dfield;
        g.in_f64 = dtype == LBM_F64;
        g.eps = c->force_eps;
        g.acc = T->frows;
        e = launch_adjoint(g);
        if (e == hipSuccess)
            e = launch_rows_reduce(T->frows, fblocks, c->D, T->frows + (size_t)fblocks * 3, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(fsum, T->frows + (size_t)fblocks * 3, (size_t)c->D * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream);
    }
    // FP64 row sums, added on the host in a fixed order
    std::vector<double> acc((size_t)T->rows), accw((size_t)3 * T->nwt);
    if (e == hipSuccess) e = hipMemcpyAsync(acc.data(), T->acc, acc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && T->nwt)
        e = hipMemcpyAsync(accw.data(), T->accw, accw.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_backward");
    if (dL_dforce)
        for (int a = 0; a < c->D; ++a) dL_dforce[a] = fsum[a];
    const int nd = c->ndomains;
    std::vector<double> dtau((size_t)nd, 0.0), duw((size_t)nd * 18, 0.0);   // duw in internal faces / axes
    if (c->batch) {
        for (int d = 0; d < nd; ++d) {
            double sum = 0.0;
            for (int64_t r = c->dom[d].block0; r < c->dom[d].block0 + c->dom[d].nblocks; ++r) sum += acc[(size_t)r];
            dtau[d] = sum / (c->dom[d].tau * c->dom[d].tau);
        }
    } else {
        double sum = 0.0;
        for (int64_t r = 0; r < c->grid; ++r) sum += acc[(size_t)r];
        dtau[0] = sum / (c->tau * c->tau);
    }
    for (int k = 0; k < T->nwt; ++k)
        for (int a = 0; a < 3; ++a) duw[(size_t)T->wdom[k] * 18 + 3 * T->wface[k] + a] += accw[(size_t)3 * k + a];
    for (int d = 0; d < nd; ++d) {
        if (dL_dtau) dL_dtau[d] = dtau[d];
        if (dL_duw) {
            // internal faces / axes -> caller faces / axes
            double *o = dL_duw + (size_t)d * 18;
            const double *S18 = duw.data() + (size_t)d * 18;
            for (int k = 0; k < 18; ++k) o[k] = 0.0;
            for (int f = 0; f < 6; ++f)
                for (int a = 0; a < 3; ++a) {
                    const double v = S18[3 * f + a];
                    if (c->D == 3) o[3 * f + a] = v;
                    else if (f >= 2 && a >= 1) o[3 * (f - 2) + (a - 1)] = v;
                }
        }
    }
    return LBM_OK;
}

extern "C" int lbm_backward(lbm_ctx *c, const void *dL_drho, const void *dL_du, int dtype, float *dL_ds,
                            double *dL_dtau, double *dL_duw) {
    return backward_impl(c, dL_drho, dL_du, dtype, dL_ds, dL_dtau, dL_duw, nullptr, nullptr);
}

extern "C" int lbm_backward_force(lbm_ctx *c, const void *dL_drho, const void *dL_du, int dtype, float *dL_ds,
                                  double *dL_dtau, double *dL_duw, void *dL_dfield, double *dL_dforce) {
    return backward_impl(c, dL_drho, dL_du, dtype, dL_ds, dL_dtau, dL_duw, dL_dfield, dL_dforce);
}
