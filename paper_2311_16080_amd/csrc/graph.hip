// graph.hip -- capture of n forward steps into one HIP graph (replayed with a
// single launch).
#include <hip/hip_runtime.h>

#include <utility>

#include "ctx.hpp"

using namespace lbm;

void lbm::drop_graph(lbm_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_steps = 0;
}

static int capture_steps(lbm_ctx *c, int n);

extern "C" int lbm_capture_graph(lbm_ctx *c, int n) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (n < 1) return fail(LBM_EINVAL, "n_steps must be >= 1");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised");
    if (c->tape_recording) return fail(LBM_ESTATE, "cannot capture while a tape is recording");
    (void)hipSetDevice(c->device);
    drop_graph(c);
    if (c->batch) {
        int rc = batch_autotune(c);
        if (rc) return rc;
    }
    // the legacy null stream cannot be captured: capture on a stream of our own
    // (the graph keeps no reference to it) and replay on the context's stream
    hipStream_t user = c->stream, own = nullptr;
    if (!user) {
        hipError_t se = hipStreamCreateWithFlags(&own, hipStreamNonBlocking);
        if (se != hipSuccess) return hip_fail(se, "capture stream");
        c->stream = own;
    }
    const int rc = capture_steps(c, n);
    c->stream = user;
    if (own) (void)hipStreamDestroy(own);
    return rc;
}

static int capture_steps(lbm_ctx *c, int n) {
    const int64_t t0 = c->t;
    void *A0 = c->A, *B0 = c->B;
    hipGraph_t g = nullptr;
    hipError_t e = hipSuccess, le = hipSuccess;
    bool captured = false;
    if (c->batch && batch_uses_persistent(c)) {
        // one persistent cooperative launch for all n steps, if the runtime can
        // capture it; otherwise fall back to one node per step
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            le = batch_persistent_steps(c, n);
            e = hipStreamEndCapture(c->stream, &g);
            if (le == hipSuccess && e == hipSuccess && g) {
                captured = true;
                c->graph_persistent = 1;
            } else {
                if (g) (void)hipGraphDestroy(g);
                g = nullptr;
                (void)hipGetLastError();
                le = e = hipSuccess;
            }
        } else {
            (void)hipGetLastError();
            e = hipSuccess;
        }
    }
    if (!captured) {
        c->graph_persistent = 0;
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        for (int k = 0; k < n && le == hipSuccess; ++k) le = forward_step(c);
        e = hipStreamEndCapture(c->stream, &g);
    }
    c->t = t0;
    c->A = A0;
    c->B = B0;
    refresh_params(c);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "kernel launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    c->graph = g;
    c->graph_exec = x;
    c->graph_steps = n;
    c->graph_t0 = t0;
    c->graph_A = A0;
    return LBM_OK;
}

extern "C" int lbm_graph_launch(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (!c->graph_exec) return fail(LBM_ESTATE, "no graph captured");
    if (c->tape_recording) return fail(LBM_ESTATE, "cannot replay a graph while a tape is recording");
    const bool same_parity = ((c->t ^ c->graph_t0) & 1) == 0;
    const bool same_buffers = c->A == c->graph_A;
    bool zh = c->pf.zhmask != 0;
    for (const Domain &D : c->dom)
        for (const lbm_face &F : D.iface)
            zh = zh || F.type == LBM_ZOUHE_VELOCITY || F.type == LBM_ZOUHE_PRESSURE || F.type == LBM_REG_VELOCITY ||
                 F.type == LBM_REG_PRESSURE;
    // the pull pattern's first step after an init is the local one
    const bool first = (c->t > 0) != (c->graph_t0 > 0);
    if (!same_buffers || (c->opt.pattern == LBM_INPLACE && !same_parity) || ((zh || c->opt.pattern == LBM_PULL) && first))
        return fail(LBM_ESTATE, "the state's step parity / buffers differ from those at capture");
    (void)hipSetDevice(c->device);
    hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    c->t += c->graph_steps;
    // buffer swaps of the replayed steps (push and pull steps swap)
    int swaps = 0;
    for (int64_t k = 0; k < c->graph_steps; ++k) swaps += step_mode_at(c, c->graph_t0 + k) >= 2 ? 1 : 0;
    if (swaps & 1) std::swap(c->A, c->B);
    c->moved_since_tape = true;
    refresh_params(c);
    return LBM_OK;
}
