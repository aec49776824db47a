// batch.hip -- batched independent domains: creation, tile list, stepping
// (one launch per step, or one persistent cooperative launch for n steps),
// moments, and the tile-shape / launch-mode autotuner.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"

using namespace lbm;

namespace lbm {
struct BatchState {
    int B = 128;                 // tile size (cells per workgroup)
    int persistent = 0;          // 1: one cooperative launch for n steps
    bool tuned = false;
    int ntiles = 0;
    int coop_grid = 0;           // resident workgroups for the persistent kernel
    std::vector<int> tile_dom, tile_start;
    std::vector<int64_t> stoff, cell0;
    void *P = nullptr;           // Params<CT>[ndom]
    void *FT = nullptr;          // FaceTab<CT>[ndom]
    int *tile_dom_d = nullptr, *tile_start_d = nullptr;
    int64_t *stoff_d = nullptr, *cell0_d = nullptr;
    std::string key;             // autotune cache key
};
}  // namespace lbm

static size_t cts(const lbm_ctx *c) { return c->opt.storage == LBM_F64 ? 8 : 4; }

void lbm::batch_release(lbm_ctx *c) {
    if (!c->bs) return;
    BatchState *S = c->bs;
    dev_free(S->P);
    dev_free(S->FT);
    dev_free((void *&)S->tile_dom_d);
    dev_free((void *&)S->tile_start_d);
    dev_free((void *&)S->stoff_d);
    dev_free((void *&)S->cell0_d);
    delete S;
    c->bs = nullptr;
}

// tile tables for tile size B (host side); per-domain block ranges for the sums
static void build_tiles(lbm_ctx *c, int B) {
    BatchState *S = c->bs;
    S->B = B;
    S->tile_dom.clear();
    S->tile_start.clear();
    for (int d = 0; d < c->ndomains; ++d) {
        Domain &D = c->dom[d];
        D.block0 = (int64_t)S->tile_dom.size();
        for (int64_t s = 0; s < D.N; s += B) {
            S->tile_dom.push_back(d);
            S->tile_start.push_back((int)s);
        }
        D.nblocks = (int64_t)S->tile_dom.size() - D.block0;
    }
    S->ntiles = (int)S->tile_dom.size();
    c->grid = S->ntiles;
}

template <class CT>
static void domain_params(Params<CT> &p, const lbm_ctx *c, const Domain &D, const FaceTab<CT> *ft) {
    std::memset(&p, 0, sizeof p);
    p.nX = D.nX;
    p.nY = D.nY;
    p.nZ = D.nZ;
    p.sX = D.nY * D.nZ;
    p.sY = D.nZ;
    p.zblocks = 1;
    p.plane = tiled_cells(D.N);
    p.omega = (CT)(1.0 / D.tau);
    p.rho0 = (CT)c->opt.rho0;
    for (int f = 0; f < 6; ++f) {
        const lbm_face &F = D.iface[f];
        p.ftype[f] = (uint8_t)F.type;
        for (int a = 0; a < 3; ++a) p.uw[f][a] = (CT)F.u[a];
        p.frho[f] = (CT)F.rho;
        if (F.type == LBM_WALL) {
            p.wallmask |= 1u << f;
            if (F.u[0] == 0.0 && F.u[1] == 0.0 && F.u[2] == 0.0) p.staticmask |= 1u << f;
        }
        if (F.type == LBM_ZOUHE_VELOCITY || F.type == LBM_ZOUHE_PRESSURE || F.type == LBM_REG_VELOCITY ||
            F.type == LBM_REG_PRESSURE)
            p.zhmask |= 1u << f;
        if (F.type == LBM_PERIODIC) p.permask |= 1u << f;
    }
    p.ft = ft;
}

template <class CT>
static int upload_params(lbm_ctx *c) {
    BatchState *S = c->bs;
    const int n = c->ndomains;
    if (!S->P) {
        int rc = dev_alloc(&S->P, (size_t)n * sizeof(Params<CT>), "batch parameters");
        if (!rc) rc = dev_alloc(&S->FT, (size_t)n * sizeof(FaceTab<CT>), "batch face tables");
        if (rc) return rc;
    }
    std::vector<Params<CT>> hp(n);
    std::vector<FaceTab<CT>> hf(n);
    for (int d = 0; d < n; ++d) {
        FaceTab<CT> &F = hf[d];
        std::memset(&F, 0, sizeof F);
        for (int f = 0; f < 6; ++f) {
            for (int a = 0; a < 3; ++a) F.uw[f][a] = (CT)c->dom[d].iface[f].u[a];
            F.rho[f] = (CT)c->dom[d].iface[f].rho;
            F.type[f] = c->dom[d].iface[f].type;
        }
        domain_params(hp[d], c, c->dom[d], static_cast<const FaceTab<CT> *>(S->FT) + d);
    }
    hipError_t e = hipMemcpy(S->P, hp.data(), hp.size() * sizeof(Params<CT>), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(S->FT, hf.data(), hf.size() * sizeof(FaceTab<CT>), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch parameter upload");
    return LBM_OK;
}

// upload the tile tables and the per-domain reduction ranges for tile size B
static int upload_tiles(lbm_ctx *c, int B) {
    BatchState *S = c->bs;
    build_tiles(c, B);
    dev_free((void *&)S->tile_dom_d);
    dev_free((void *&)S->tile_start_d);
    int rc = dev_alloc((void **)&S->tile_dom_d, (size_t)S->ntiles * sizeof(int), "tile list");
    if (!rc) rc = dev_alloc((void **)&S->tile_start_d, (size_t)S->ntiles * sizeof(int), "tile list");
    if (rc) return rc;
    std::vector<int64_t> b(c->ndomains), e(c->ndomains);
    for (int d = 0; d < c->ndomains; ++d) {
        b[d] = c->dom[d].block0;
        e[d] = c->dom[d].block0 + c->dom[d].nblocks;
    }
    hipError_t he = hipMemcpy(S->tile_dom_d, S->tile_dom.data(), S->ntiles * sizeof(int), hipMemcpyHostToDevice);
    if (he == hipSuccess)
        he = hipMemcpy(S->tile_start_d, S->tile_start.data(), S->ntiles * sizeof(int), hipMemcpyHostToDevice);
    if (he == hipSuccess && c->rbeg) he = hipMemcpy(c->rbeg, b.data(), b.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (he == hipSuccess && c->rend) he = hipMemcpy(c->rend, e.data(), e.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (he != hipSuccess) return hip_fail(he, "tile list upload");
    // resident workgroups for the persistent kernel
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = batch_persistent_occupancy(c->lattice, c->opt.storage, B);
    S->coop_grid = per_cu * cus;
    if (S->coop_grid > S->ntiles) S->coop_grid = S->ntiles;
    return LBM_OK;
}

// Each domain's state: Q sub-planes of its cells rounded up to whole tiles of
// the population layout (core.hpp, pidx), domains back to back.
void lbm::batch_layout(lbm_ctx *c) {
    BatchState *S = c->bs;
    int64_t so = 0;
    for (int d = 0; d < c->ndomains; ++d) {
        S->stoff[d] = so;
        so += (int64_t)c->Q * tiled_cells(c->dom[d].N);
    }
    c->plane = so / c->Q;  // Q * plane = total state elements
}

int lbm::batch_upload(lbm_ctx *c) {
    BatchState *S = c->bs;
    if (!S->stoff_d) {
        int rc = dev_alloc((void **)&S->stoff_d, (size_t)c->ndomains * sizeof(int64_t), "batch offsets");
        if (!rc) rc = dev_alloc((void **)&S->cell0_d, (size_t)c->ndomains * sizeof(int64_t), "batch offsets");
        if (rc) return rc;
        hipError_t e = hipMemcpy(S->stoff_d, S->stoff.data(), S->stoff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(S->cell0_d, S->cell0.data(), S->cell0.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "batch offsets upload");
    }
    int rc = (c->opt.storage == LBM_F64) ? upload_params<double>(c) : upload_params<float>(c);
    if (rc) return rc;
    return upload_tiles(c, S->B);
}

static BatchLaunch blaunch(lbm_ctx *c) {
    BatchState *S = c->bs;
    BatchLaunch g;
    std::memset(&g, 0, sizeof g);
    g.lattice = c->lattice;
    g.storage = c->opt.storage;
    g.b.P = S->P;
    g.b.tile_dom = S->tile_dom_d;
    g.b.tile_start = S->tile_start_d;
    g.b.stoff = S->stoff_d;
    g.b.cell0 = S->cell0_d;
    g.b.ntiles = S->ntiles;
    g.b.ndom = c->ndomains;
    g.b.ncells = c->N;
    g.A = c->A;
    g.block = (unsigned)S->B;
    g.grid = (unsigned)S->ntiles;
    g.stream = c->stream;
    return g;
}

BatchLaunch lbm::batch_launch_of(lbm_ctx *c) { return blaunch(c); }

hipError_t lbm::batch_init(lbm_ctx *c, const void *rho, const void *u, bool f64) {
    return batch_launch_init(blaunch(c), rho, u, f64 ? 1 : 0);
}

hipError_t lbm::batch_step(lbm_ctx *c) {
    return batch_launch_step(blaunch(c), (int)(c->t & 1), c->t > 0 ? 1 : 0);
}

hipError_t lbm::batch_moments(lbm_ctx *c, bool odd, void *rho, void *u, bool f64, double *partial) {
    return batch_launch_moments(blaunch(c), odd, c->t > 0 ? 1 : 0, rho, u, f64 ? 1 : 0, partial);
}

// n steps with one cooperative launch (all workgroups resident)
hipError_t lbm::batch_persistent_steps(lbm_ctx *c, int n) {
    BatchLaunch g = blaunch(c);
    g.grid = (unsigned)c->bs->coop_grid;
    if (g.grid == 0) return hipErrorInvalidConfiguration;
    return batch_launch_persistent(g, n, c->t);
}

bool lbm::batch_uses_persistent(const lbm_ctx *c) { return c->bs && c->bs->persistent && c->bs->coop_grid > 0; }

// ---- autotuner ----------------------------------------------------------------
static std::string cache_path() {
    const char *p = std::getenv("LBM_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char *h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/lbm_mi355x_autotune.txt";
}

static bool cache_lookup(const std::string &key, int &B, int &mode) {
    FILE *f = std::fopen(cache_path().c_str(), "r");
    if (!f) return false;
    char k[512];
    int b, m;
    double ms;
    bool found = false;
    while (std::fscanf(f, "%511s %d %d %lf", k, &b, &m, &ms) == 4)
        if (key == k) {
            B = b;
            mode = m;
            found = true;
        }
    std::fclose(f);
    return found;
}

static void cache_store(const std::string &key, int B, int mode, double ms) {
    const std::string path = cache_path();
    const std::string dir = path.substr(0, path.find_last_of('/'));
    std::string cmd = "mkdir -p '" + dir + "' 2>/dev/null";
    (void)!std::system(cmd.c_str());
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %.6f\n", key.c_str(), B, mode, ms);
    std::fclose(f);
}

// Time `steps` steps of each (tile size, launch mode) candidate from the
// current state, restoring the state after each; keep the fastest.
int lbm::batch_autotune(lbm_ctx *c) {
    BatchState *S = c->bs;
    if (S->tuned) return LBM_OK;
    S->tuned = true;
    const char *env = std::getenv("LBM_AUTOTUNE");
    int B = S->B, mode = S->persistent;
    const std::string key = S->key + "_s" + std::to_string(c->opt.storage);
    if (cache_lookup(key, B, mode)) {
        S->persistent = mode;
        return (B != S->B) ? upload_tiles(c, B) : LBM_OK;
    }
    if (env && env[0] == '0') return LBM_OK;
    const size_t bytes = (size_t)c->Q * (size_t)c->plane * storage_size(c->opt.storage);
    void *save = nullptr;
    if (dev_alloc(&save, bytes, "autotune scratch") != LBM_OK) return LBM_OK;  // tuning is optional
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int steps = 8;
    double best = 1e30;
    int bestB = S->B, bestM = 0;
    const int64_t t_saved = c->t;
    hipError_t err = hipMemcpyAsync(save, c->A, bytes, hipMemcpyDeviceToDevice, c->stream);
    for (int cand_B : {64, 128, 256}) {
        if (err != hipSuccess) break;
        if (upload_tiles(c, cand_B) != LBM_OK) break;
        for (int m = 0; m < 2 && err == hipSuccess; ++m) {
            if (m == 1 && S->coop_grid == 0) continue;
            S->persistent = m;
            // warm-up then timed steps
            for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
                if (rep == 1) err = hipEventRecord(e0, c->stream);
                if (m == 1) {
                    err = batch_persistent_steps(c, steps);
                    c->t += steps;
                } else {
                    for (int k = 0; k < steps && err == hipSuccess; ++k) {
                        err = batch_step(c);
                        c->t += 1;
                    }
                }
            }
            if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
            if (err == hipSuccess && ms < best) {
                best = ms;
                bestB = cand_B;
                bestM = m;
            }
            c->t = t_saved;
            if (err == hipSuccess) err = hipMemcpyAsync(c->A, save, bytes, hipMemcpyDeviceToDevice, c->stream);
        }
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free(save);
    c->t = t_saved;
    if (err != hipSuccess) return hip_fail(err, "batch autotune");
    S->persistent = bestM;
    int rc = upload_tiles(c, bestB);
    if (rc) return rc;
    cache_store(key, bestB, bestM, best / steps);
    return LBM_OK;
}

extern "C" int lbm_batch_tuning(lbm_ctx *c, int tile, int persistent) {
    if (!c || !c->batch) return fail(LBM_EINVAL, "not a batch context");
    if (tile != 0 && tile != 64 && tile != 128 && tile != 256) return fail(LBM_EINVAL, "tile must be 0, 64, 128 or 256");
    if (persistent < -1 || persistent > 1) return fail(LBM_EINVAL, "persistent must be -1, 0 or 1");
    BatchState *S = c->bs;
    if (tile == 0 && persistent == -1) {  // back to automatic
        S->tuned = false;
        return LBM_OK;
    }
    S->tuned = true;
    if (persistent >= 0) S->persistent = persistent;
    if (tile != 0 && tile != S->B) {
        if (c->A) {
            int rc = upload_tiles(c, tile);
            if (rc) return rc;
        } else {
            S->B = tile;
        }
    }
    drop_graph(c);
    return LBM_OK;
}

extern "C" int lbm_batch_config(const lbm_ctx *c, int *tile, int *persistent) {
    if (!c || !c->batch) return fail(LBM_EINVAL, "not a batch context");
    if (tile) *tile = c->bs->B;
    if (persistent) *persistent = batch_uses_persistent(c) ? 1 : 0;
    return LBM_OK;
}

// ---- creation -------------------------------------------------------------------
static void map_domain_faces(Domain &D, int Dim, const lbm_bc *bc) {
    for (int f = 0; f < 6; ++f) {
        D.iface[f] = lbm_face{};
        D.iface[f].type = LBM_PERIODIC;
        D.iface[f].rho = 1.0;
    }
    if (!bc) return;
    if (Dim == 3) {
        for (int f = 0; f < 6; ++f) D.iface[f] = bc->face[f];
    } else {
        for (int f = 0; f < 4; ++f) {
            lbm_face G = bc->face[f];
            G.u[0] = 0.0;
            G.u[1] = bc->face[f].u[0];
            G.u[2] = bc->face[f].u[1];
            D.iface[f + 2] = G;
        }
    }
}

extern "C" lbm_ctx *lbm_create_batch(int lattice, int n, const int *nx, const int *ny, const int *nz,
                                     const double *tau, const lbm_bc *bcs) {
    if (n < 1 || !nx || !ny || !tau || (lattice != LBM_D2Q9 && !nz)) {
        fail(LBM_EINVAL, "n >= 1 and the nx, ny, tau arrays (and nz for 3-D) are required");
        return nullptr;
    }
    int64_t total = 0;
    for (int d = 0; d < n; ++d) {
        const int z = nz ? nz[d] : 0;
        if (validate_domain(lattice, nx[d], ny[d], z, tau[d], bcs ? &bcs[d] : nullptr) != LBM_OK) {
            std::string m = lbm_last_error();
            fail(LBM_EINVAL, "domain %d: %s", d, m.c_str());
            return nullptr;
        }
        const int64_t Nd = (int64_t)nx[d] * ny[d] * ((lattice == LBM_D2Q9 || z < 1) ? 1 : z);
        if (Nd >= (1 << 24)) {
            fail(LBM_EINVAL, "domain %d has %lld cells; batch domains are limited to 2^24 - 1 cells", d, (long long)Nd);
            return nullptr;
        }
        total += Nd;
    }
    if (total >= ((int64_t)1 << 31)) {
        fail(LBM_EINVAL, "batch has %lld cells; the limit is 2^31 - 1", (long long)total);
        return nullptr;
    }
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) {
        fail(LBM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    c->bs = new (std::nothrow) BatchState();
    if (!c->bs) {
        delete c;
        fail(LBM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    c->batch = true;
    c->lattice = lattice;
    c->Q = lattice == LBM_D2Q9 ? 9 : (lattice == LBM_D3Q19 ? 19 : 27);
    c->D = lattice == LBM_D2Q9 ? 2 : 3;
    c->ndomains = n;
    c->opt.storage = LBM_F32;
    c->opt.compute = LBM_F32;
    c->opt.pattern = LBM_INPLACE;
    c->opt.rho0 = 1.0;
    c->tau = tau[0];
    c->dom.resize(n);
    BatchState *S = c->bs;
    S->stoff.resize(n);
    S->cell0.resize(n);
    int64_t c0 = 0;
    std::string key = "L" + std::to_string(lattice) + "n" + std::to_string(n);
    uint64_t hsh = 1469598103934665603ull;
    for (int d = 0; d < n; ++d) {
        Domain &D = c->dom[d];
        D.nx = nx[d];
        D.ny = ny[d];
        D.nz = (lattice == LBM_D2Q9) ? 1 : nz[d];
        if (c->D == 3) {
            D.nX = D.nx;
            D.nY = D.ny;
            D.nZ = D.nz;
        } else {
            D.nX = 1;
            D.nY = D.nx;
            D.nZ = D.ny;
        }
        D.N = (int64_t)D.nX * D.nY * D.nZ;
        D.tau = tau[d];
        D.cell0 = c0;
        map_domain_faces(D, c->D, bcs ? &bcs[d] : nullptr);
        S->cell0[d] = c0;
        c0 += D.N;
        for (int64_t v : {(int64_t)D.nx, (int64_t)D.ny, (int64_t)D.nz}) hsh = (hsh ^ (uint64_t)v) * 1099511628211ull;
    }
    c->N = c0;
    batch_layout(c);
    c->nx = c->ny = c->nz = 0;
    S->B = 128;
    build_tiles(c, 64);    // partial-sum rows sized for the smallest tile
    c->bgrid = S->ntiles;
    build_tiles(c, S->B);
    char hb[32];
    std::snprintf(hb, sizeof hb, "h%016llx", (unsigned long long)hsh);
    S->key = key + hb;
    return c;
}

extern "C" int lbm_batch_offsets(const lbm_ctx *c, int64_t *off) {
    if (!c || !off) return fail(LBM_EINVAL, "null argument");
    if (!c->batch) return fail(LBM_EINVAL, "not a batch context");
    for (int d = 0; d < c->ndomains; ++d) off[d] = c->bs->cell0[d];
    off[c->ndomains] = c->N;
    return LBM_OK;
}
