// capi.hip -- host side of liblbm.so: the C-ABI declared in include/lbm.h.
//
// A context owns the population state (one buffer for the in-place pattern,
// two for the double-buffer one), the solid flags, the solid-fraction field,
// reduction scratch, the adjoint tape and captured graphs.  Every argument is
// checked before any device work.  Device memory is allocated on the device
// that is current at the first lbm_init_equilibrium.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace lbm;

static thread_local std::string g_err;

int lbm::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int lbm::hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(LBM_ENOMEM, "%s: out of device memory", what);
    return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *lbm_last_error(void) { return g_err.c_str(); }

extern "C" const char *lbm_version(void) { return "lbm-mi355x 0.2 (gfx950)"; }

template <class L>
static int lattice_info_t(int32_t *c, double *w) {
    for (int i = 0; i < L::Q; ++i) {
        if (c) {
            // internal (X, Y, Z) -> caller axes (2-D: (Y, Z) -> (x, y))
            if (L::D == 3) {
                for (int a = 0; a < 3; ++a) c[3 * i + a] = L::c[i][a];
            } else {
                c[3 * i + 0] = L::c[i][1];
                c[3 * i + 1] = L::c[i][2];
                c[3 * i + 2] = 0;
            }
        }
        if (w) w[i] = weight<L>(i);
    }
    return L::Q;
}

extern "C" int lbm_lattice_info(int lattice, int32_t *c, double *w) {
    switch (lattice) {
        case LBM_D2Q9: return lattice_info_t<D2Q9>(c, w);
        case LBM_D3Q19: return lattice_info_t<D3Q19>(c, w);
        case LBM_D3Q27: return lattice_info_t<D3Q27>(c, w);
    }
    return fail(LBM_EINVAL, "unknown lattice %d", lattice);
}

// ---------------------------------------------------------------------------
// validation and setup
// ---------------------------------------------------------------------------
static int lattice_q(int lattice) { return lattice == LBM_D2Q9 ? 9 : (lattice == LBM_D3Q19 ? 19 : 27); }

int lbm::validate_domain(int lattice, int nx, int ny, int nz, double tau, const lbm_bc *bc) {
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q27)
        return fail(LBM_EINVAL, "unknown lattice %d", lattice);
    if (nx < 1 || ny < 1) return fail(LBM_EINVAL, "nx, ny must be >= 1 (got %d, %d)", nx, ny);
    if (lattice == LBM_D2Q9) {
        if (nz != 0 && nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz = 0 or 1 (got %d)", nz);
    } else if (nz < 1) {
        return fail(LBM_EINVAL, "3-D lattices need nz >= 1 (got %d)", nz);
    }
    const int64_t N = (int64_t)nx * ny * (nz < 1 ? 1 : nz);
    if (N >= ((int64_t)1 << 31)) return fail(LBM_EINVAL, "grid has %lld cells; the limit is 2^31 - 1", (long long)N);
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(LBM_EINVAL, "tau must be finite and > 1/2 (got %g)", tau);
    if (!bc) return LBM_OK;
    const int naxes = (lattice == LBM_D2Q9) ? 2 : 3;
    const int n[3] = {nx, ny, nz < 1 ? 1 : nz};
    int open_axis = -1;
    for (int a = 0; a < naxes; ++a) {
        const lbm_face &lo = bc->face[2 * a], &hi = bc->face[2 * a + 1];
        for (const lbm_face *F : {&lo, &hi}) {
            if (F->type < LBM_PERIODIC || F->type > LBM_REG_PRESSURE)
                return fail(LBM_EINVAL, "face %d: unknown boundary type %d", (int)(F - bc->face), F->type);
            for (int c = 0; c < 3; ++c)
                if (!std::isfinite(F->u[c])) return fail(LBM_EINVAL, "face %d: velocity not finite", (int)(F - bc->face));
        }
        if ((lo.type == LBM_PERIODIC) != (hi.type == LBM_PERIODIC))
            return fail(LBM_EINVAL, "axis %d: periodic must be set on both faces or neither", a);
        for (int sd = 0; sd < 2; ++sd) {
            const lbm_face &F = bc->face[2 * a + sd];
            if (F.type == LBM_WALL && F.u[a] != 0.0)
                return fail(LBM_EINVAL, "face %d: a wall velocity must be tangential", 2 * a + sd);
            const bool vel = F.type == LBM_ZOUHE_VELOCITY || F.type == LBM_REG_VELOCITY;
            const bool pres = F.type == LBM_ZOUHE_PRESSURE || F.type == LBM_REG_PRESSURE;
            if (vel && std::fabs(F.u[a]) >= 1.0)
                return fail(LBM_EINVAL, "face %d: inlet normal velocity must be below 1", 2 * a + sd);
            if ((pres || F.type == LBM_EQ_OUTFLOW) && !(F.rho > 0.0))
                return fail(LBM_EINVAL, "face %d: density must be > 0", 2 * a + sd);
            if (vel || pres || F.type == LBM_EQ_OUTFLOW) {
                if (open_axis >= 0 && open_axis != a)
                    return fail(LBM_EINVAL, "Zou-He / regularized / outflow faces must all lie on one axis");
                open_axis = a;
                if (n[a] < 2) return fail(LBM_EINVAL, "axis %d carries an open face and needs >= 2 cells", a);
            }
        }
        if (lattice == LBM_D2Q9) {
            for (int sd = 0; sd < 2; ++sd)
                if (bc->face[2 * a + sd].u[2] != 0.0)
                    return fail(LBM_EINVAL, "face %d: a 2-D lattice has no z velocity", 2 * a + sd);
        }
    }
    return LBM_OK;
}

template <class CT>
static const FaceTab<CT> *face_table(const lbm_ctx *c);
template <>
const FaceTab<double> *face_table<double>(const lbm_ctx *c) { return c->ftd; }
template <>
const FaceTab<float> *face_table<float>(const lbm_ctx *c) { return c->ftf; }

template <class CT>
static void host_face_table(FaceTab<CT> &F, const lbm_face *iface) {
    std::memset(&F, 0, sizeof F);
    for (int f = 0; f < 6; ++f) {
        for (int a = 0; a < 3; ++a) F.uw[f][a] = (CT)iface[f].u[a];
        F.rho[f] = (CT)iface[f].rho;
        F.type[f] = iface[f].type;
    }
}

// Upload the face tables (device copies of the per-face data).
static int upload_faces(lbm_ctx *c) {
    if (!c->ftd) {
        int rc = dev_alloc((void **)&c->ftd, sizeof(FaceTab<double>), "face table");
        if (!rc) rc = dev_alloc((void **)&c->ftf, sizeof(FaceTab<float>), "face table");
        if (rc) return rc;
    }
    FaceTab<double> hd;
    FaceTab<float> hf;
    host_face_table(hd, c->iface);
    host_face_table(hf, c->iface);
    hipError_t e = hipMemcpy(c->ftd, &hd, sizeof hd, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->ftf, &hf, sizeof hf, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "face table upload");
    return LBM_OK;
}

// Fill the internal-axis parameter block (both precisions).
template <class CT>
static void fill_params(Params<CT> &p, const lbm_ctx *c) {
    std::memset(&p, 0, sizeof p);
    p.nX = c->nX;
    p.nY = c->nY;
    p.nZ = c->nZ;
    p.sX = c->nY * c->nZ;
    p.sY = c->nZ;
    p.zblocks = c->zblocks;
    p.plane = c->plane;
    p.omega = (CT)(1.0 / c->tau);
    p.rho0 = (CT)c->opt.rho0;
    for (int f = 0; f < 6; ++f) {
        const lbm_face &F = c->iface[f];
        p.ftype[f] = (uint8_t)F.type;
        for (int a = 0; a < 3; ++a) p.uw[f][a] = (CT)F.u[a];
        p.frho[f] = (CT)F.rho;
        if (F.type == LBM_WALL) {
            p.wallmask |= 1u << f;
            if (F.u[0] == 0.0 && F.u[1] == 0.0 && F.u[2] == 0.0) p.staticmask |= 1u << f;
        }
        if (F.type == LBM_ZOUHE_VELOCITY || F.type == LBM_ZOUHE_PRESSURE || F.type == LBM_REG_VELOCITY ||
            F.type == LBM_REG_PRESSURE)
            p.zhmask |= 1u << f;   // faces closed at read time
        if (F.type == LBM_PERIODIC) p.permask |= 1u << f;
    }
    p.zh_pending = c->t > 0 ? 1 : 0;
    p.xcd_remap = c->xcd_remap;
    // measured: with the wall path, aligned rows (no rotation) are as fast or
    // faster on every lattice; the rotation stays available for measurement
    p.zrot = (c->zrot > 0 && c->nZ >= 64 && !c->flat) ? 32 : 0;
    p.flat = c->flat;
    p.spk = c->split;
    p.nh = c->N / 2;
    p.ft = face_table<CT>(c);
    p.flags = c->flags;
    p.nbm = c->nbm;
    p.s = c->s;
    if (c->force_on) {
        // caller axis a -> internal axis (2-D: x, y -> Y, Z)
        const int off = (c->D == 3) ? 0 : 1;
        const CT *field = static_cast<const CT *>(c->force_field);
        for (int a = 0; a < c->D; ++a) {
            p.fu[a + off] = (CT)c->force_u[a];
            p.fld[a + off] = field ? field + (int64_t)a * c->N : nullptr;
        }
        p.feps = (CT)c->force_eps;
    }
}

void lbm::refresh_params(lbm_ctx *c) {
    fill_params(c->pd, c);
    fill_params(c->pf, c);
}

// internal faces / velocities from the caller's (external) description
static void map_faces(lbm_ctx *c, const lbm_bc *bc) {
    for (int f = 0; f < 6; ++f) {
        c->iface[f] = lbm_face{};
        c->iface[f].type = LBM_PERIODIC;
        c->iface[f].rho = 1.0;
    }
    if (!bc) return;
    if (c->D == 3) {
        for (int f = 0; f < 6; ++f) c->iface[f] = bc->face[f];
    } else {
        // 2-D (x, y) -> internal (Y, Z); internal X is a dummy axis of length 1
        for (int f = 0; f < 4; ++f) {
            lbm_face F = bc->face[f];
            lbm_face G = F;
            G.u[0] = 0.0;
            G.u[1] = F.u[0];
            G.u[2] = F.u[1];
            c->iface[f + 2] = G;
        }
    }
}

static void setup_mapping(lbm_ctx *c);

static void setup_shape(lbm_ctx *c, int lattice, int nx, int ny, int nz, double tau) {
    c->lattice = lattice;
    c->Q = lattice_q(lattice);
    c->D = lattice == LBM_D2Q9 ? 2 : 3;
    c->nx = nx;
    c->ny = ny;
    c->nz = (lattice == LBM_D2Q9) ? 1 : nz;
    if (c->D == 3) {
        c->nX = nx;
        c->nY = ny;
        c->nZ = nz;
    } else {
        c->nX = 1;
        c->nY = nx;
        c->nZ = ny;
    }
    c->N = (int64_t)c->nX * c->nY * c->nZ;
    // values per direction: the cells rounded up to whole tiles of the
    // population layout (core.hpp, pidx)
    c->plane = tiled_cells(c->N);
    c->tau = tau;
    setup_mapping(c);
}

// Lanes -> cells.  2-byte storage on a 3-D box of even nX runs in split pairs
// (the two X-halves share each 32-bit word, core.hpp): blocks of 256 lanes in
// storage order, and one lane per pair in the two-cell step.
static void setup_mapping(lbm_ctx *c) {
    const bool two = c->opt.storage == LBM_F16 || c->opt.storage == LBM_BF16;
    c->split = (two && c->split_req != 0 && c->pair && !c->batch && c->D == 3 && c->nX >= 4 && c->nX % 2 == 0) ? 1 : 0;
    if (c->split) {
        c->flat = 1;
        c->block = 256;
        c->zblocks = 1;
        c->grid = (c->N + 255) / 256;
        return;
    }
    // threads per block along Z: LBM_BLOCK if set, else the size among 256 /
    // 128 / 192 that launches the fewest lanes per row (ties: in that order;
    // measured on a 768 x 256 x 384 channel: 128 lanes per block run 20%
    // faster than 256, whose second block per row is half idle, and 7% faster
    // than 192)
    const int r64 = (c->nZ + 63) / 64 * 64;
    // rows whose length is not a multiple of 64 cells: blocks of 256 consecutive
    // cells of the whole grid instead of row chunks (aligned, fully occupied
    // wavefronts; measured on 256 x 256 x 300: row chunks start misaligned in
    // every row and leave 22% of the lanes idle)
    c->flat = (c->flat_req >= 0) ? c->flat_req : ((c->nZ % 64) != 0 ? 1 : 0);
    if (c->flat) {
        c->block = c->block_req > 0 ? c->block_req : 256;
        c->zblocks = 1;
        c->grid = (c->N + c->block - 1) / c->block;
        return;
    }
    int blk = r64;
    if (c->block_req > 0) {
        if (blk > c->block_req) blk = c->block_req;
    } else if (r64 > 128) {
        int best = 0;
        for (int b : {256, 128, 192}) {
            const int lanes = (c->nZ + b - 1) / b * b;
            if (best == 0 || lanes < (c->nZ + best - 1) / best * best) best = b;
        }
        blk = best;
    }
    c->block = blk;
    c->zblocks = (c->nZ + blk - 1) / blk;
    c->grid = (int64_t)c->nX * c->nY * c->zblocks;
}

size_t lbm::storage_size(int storage) {
    switch (storage) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        default: return 2;
    }
}

extern "C" lbm_ctx *lbm_create(int lattice, int nx, int ny, int nz, double tau, const lbm_bc *bc) {
    if (validate_domain(lattice, nx, ny, nz, tau, bc) != LBM_OK) return nullptr;
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) {
        fail(LBM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    {
        // launch-shape knobs (measurement sweeps); defaults are the tuned ones
        const char *nt = std::getenv("LBM_NT");
        if (nt && nt[0] >= '0' && nt[0] <= '4') c->nt = nt[0] - '0';
        const char *xr = std::getenv("LBM_XCD_REMAP");
        if (xr && (xr[0] == '0' || xr[0] == '1')) c->xcd_remap = xr[0] - '0';
        const char *pr = std::getenv("LBM_PAIR");
        if (pr && pr[0] >= '0' && pr[0] <= '2') c->pair = pr[0] - '0';
        const char *zr = std::getenv("LBM_ZROT");
        if (zr && (zr[0] == '0' || zr[0] == '1')) c->zrot = zr[0] - '0';
        const char *wo = std::getenv("LBM_WALLS_ONLY");
        if (wo && (wo[0] == '0' || wo[0] == '1')) c->walls_only = wo[0] - '0';
        const char *fl = std::getenv("LBM_FLAT");
        if (fl && (fl[0] == '0' || fl[0] == '1')) c->flat_req = fl[0] - '0';
        const char *sp = std::getenv("LBM_SPLIT");
        if (sp && (sp[0] == '0' || sp[0] == '1')) c->split_req = sp[0] - '0';
        const char *bl = std::getenv("LBM_BLOCK");
        if (bl) {
            const int v = std::atoi(bl);
            if (v == 64 || v == 128 || v == 192 || v == 256) c->block_req = v;
        }
    }
    setup_shape(c, lattice, nx, ny, nz, tau);
    map_faces(c, bc);
    if (bc) c->bc = *bc;
    c->opt.storage = LBM_F32;
    c->opt.compute = LBM_F32;
    c->opt.pattern = LBM_INPLACE;
    c->opt.rho0 = 1.0;
    c->ndomains = 1;
    refresh_params(c);
    g_err.clear();
    return c;
}

extern "C" int lbm_set_options(lbm_ctx *c, const lbm_options *o) {
    if (!c || !o) return fail(LBM_EINVAL, "null argument");
    if (c->A) return fail(LBM_ESTATE, "options must be set before the state exists (first lbm_init_equilibrium)");
    if (o->storage < LBM_F64 || o->storage > LBM_BF16) return fail(LBM_EINVAL, "unknown storage type %d", o->storage);
    if (o->compute != LBM_F64 && o->compute != LBM_F32) return fail(LBM_EINVAL, "unknown compute type %d", o->compute);
    if ((o->storage == LBM_F64) != (o->compute == LBM_F64))
        return fail(LBM_EUNSUPPORTED, "F64 compute goes with F64 storage only; F32/F16/BF16 storage computes in F32");
    if (o->pattern != LBM_INPLACE && o->pattern != LBM_DOUBLE && o->pattern != LBM_PULL)
        return fail(LBM_EINVAL, "unknown pattern %d", o->pattern);
    if (!(o->rho0 > 0.0) || !std::isfinite(o->rho0)) return fail(LBM_EINVAL, "rho0 must be > 0");
    if (c->batch && o->pattern != LBM_INPLACE) return fail(LBM_EUNSUPPORTED, "batch contexts use the in-place pattern");
    // a force field set earlier is typed by the compute type
    if (c->force_field && o->compute != c->opt.compute)
        return fail(LBM_ESTATE, "the compute type cannot change while a force field is set (lbm_set_force)");
    // the curved-link tables hold the wall fractions in the compute type
    if (c->nlinks && o->compute != c->opt.compute)
        return fail(LBM_ESTATE, "the compute type cannot change while curved links are set (lbm_set_curved_links)");
    c->opt = *o;
    if (!c->batch) setup_mapping(c);   // the storage type decides the split-pair layout
    refresh_params(c);
    return LBM_OK;
}

extern "C" int lbm_set_params(lbm_ctx *c, double tau, const lbm_bc *bc) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "batch contexts take per-domain parameters at creation");
    const int nz_arg = (c->lattice == LBM_D2Q9) ? 1 : c->nz;
    if (validate_domain(c->lattice, c->nx, c->ny, nz_arg, tau, bc) != LBM_OK) return LBM_EINVAL;
    if (bc) {
        const int nf = (c->D == 3) ? 6 : 4;
        for (int f = 0; f < nf; ++f)
            if (bc->face[f].type != c->bc.face[f].type && !(c->bc.face[f].type == 0 && bc->face[f].type == 0))
                return fail(LBM_EINVAL, "face %d: the boundary type cannot change (%d -> %d)", f, c->bc.face[f].type,
                            bc->face[f].type);
    }
    c->tau = tau;
    if (bc) {
        c->bc = *bc;
        map_faces(c, bc);
    }
    drop_graph(c);
    tape_invalidate(c);
    if (c->A) {
        int rc = upload_faces(c);
        if (rc) return rc;
    }
    refresh_params(c);
    return LBM_OK;
}

extern "C" int lbm_set_stream(lbm_ctx *c, void *s) {
    if (!c) return fail(LBM_EINVAL, "null context");
    c->stream = static_cast<hipStream_t>(s);
    drop_graph(c);
    return LBM_OK;
}

static int ensure_device(lbm_ctx *c) {
    if (c->device < 0) {
        int d = 0;
        hipError_t e = hipGetDevice(&d);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        c->device = d;
    }
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return LBM_OK;
}

int lbm::dev_alloc(void **p, size_t bytes, const char *what) {
    *p = nullptr;
    if (bytes == 0) return LBM_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "hipMalloc(%zu bytes) for %s: %s", bytes, what,
                    hipGetErrorString(e));
    }
    return LBM_OK;
}

void lbm::dev_free(void *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

static int ensure_state(lbm_ctx *c) {
    int rc = ensure_device(c);
    if (rc) return rc;
    if (c->A) return LBM_OK;
    const size_t bytes = (size_t)c->Q * (size_t)c->plane * storage_size(c->opt.storage);
    rc = dev_alloc(&c->A, bytes, "population state");
    if (rc) return rc;
    if (c->opt.pattern != LBM_INPLACE) {
        rc = dev_alloc(&c->B, bytes, "second population buffer");
        if (rc) {
            dev_free(c->A);
            return rc;
        }
    }
    const size_t prow = (size_t)(c->batch ? c->bgrid : c->grid);
    rc = dev_alloc((void **)&c->partial, prow * 5 * sizeof(double), "reduction scratch");
    if (!rc) rc = dev_alloc((void **)&c->sums_dev, (size_t)c->ndomains * 5 * sizeof(double), "sums");
    if (!rc) rc = dev_alloc((void **)&c->rbeg, (size_t)c->ndomains * sizeof(int64_t), "reduction rows");
    if (!rc) rc = dev_alloc((void **)&c->rend, (size_t)c->ndomains * sizeof(int64_t), "reduction rows");
    if (!rc) rc = upload_faces(c);
    if (rc) {
        free_all(c);
        return rc;
    }
    std::vector<int64_t> b(c->ndomains), e(c->ndomains);
    if (!c->batch) {
        b[0] = 0;
        e[0] = c->grid;
    } else {
        for (int d = 0; d < c->ndomains; ++d) {
            b[d] = c->dom[d].block0;
            e[d] = c->dom[d].block0 + c->dom[d].nblocks;
        }
    }
    hipError_t he = hipMemcpy(c->rbeg, b.data(), b.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(c->rend, e.data(), e.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        free_all(c);
        return hip_fail(he, "hipMemcpy");
    }
    if (c->batch) {
        rc = batch_upload(c);
        if (rc) {
            free_all(c);
            return rc;
        }
    }
    refresh_params(c);
    return LBM_OK;
}

void lbm::free_all(lbm_ctx *c) {
    drop_graph(c);
    tape_release(c);
    dev_free(c->A);
    dev_free(c->B);
    dev_free((void *&)c->partial);
    dev_free((void *&)c->sums_dev);
    dev_free((void *&)c->rbeg);
    dev_free((void *&)c->rend);
    dev_free((void *&)c->flags);
    dev_free((void *&)c->nbm);
    dev_free((void *&)c->s);
    dev_free((void *&)c->ftd);
    dev_free((void *&)c->ftf);
    dev_free((void *&)c->frows);
    dev_free(c->links);
    c->nlinks = 0;
    c->ltd = LinkTab<double>{};
    c->ltf = LinkTab<float>{};
    batch_release(c);
}

extern "C" void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
    }
    free_all(c);
    delete c;
}

Launch lbm::make_launch(lbm_ctx *c) {
    Launch g;
    g.lattice = c->lattice;
    g.storage = c->opt.storage;
    g.params = (c->opt.storage == LBM_F64) ? (const void *)&c->pd : (const void *)&c->pf;
    g.A = c->A;
    g.B = c->B;
    g.grid = (unsigned)c->grid;
    g.block = (unsigned)c->block;
    g.stream = c->stream;
    // memory hints (measured): non-temporal where wavefront-aligned for 4- and
    // 8-byte storage; plain for 2-byte storage, whose one-cell-per-lane odd step
    // runs 2-3% faster without them
    g.nt = c->nt >= 0 ? c->nt : ((c->opt.storage == LBM_F16 || c->opt.storage == LBM_BF16) ? 0 : 1);
    // push steps (the double-buffer pattern and the adjoint tape's recompute)
    // store every direction to a shifted address in a second buffer; there,
    // plain accesses measured faster on D3Q19 and D2Q9 FP32 (256^3 cavity
    // 489 -> 477 us, 8192^2 966 -> 865 us, the latter off the walls-only
    // variant, which takes the default hints only); D3Q27 keeps the default
    // (773 vs 807 us)
    g.nt_push = (c->nt < 0 && c->opt.storage == LBM_F32 && c->lattice != LBM_D3Q27) ? 0 : g.nt;
    g.pair = 0;
    g.pgrid = g.pblock = 0;
    g.force = c->force_on ? 1 : 0;
    g.kbc = c->collision == LBM_KBC ? 1 : 0;
    g.walls_only = c->walls_only;
    if (g.force || g.kbc) return g;   // these run on the one-cell-per-lane kernel
    if (c->split) {
        // split pairs: one lane per pair of cells
        g.pair = c->pair;
        g.pblock = 256;
        g.pgrid = (unsigned)((c->N / 2 + 255) / 256);
        return g;
    }
    // two cells per lane for 2-byte storage: rows of nZ % 128 == 0 cells, no
    // lane rotation or XCD remap (the pair kernel's row mapping is fixed)
    if ((c->opt.storage == LBM_F16 || c->opt.storage == LBM_BF16) && c->pair && !c->batch && c->nZ % 128 == 0 &&
        c->zrot == 0 && c->xcd_remap == 0) {
        const int pairs = c->nZ / 2;
        int blk = 256;
        while (pairs % blk) blk -= 64;
        g.pair = c->pair;
        g.pblock = (unsigned)blk;
        g.pgrid = (unsigned)((int64_t)c->nX * c->nY * (pairs / blk));
    }
    return g;
}

extern "C" int lbm_set_solid(lbm_ctx *c, const uint8_t *flags, int on_device) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (on_device != 0 && on_device != 1) return fail(LBM_EINVAL, "on_device must be 0 or 1");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "solid cells are not supported on batch contexts");
    int rc = ensure_device(c);
    if (rc) return rc;
    drop_graph(c);
    tape_invalidate(c);
    // the curved links refer to the old mask
    dev_free(c->links);
    c->nlinks = 0;
    c->ltd = LinkTab<double>{};
    c->ltf = LinkTab<float>{};
    dev_free((void *&)c->frows);
    if (!flags) {
        dev_free((void *&)c->flags);
        dev_free((void *&)c->nbm);
        c->solid_host.clear();
        refresh_params(c);
        return LBM_OK;
    }
    const size_t N = (size_t)c->N;
    try {
        c->solid_host.assign(N, 0);
    } catch (...) {
        return fail(LBM_ENOMEM, "host copy of the solid mask");
    }
    if (!c->flags) {
        rc = dev_alloc((void **)&c->flags, N, "solid flags");
        if (!rc) rc = dev_alloc((void **)&c->nbm, N * sizeof(uint32_t), "solid neighbour masks");
        if (rc) {
            dev_free((void *&)c->flags);
            dev_free((void *&)c->nbm);
            return rc;
        }
    }
    void *tmp = nullptr;
    rc = dev_alloc(&tmp, N, "solid input");
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(tmp, flags, N, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        refresh_params(c);
        Launch g = make_launch(c);
        g.params = &c->pf;
        e = launch_solid(c->lattice, g, static_cast<const uint8_t *>(tmp), c->flags, c->nbm);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(c->solid_host.data(), tmp, N, hipMemcpyDeviceToHost);
    dev_free(tmp);
    if (e != hipSuccess) {
        c->solid_host.clear();
        return hip_fail(e, "lbm_set_solid");
    }
    for (size_t k = 0; k < N; ++k) c->solid_host[k] = c->solid_host[k] ? 1 : 0;
    refresh_params(c);
    return LBM_OK;
}

// One lattice neighbour y = x + d (internal axes) of cell x: false when it lies
// across a face that is not periodic; periodic faces wrap.
static bool neighbour_cell(const lbm_ctx *c, int64_t cell, const int d[3], int64_t *out) {
    int x[3];
    x[2] = (int)(cell % c->nZ);
    x[1] = (int)((cell / c->nZ) % c->nY);
    x[0] = (int)(cell / ((int64_t)c->nZ * c->nY));
    const int n[3] = {c->nX, c->nY, c->nZ};
    for (int a = 0; a < 3; ++a) {
        x[a] += d[a];
        if (x[a] < 0 || x[a] >= n[a]) {
            const int f = 2 * a + (x[a] < 0 ? 0 : 1);
            if (c->iface[f].type != LBM_PERIODIC) return false;
            x[a] = (x[a] + n[a]) % n[a];
        }
    }
    *out = ((int64_t)x[0] * c->nY + x[1]) * c->nZ + x[2];
    return true;
}

template <class L>
static void lattice_vec(int i, int d[3]) {
    for (int a = 0; a < 3; ++a) d[a] = L::c[i][a];
}

template <class CT>
static LinkTab<CT> link_views(void *base, int64_t n) {
    LinkTab<CT> t{};
    char *p = static_cast<char *>(base);
    t.q = reinterpret_cast<const CT *>(p);
    p += (size_t)n * sizeof(CT);
    t.dlt = reinterpret_cast<CT *>(p);
    p += (size_t)n * sizeof(CT);
    t.cell = reinterpret_cast<const int32_t *>(p);
    p += (size_t)n * 4;
    t.cff = reinterpret_cast<const int32_t *>(p);
    p += (size_t)n * 4;
    t.cfff = reinterpret_cast<const int32_t *>(p);
    p += (size_t)n * 4;
    t.dir = reinterpret_cast<const uint8_t *>(p);
    p += (size_t)n;
    t.kind = reinterpret_cast<const uint8_t *>(p);
    t.n = n;
    return t;
}

extern "C" int lbm_set_curved_links(lbm_ctx *c, int64_t n, const int64_t *cell, const int32_t *dir, const double *q,
                                    int order) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "curved links are not supported on batch contexts");
    if (order != 1 && order != 2) return fail(LBM_EINVAL, "order must be 1 (linear) or 2 (quadratic)");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    if (n > 0 && (!cell || !dir || !q)) return fail(LBM_EINVAL, "null link array");
    if (n > 0 && c->solid_host.empty()) return fail(LBM_EINVAL, "curved links need solid cells (lbm_set_solid)");
    if (n >= ((int64_t)1 << 31)) return fail(LBM_EINVAL, "too many links");
    // validate everything before any change
    struct Link { int64_t cell, ff, fff; double q; int dir, kind; };
    std::vector<Link> keep;
    std::vector<int64_t> keys;
    try {
        keep.reserve((size_t)n);
        keys.reserve((size_t)n);
    } catch (...) {
        return fail(LBM_ENOMEM, "host link tables");
    }
    const int Q = c->Q;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t x = cell[k];
        const int i = dir[k];
        if (x < 0 || x >= c->N) return fail(LBM_EINVAL, "link %lld: cell %lld out of range", (long long)k, (long long)x);
        if (i < 1 || i >= Q) return fail(LBM_EINVAL, "link %lld: direction %d out of range", (long long)k, i);
        if (!(q[k] > 0.0 && q[k] <= 1.0)) return fail(LBM_EINVAL, "link %lld: q = %g outside (0, 1]", (long long)k, q[k]);
        if (c->solid_host[(size_t)x]) return fail(LBM_EINVAL, "link %lld: cell %lld is solid", (long long)k, (long long)x);
        int d[3];
        if (c->lattice == LBM_D2Q9) lattice_vec<D2Q9>(i, d);
        else if (c->lattice == LBM_D3Q19) lattice_vec<D3Q19>(i, d);
        else lattice_vec<D3Q27>(i, d);
        int64_t y;
        if (!neighbour_cell(c, x, d, &y) || !c->solid_host[(size_t)y])
            return fail(LBM_EINVAL, "link %lld: the neighbour of cell %lld along direction %d is not a solid cell",
                        (long long)k, (long long)x, i);
        keys.push_back(x * Q + i);
        const int md[3] = {-d[0], -d[1], -d[2]};
        int64_t ff, fff;
        // x - c_i must be a fluid cell, else the link keeps halfway bounce-back
        if (!neighbour_cell(c, x, md, &ff) || c->solid_host[(size_t)ff]) continue;
        int kind = (q[k] >= 0.5) ? 1 : 0;
        if (order == 2 && neighbour_cell(c, ff, md, &fff) && !c->solid_host[(size_t)fff]) kind |= 2;
        else fff = ff;
        if (ff == x || fff == x)
            return fail(LBM_EUNSUPPORTED, "link %lld: its interpolation cells wrap onto its own cell", (long long)k);
        keep.push_back(Link{x, ff, fff, q[k], i, kind});
    }
    std::vector<int64_t> sorted(keys);
    std::sort(sorted.begin(), sorted.end());
    for (size_t k = 1; k < sorted.size(); ++k)
        if (sorted[k] == sorted[k - 1])
            return fail(LBM_EINVAL, "link (cell %lld, direction %d) given twice", (long long)(sorted[k] / Q),
                        (int)(sorted[k] % Q));
    int rc = ensure_device(c);
    if (rc) return rc;
    drop_graph(c);
    tape_invalidate(c);
    dev_free(c->links);
    dev_free((void *&)c->frows);
    c->nlinks = 0;
    c->ltd = LinkTab<double>{};
    c->ltf = LinkTab<float>{};
    c->link_order = order;
    const int64_t m = (int64_t)keep.size();
    if (m == 0) return LBM_OK;
    const size_t cs = (c->opt.storage == LBM_F64) ? 8 : 4;
    const size_t bytes = (size_t)m * (2 * cs + 12 + 2);
    std::vector<char> host(bytes);
    char *p = host.data();
    for (int64_t k = 0; k < m; ++k) {
        if (cs == 8) reinterpret_cast<double *>(p)[k] = keep[k].q;
        else reinterpret_cast<float *>(p)[k] = (float)keep[k].q;
    }
    std::memset(p + (size_t)m * cs, 0, (size_t)m * cs);
    int32_t *ic = reinterpret_cast<int32_t *>(p + 2 * (size_t)m * cs);
    for (int64_t k = 0; k < m; ++k) {
        ic[k] = (int32_t)keep[k].cell;
        ic[m + k] = (int32_t)keep[k].ff;
        ic[2 * m + k] = (int32_t)keep[k].fff;
    }
    uint8_t *b8 = reinterpret_cast<uint8_t *>(ic + 3 * m);
    for (int64_t k = 0; k < m; ++k) {
        b8[k] = (uint8_t)keep[k].dir;
        b8[m + k] = (uint8_t)keep[k].kind;
    }
    rc = dev_alloc(&c->links, bytes, "curved links");
    if (rc) return rc;
    hipError_t e = hipMemcpy(c->links, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(c->links);
        return hip_fail(e, "curved link upload");
    }
    c->nlinks = m;
    c->ltd = link_views<double>(c->links, m);
    c->ltf = link_views<float>(c->links, m);
    return LBM_OK;
}

extern "C" int lbm_set_solid_fraction(lbm_ctx *c, const float *s, int on_device) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "partial bounce-back is not supported on batch contexts");
    if (on_device != 0 && on_device != 1) return fail(LBM_EINVAL, "on_device must be 0 or 1");
    if (s && c->collision == LBM_KBC)
        return fail(LBM_EUNSUPPORTED, "KBC does not combine with a partial bounce-back field");
    int rc = ensure_device(c);
    if (rc) return rc;
    drop_graph(c);
    tape_invalidate(c);
    if (!s) {
        dev_free((void *&)c->s);
        refresh_params(c);
        return LBM_OK;
    }
    const size_t N = (size_t)c->N;
    if (!c->s) {
        rc = dev_alloc((void **)&c->s, N * sizeof(float), "solid fraction");
        if (rc) return rc;
    }
    hipError_t e = hipMemcpyAsync(c->s, s, N * sizeof(float), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_solid_fraction");
    refresh_params(c);
    return LBM_OK;
}

extern "C" int lbm_init_equilibrium(lbm_ctx *c, const void *rho, const void *u, int dtype) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if ((rho || u) && dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
    int rc = ensure_state(c);
    if (rc) return rc;
    drop_graph(c);
    tape_release(c);
    c->t = 0;
    c->moved_since_tape = true;
    refresh_params(c);
    hipError_t e;
    if (c->batch) e = batch_init(c, rho, u, dtype == LBM_F64);
    else e = launch_init(make_launch(c), rho, u, dtype == LBM_F64, c->N);
    if (e != hipSuccess) return hip_fail(e, "lbm_init_equilibrium");
    return LBM_OK;
}

// One forward step of the whole context (no tape bookkeeping).
hipError_t lbm::forward_step(lbm_ctx *c) {
    if (c->batch) {
        hipError_t e = batch_step(c);
        c->t += 1;
        return e;
    }
    c->pd.zh_pending = c->pf.zh_pending = c->t > 0 ? 1 : 0;
    Launch g = make_launch(c);
    const int mode = step_mode(c);
    hipError_t e = launch_step(g, mode, c->s != nullptr);
    if (mode >= 2) std::swap(c->A, c->B);
    if (e == hipSuccess && c->nlinks) {
        // interpolated bounce-back on the curved links, on the state just written
        Launch b = make_launch(c);
        const void *lt = (c->opt.storage == LBM_F64) ? (const void *)&c->ltd : (const void *)&c->ltf;
        e = launch_bouzidi(b, lt, mode == 1 || mode == 2);
    }
    c->t += 1;
    return e;
}

extern "C" int lbm_step(lbm_ctx *c, int n) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised (call lbm_init_equilibrium)");
    int rc = ensure_device(c);
    if (rc) return rc;
    if (c->batch && n > 0) {
        rc = batch_autotune(c);
        if (rc) return rc;
        if (!c->tape_recording && batch_uses_persistent(c)) {
            hipError_t e = batch_persistent_steps(c, n);
            if (e != hipSuccess) return hip_fail(e, "lbm_step (persistent batch)");
            c->t += n;
            c->moved_since_tape = true;
            return LBM_OK;
        }
    }
    for (int k = 0; k < n; ++k) {
        hipError_t e = forward_step(c);
        if (e != hipSuccess) return hip_fail(e, "lbm_step");
        rc = tape_after_step(c);
        if (rc) return rc;
    }
    if (n > 0 && !c->tape_recording) c->moved_since_tape = true;
    return LBM_OK;
}

extern "C" int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

extern "C" int lbm_moments(lbm_ctx *c, void *rho, void *u, int dtype, double *sums_host) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if ((rho || u) && dtype != LBM_F64 && dtype != LBM_F32) return fail(LBM_EINVAL, "dtype must be LBM_F64 or LBM_F32");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised (call lbm_init_equilibrium)");
    int rc = ensure_device(c);
    if (rc) return rc;
    refresh_params(c);
    hipError_t e;
    const bool odd = swapped_at(c, c->t);
    if (c->batch) e = batch_moments(c, odd, rho, u, dtype == LBM_F64, c->partial);
    else e = launch_moments(make_launch(c), odd, rho, u, dtype == LBM_F64, c->partial, c->N);
    if (e == hipSuccess) e = launch_reduce(c->partial, c->rbeg, c->rend, c->sums_dev, c->ndomains, c->stream);
    if (e == hipSuccess && sums_host) {
        std::vector<double> tmp((size_t)c->ndomains * 5);
        e = hipMemcpyAsync(tmp.data(), c->sums_dev, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) {
            // internal axes -> caller axes
            for (int d = 0; d < c->ndomains; ++d) {
                double *o = sums_host + 5 * d;
                const double *m = tmp.data() + 5 * d;
                o[0] = m[0];
                if (c->D == 3) {
                    o[1] = m[1];
                    o[2] = m[2];
                    o[3] = m[3];
                } else {
                    o[1] = m[2];
                    o[2] = m[3];
                    o[3] = 0.0;
                }
                o[4] = m[4];
            }
        }
    }
    if (e != hipSuccess) return hip_fail(e, "lbm_moments");
    return LBM_OK;
}

extern "C" int lbm_forces(lbm_ctx *c, double *out) {
    if (!c || !out) return fail(LBM_EINVAL, "null argument");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "lbm_forces takes a single-domain context");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised (call lbm_init_equilibrium)");
    if (c->t < 1) return fail(LBM_ESTATE, "no step taken since the last init / load");
    int rc = ensure_device(c);
    if (rc) return rc;
    constexpr int kSlots = 21;
    // rows: one per step-kernel workgroup, one per 256 curved links, then the total
    const int64_t lrows = (c->nlinks + 255) / 256;
    const int64_t rows = c->grid + lrows;
    if (!c->frows) {
        rc = dev_alloc((void **)&c->frows, ((size_t)rows + 1) * kSlots * sizeof(double), "force sums");
        if (rc) return rc;
    }
    refresh_params(c);
    double *sum_dev = c->frows + (size_t)rows * kSlots;
    hipError_t e = launch_forces(make_launch(c), c->frows);
    if (e == hipSuccess && c->nlinks) {
        const void *lt = (c->opt.storage == LBM_F64) ? (const void *)&c->ltd : (const void *)&c->ltf;
        e = launch_link_forces(make_launch(c), lt, c->frows + (size_t)c->grid * kSlots);
    }
    if (e == hipSuccess) e = launch_rows_reduce(c->frows, rows, kSlots, sum_dev, c->stream);
    double m[kSlots];
    if (e == hipSuccess) e = hipMemcpyAsync(m, sum_dev, sizeof m, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_forces");
    // internal faces / axes -> caller faces / axes
    for (int k = 0; k < kSlots; ++k) out[k] = 0.0;
    if (c->D == 3) {
        for (int k = 0; k < kSlots; ++k) out[k] = m[k];
    } else {
        out[0] = m[1];
        out[1] = m[2];
        for (int f = 2; f < 6; ++f)
            for (int a = 1; a < 3; ++a) out[3 + 3 * (f - 2) + (a - 1)] = m[3 + 3 * f + a];
    }
    return LBM_OK;
}

extern "C" int lbm_set_collision(lbm_ctx *c, int model) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (model != LBM_BGK && model != LBM_KBC) return fail(LBM_EINVAL, "unknown collision model %d", model);
    if (model == LBM_KBC) {
        if (c->lattice == LBM_D3Q19) return fail(LBM_EUNSUPPORTED, "KBC is defined here for D2Q9 and D3Q27");
        if (c->batch) return fail(LBM_EUNSUPPORTED, "KBC is not supported on batch contexts");
        if (c->s) return fail(LBM_EUNSUPPORTED, "KBC does not combine with a partial bounce-back field");
    }
    drop_graph(c);
    tape_invalidate(c);
    c->collision = model;
    return LBM_OK;
}

extern "C" int lbm_set_force(lbm_ctx *c, const double *force, const void *field, double eps) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->batch) return fail(LBM_EUNSUPPORTED, "body forces are not supported on batch contexts");
    if (!std::isfinite(eps)) return fail(LBM_EINVAL, "eps must be finite");
    double u[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < c->D; ++a) {
        if (force) {
            if (!std::isfinite(force[a])) return fail(LBM_EINVAL, "force must be finite");
            u[a] = eps * force[a];
        }
    }
    drop_graph(c);
    tape_invalidate(c);
    c->force_on = (field != nullptr && eps != 0.0) || u[0] != 0.0 || u[1] != 0.0 || u[2] != 0.0;
    for (int a = 0; a < 3; ++a) c->force_u[a] = u[a];
    c->force_field = c->force_on ? field : nullptr;
    c->force_eps = eps;
    refresh_params(c);
    return LBM_OK;
}

extern "C" int lbm_sync(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    if (c->device < 0) return LBM_OK;
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_sync");
    return LBM_OK;
}

// ---- checkpoint / resume ----------------------------------------------------
struct StateHeader {
    char magic[8];
    int32_t lattice, storage, pattern, Q;
    int64_t N, plane, t;
};

extern "C" size_t lbm_state_bytes(const lbm_ctx *c) {
    if (!c) return 0;
    return sizeof(StateHeader) + (size_t)c->Q * (size_t)c->plane * storage_size(c->opt.storage);
}

extern "C" int lbm_save(lbm_ctx *c, void *host, size_t bytes) {
    if (!c || !host) return fail(LBM_EINVAL, "null argument");
    if (!c->A) return fail(LBM_ESTATE, "state not initialised");
    if (bytes < lbm_state_bytes(c)) return fail(LBM_EINVAL, "buffer too small: need %zu bytes", lbm_state_bytes(c));
    int rc = ensure_device(c);
    if (rc) return rc;
    StateHeader h;
    std::memcpy(h.magic, "LBMSTAT1", 8);
    h.lattice = c->lattice;
    h.storage = c->opt.storage;
    h.pattern = c->opt.pattern | (c->split ? 0x100 : 0);   // the split-pair layout is part of the image
    h.Q = c->Q;
    h.N = c->N;
    h.plane = c->plane;
    h.t = c->t;
    std::memcpy(host, &h, sizeof h);
    const size_t sb = lbm_state_bytes(c) - sizeof h;
    hipError_t e = hipMemcpyAsync(static_cast<char *>(host) + sizeof h, c->A, sb, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_save");
    return LBM_OK;
}

extern "C" int lbm_load(lbm_ctx *c, const void *host, size_t bytes) {
    if (!c || !host) return fail(LBM_EINVAL, "null argument");
    if (bytes < sizeof(StateHeader)) return fail(LBM_EINVAL, "buffer too small");
    StateHeader h;
    std::memcpy(&h, host, sizeof h);
    if (std::memcmp(h.magic, "LBMSTAT1", 8) != 0) return fail(LBM_EINVAL, "not a state image");
    if (h.lattice != c->lattice || h.storage != c->opt.storage || h.pattern != (c->opt.pattern | (c->split ? 0x100 : 0)) ||
        h.N != c->N ||
        h.plane != c->plane || h.Q != c->Q)
        return fail(LBM_EINVAL, "state image does not match this context (lattice/storage/pattern/shape)");
    if (bytes < lbm_state_bytes(c)) return fail(LBM_EINVAL, "buffer too small: need %zu bytes", lbm_state_bytes(c));
    int rc = ensure_state(c);
    if (rc) return rc;
    drop_graph(c);
    tape_release(c);
    const size_t sb = lbm_state_bytes(c) - sizeof h;
    hipError_t e = hipMemcpyAsync(c->A, static_cast<const char *>(host) + sizeof h, sb, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_load");
    c->t = h.t;
    c->moved_since_tape = true;
    refresh_params(c);
    return LBM_OK;
}

extern "C" int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return fail(LBM_EINVAL, "null pointer");
    if ((bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return fail(LBM_EINVAL, "pointers and size must be 16-byte aligned");
    hipError_t e = launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "lbm_copy_probe");
    return LBM_OK;
}
