// core.hpp -- per-cell device arithmetic and the kernel parameter block.
//
// State format.  Populations are stored as deviations from the rest state,
// h_i = f_i - w_i rho0, one plane per direction (structure of arrays, Z
// contiguous).  FP16/BF16 storage keeps h_i / w_i (rounded to nearest even)
// and the kernels widen to FP32.  This is the renormalisation around zero
// that the paper says single precision needs (Sec. 4.1).
//
// Step semantics (paper Sec. 3.6: collide, post-collision BC, stream,
// post-stream BC).  One kernel pass per time step does, per fluid cell:
//   read   : the Q populations f(x, t) (post-stream, post-boundary);
//   close  : on a Zou-He face cell, the unknown populations from the known
//            ones (the post-stream BC of the previous step, applied where the
//            knowns are first all in registers);
//   collide: moments (eqs. density, velocity), equilibrium (eq. feq), BGK
//            relaxation (eq. LBM-BGK), optional partial bounce-back mix;
//   write  : each post-collision value to the cell it streams to
//            (eq. streaming), or, where that cell is not fluid, the boundary
//            value of the population that comes back to this cell instead:
//            halfway bounce-back (+ moving-wall term), or the equilibrium of an
//            outflow / perimeter face.  These are exactly the values the next
//            step would have to fill, computed where they are known.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <utility>

#include "lattice.hpp"

namespace lbm {

enum : uint8_t { F_PERIODIC = 0, F_WALL = 1, F_ZH_VEL = 2, F_ZH_PRES = 3, F_OUT = 4, F_REG_VEL = 5, F_REG_PRES = 6 };

constexpr int kMaxBlock = 256;

// Per-face data read with a runtime face index (boundary lanes only).  Kept in
// device memory: indexing the by-value kernel argument block with a runtime
// index would force a private copy of the whole block.
template <class CT>
struct FaceTab {
    CT uw[6][3];
    CT rho[6];
    int type[6];
    int pad[2];
};

// Curved-wall links (interpolated bounce-back), structure of arrays on the
// device.  Link k: fluid cell cell[k], direction dir[k] (cell + c_dir solid),
// wall fraction q[k]; cff[k] = cell - c_dir and cfff[k] = cell - 2 c_dir
// (periodic wrap applied; cfff only for quadratic links); kind[k] bit 0:
// q >= 1/2, bit 1: quadratic weights.  dlt[k] receives, each step,
// f*_dir(cell, t) - f_-dir(cell, t + 1) in deviation units (the part of the
// link's momentum exchange that halfway bounce-back would not have).
template <class CT>
struct LinkTab {
    const CT *q;
    CT *dlt;
    const int32_t *cell, *cff, *cfff;
    const uint8_t *dir, *kind;
    int64_t n;
};

template <class CT>
struct Params {
    int nX, nY, nZ;        // internal extents (Z contiguous)
    int sX, sY;            // cell strides of X and Y (Z stride 1)
    int zblocks;           // blocks per Z row
    int64_t plane;         // cells of the state rounded up to whole tiles (values per direction)
    uint32_t wallmask;     // faces of type wall
    uint32_t staticmask;   // wall faces with zero velocity
    uint32_t zhmask;       // Zou-He faces
    uint32_t permask;      // periodic faces
    uint8_t ftype[8];
    CT uw[6][3];           // wall / inlet velocity per face (internal axes)
    CT frho[6];            // face density (pressure / outflow)
    CT omega;              // 1 / tau
    CT rho0;
    int zh_pending;        // the state read needs the Zou-He closure (t > 0)
    int xcd_remap;         // give each XCD a contiguous range of rows
    int zrot;              // lane rotation within a Z row (block_cell)
    int flat;              // lanes cover consecutive cells of the whole grid (rows not a multiple of 64 cells)
    int spk;               // 2-byte storage in split pairs (the two X-halves share a 32-bit word)
    int64_t nh;            // cells of the low X-half (split pairs)
    const uint8_t *flags;  // N bytes or null: bit0 solid, bit1 a neighbour is solid
    const uint32_t *nbm;   // N words: bit k set when x - c_k is a solid cell
    const float *s;        // N or null: partial bounce-back solid fraction
    const FaceTab<CT> *ft; // device copy of the face data
    const CT *fld[3];      // body-force field per internal axis (N values, cell order) or null
    CT fu[3];              // uniform body force per internal axis, scale applied
    CT feps;               // scale of the field
};

// ---- storage formats -------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

template <class ST>
struct Store;

// ld / st: plain accesses; ldn / stn: non-temporal (streaming) accesses, for
// state that is touched once per step and not reused before it leaves the caches
template <>
struct Store<double> {
    using CT = double;
    static constexpr bool scaled = false;
    __device__ static double ld(const double *p) { return *p; }
    __device__ static void st(double *p, double v) { *p = v; }
    __device__ static double ldn(const double *p) { return __builtin_nontemporal_load(p); }
    __device__ static void stn(double *p, double v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<float> {
    using CT = float;
    static constexpr bool scaled = false;
    __device__ static float ld(const float *p) { return *p; }
    __device__ static void st(float *p, float v) { *p = v; }
    __device__ static float ldn(const float *p) { return __builtin_nontemporal_load(p); }
    __device__ static void stn(float *p, float v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<_Float16> {
    using CT = float;
    static constexpr bool scaled = true;
    __device__ static float ld(const _Float16 *p) { return (float)*p; }
    __device__ static void st(_Float16 *p, float v) { *p = (_Float16)v; }  // round to nearest even
    __device__ static float ldn(const _Float16 *p) { return (float)__builtin_nontemporal_load(p); }
    __device__ static void stn(_Float16 *p, float v) { __builtin_nontemporal_store((_Float16)v, p); }
};
template <>
struct Store<bf16_t> {
    using CT = float;
    static constexpr bool scaled = true;
    // round to nearest even: gfx950's conversion instruction (v_cvt_pk_bf16_f32)
    __device__ static uint16_t round(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    __device__ static float ld(const bf16_t *p) { return __uint_as_float(((uint32_t)p->bits) << 16); }
    __device__ static void st(bf16_t *p, float v) { p->bits = round(v); }
    __device__ static float ldn(const bf16_t *p) {
        return __uint_as_float(((uint32_t)__builtin_nontemporal_load(&p->bits)) << 16);
    }
    __device__ static void stn(bf16_t *p, float v) { __builtin_nontemporal_store(round(v), &p->bits); }
};

// Population layout: tiles of kTile = 4096 consecutive cells (flat cell
// index), each tile holding the Q sub-planes of its cells back to back --
// population i of cell c at ((c / kTile) Q + i) kTile + c % kTile.  Within a
// tile a direction is one contiguous run, so a wavefront's access to one
// direction is one aligned run as with whole planes, while the Q accesses of a
// cell fall within Q kTile values instead of Q planes a whole grid apart.
// Measured on gfx950 (D3Q19 256^3 cavity): FP32 40.1k -> 41.1k MLUPS, D3Q27
// 26.6k -> 27.8k, the D3Q27 obstacle channel 22.8k -> 23.4k, the batched
// D2Q9 cavities 80.2k -> 81.8k; FP16 68.3-68.6k against 69.6k with whole
// planes (its even step gains 9%, its one-cell-per-lane odd step loses 7%;
// 16384-cell tiles for 2-byte values measured the same).  Tiles of 64 cells
// measured no faster than planes.  A domain's state holds Q tiled_cells(N)
// values.
constexpr int kTileLog = 12;
constexpr int64_t kTile = (int64_t)1 << kTileLog;
template <int Q>
__host__ __device__ __forceinline__ int64_t pidx(int i, int64_t cell) {
    // ((c >> 12) Q + i) 4096 + (c & 4095) written as c + ((c >> 12) (Q - 1) + i) 4096:
    // the same integer, with no mask and no OR (cells < 2^31, so the bracket
    // is < 2^24 and fits 32-bit arithmetic; the sum is taken in 64 bits)
    const uint32_t c = (uint32_t)cell;
    const uint32_t t = (c >> kTileLog) * (uint32_t)(Q - 1) + (uint32_t)i;
    return (int64_t)((uint64_t)c + ((uint64_t)t << kTileLog));
}
__host__ __device__ constexpr int64_t tiled_cells(int64_t n) { return (n + kTile - 1) / kTile * kTile; }

// Split pairs (2-byte storage, nX even).  The cell (X', Y, Z) of the low
// X-half and the cell (X' + nX/2, Y, Z) of the high half share one 32-bit word
// per population: storage index 2 c' + h with c' = (X' nY + Y) nZ + Z and
// h = 1 for the high half, tiled like a cell index.  A neighbour in the same
// half lies 2 x its cell offset away in storage indices, so a two-cell step
// moves aligned 32-bit words under every lattice shift; only the planes
// X' = nX/2 - 1 and X = nX/2, whose X-neighbours sit in the other half (the
// seam), take the general path.  Other storage types: the cell index itself.
template <class ST, class CT>
__device__ __forceinline__ int64_t sidx(const Params<CT> &p, int64_t cell) {
    if constexpr (sizeof(ST) == 2) {
        if (p.spk) {
            const int64_t h = cell >= p.nh ? 1 : 0;
            return 2 * (cell - h * p.nh) + h;
        }
    }
    return cell;
}
// storage-index step of one cell-index step within a half
template <class ST, class CT>
__device__ __forceinline__ int64_t smul(const Params<CT> &p) {
    if constexpr (sizeof(ST) == 2) return p.spk ? 2 : 1;
    return 1;
}

template <class L, int I, class ST>
__device__ __forceinline__ const ST *pop_ptr(const ST *base, int64_t cell) {
    return base + pidx<L::Q>(I, cell);
}
template <class L, int I, class ST>
__device__ __forceinline__ ST *pop_ptr(ST *base, int64_t cell) {
    return base + pidx<L::Q>(I, cell);
}

// load / store of population I through a pointer, with the storage scale
template <class L, class ST, int I, bool NT = false>
__device__ __forceinline__ typename Store<ST>::CT ldp(const ST *ptr) {
    using CT = typename Store<ST>::CT;
    CT v = NT ? Store<ST>::ldn(ptr) : Store<ST>::ld(ptr);
    if constexpr (Store<ST>::scaled) v *= (CT)weight<L>(I);
    return v;
}
template <class L, class ST, int I, bool NT = false>
__device__ __forceinline__ void stp(ST *ptr, typename Store<ST>::CT v) {
    using CT = typename Store<ST>::CT;
    if constexpr (Store<ST>::scaled) v *= (CT)(1.0 / weight<L>(I));
    if constexpr (NT) Store<ST>::stn(ptr, v);
    else Store<ST>::st(ptr, v);
}

// load / store of population i with the storage scale
template <class L, class ST, int I, bool NT = false>
__device__ __forceinline__ typename Store<ST>::CT ldh(const ST *base, int64_t cell) {
    using CT = typename Store<ST>::CT;
    const ST *ptr = pop_ptr<L, I>(base, cell);
    CT v = NT ? Store<ST>::ldn(ptr) : Store<ST>::ld(ptr);
    if constexpr (Store<ST>::scaled) v *= (CT)weight<L>(I);
    return v;
}
template <class L, class ST, int I, bool NT = false>
__device__ __forceinline__ void sth(ST *base, int64_t cell, typename Store<ST>::CT v) {
    using CT = typename Store<ST>::CT;
    if constexpr (Store<ST>::scaled) v *= (CT)(1.0 / weight<L>(I));
    ST *ptr = pop_ptr<L, I>(base, cell);
    if constexpr (NT) Store<ST>::stn(ptr, v);
    else Store<ST>::st(ptr, v);
}

// compile-time loop
template <int N, class F, int... Is>
__device__ __forceinline__ void unroll_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F &&f) {
    unroll_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// ---- neighbour classification (only for cells on a face or next to a solid)
enum : int { NB_FLUID = 0, NB_WALL = 1, NB_ZH = 2, NB_OUT = 3 };

struct Nb {
    int kind;
    int face;      // moving wall face (NB_WALL, -1 = static) or open face
    int64_t cell;  // NB_FLUID: source cell (periodic wrap applied)
};

// Source y = x - c_k of population k at cell (X, Y, Z).
template <class L, class CT>
__device__ __forceinline__ Nb classify_src(const Params<CT> &p, int X, int Y, int Z, int k, uint32_t nbm) {
    int yx = X - L::c[k][0], yy = Y - L::c[k][1], yz = Z - L::c[k][2];
    uint32_t crossed = 0;
    if (yx < 0) { if (p.ftype[0] == F_PERIODIC) yx += p.nX; else crossed |= 1u; }
    else if (yx >= p.nX) { if (p.ftype[1] == F_PERIODIC) yx -= p.nX; else crossed |= 2u; }
    if (yy < 0) { if (p.ftype[2] == F_PERIODIC) yy += p.nY; else crossed |= 4u; }
    else if (yy >= p.nY) { if (p.ftype[3] == F_PERIODIC) yy -= p.nY; else crossed |= 8u; }
    if (yz < 0) { if (p.ftype[4] == F_PERIODIC) yz += p.nZ; else crossed |= 16u; }
    else if (yz >= p.nZ) { if (p.ftype[5] == F_PERIODIC) yz -= p.nZ; else crossed |= 32u; }
    Nb r;
    r.face = -1;
    r.cell = 0;
    if (!crossed) {
        r.kind = ((nbm >> k) & 1u) ? NB_WALL : NB_FLUID;
        r.cell = ((int64_t)yx * p.nY + yy) * p.nZ + yz;
        return r;
    }
    const uint32_t walls = crossed & p.wallmask;
    if (walls) {
        r.kind = NB_WALL;
        r.face = (walls & p.staticmask) ? -1 : (int)__builtin_ctz(walls);
        return r;
    }
    r.face = (int)__builtin_ctz(crossed);
    r.kind = (p.ft->type[r.face] == F_OUT) ? NB_OUT : NB_ZH;
    return r;
}

// ---- equilibrium in deviation form: feq_i - w_i rho0 -------------------------
// c_I . u with the components of c_I (0 or +-1) resolved at compile time: the
// same value, rounded the same way, as the full product sum, without the
// multiplications by zero the compiler has to keep in IEEE arithmetic.
template <class L, int I, class CT>
__device__ __forceinline__ CT cdot(CT ux, CT uy, CT uz) {
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    CT v = (cx > 0) ? ux : ((cx < 0) ? -ux : (CT)0);
    if constexpr (cx == 0) {
        if constexpr (cy != 0) v = (cy > 0) ? uy : -uy;
        if constexpr (cz != 0) v = (cy != 0) ? ((cz > 0) ? v + uz : v - uz) : ((cz > 0) ? uz : -uz);
    } else {
        if constexpr (cy != 0) v = (cy > 0) ? v + uy : v - uy;
        if constexpr (cz != 0) v = (cz > 0) ? v + uz : v - uz;
    }
    return v;
}

template <class L, int I, class CT>
__device__ __forceinline__ CT heq(CT drho, CT rho, CT ux, CT uy, CT uz, CT usq15) {
    const CT cu = (CT)3 * cdot<L, I>(ux, uy, uz);
    return (CT)weight<L>(I) * (drho + rho * (cu + (CT)0.5 * cu * cu - usq15));
}

// ---- Zou-He closure at a face cell (the generic 2-D/3-D non-equilibrium
// bounce-back; reduces to Zou & He's D2Q9 formulas, cited in Sec. 4.3) ------
// Zou-He closure (non-equilibrium bounce-back; the paper cites Zou & He for
// its inlet/outlet, Sec. 4.3) at a cell on open face `face` with inward
// normal n.  U = {c.n = 1} unknown, Z = {c.n = 0}, O = {c.n = -1} known:
//   velocity face: rho = (sum_Z f + 2 sum_O f) / (1 - u_w.n), u = u_w
//   pressure face: rho = rho_w, u = n (1 - (sum_Z f + 2 sum_O f) / rho_w)
//   f_i = f_opp(i) + 6 w_i rho c_i.u - sum_t c_it N_t               (i in U)
//   N_t = (sum_Z f_j c_jt - 2/3 rho u_t) / sum_U c_kt^2            (t tangential)
// In deviation variables the rho0 parts cancel except in rho itself
// (sum_Z w + 2 sum_O w = 1).  The face is a runtime value and every choice
// below is a value select, so the populations stay in registers.
template <class L, class CT>
__device__ __forceinline__ void regularize(CT *h, const Params<CT> &p, int face);

template <class L, class CT>
__device__ __forceinline__ void zouhe(CT *h, const Params<CT> &p, int face) {
    if (p.ft->type[face] >= F_REG_VEL) {
        regularize<L>(h, p, face);
        return;
    }
    const int ax = face >> 1;
    const int sg = (face & 1) ? -1 : 1;
    int cn[L::Q];
    unroll<L::Q>([&](auto I) {
        const int ca = (ax == 0) ? L::c[I][0] : ((ax == 1) ? L::c[I][1] : L::c[I][2]);
        cn[I] = sg * ca;
    });
    CT SZ = 0, SO = 0;
    unroll<L::Q>([&](auto I) {
        SZ += (cn[I] == 0) ? h[I] : (CT)0;
        SO += (cn[I] == -1) ? h[I] : (CT)0;
    });
    const CT known = SZ + (CT)2 * SO;  // sum_Z f + 2 sum_O f - rho0
    const FaceTab<CT> &F = *p.ft;
    CT rho, u[3];
    if (F.type[face] == F_ZH_VEL) {
        u[0] = F.uw[face][0];
        u[1] = F.uw[face][1];
        u[2] = F.uw[face][2];
        const CT un = (CT)sg * ((ax == 0) ? u[0] : ((ax == 1) ? u[1] : u[2]));
        rho = p.rho0 + (known + p.rho0 * un) / ((CT)1 - un);
    } else {
        rho = F.rho[face];
        const CT un = (rho - p.rho0 - known) / rho;
        u[0] = (ax == 0) ? (CT)sg * un : (CT)0;
        u[1] = (ax == 1) ? (CT)sg * un : (CT)0;
        u[2] = (ax == 2) ? (CT)sg * un : (CT)0;
    }
    CT Nt[3];
    unroll<3>([&](auto T) {
        CT num = 0;
        unroll<L::Q>([&](auto I) {
            if constexpr (L::c[I][T] != 0) num += (cn[I] == 0) ? (CT)L::c[I][T] * h[I] : (CT)0;
        });
        const CT v = (num - (CT)(2.0 / 3.0) * rho * u[T]) * (CT)(1.0 / L::den_t);
        Nt[T] = (ax == T) ? (CT)0 : v;
    });
    // in place: the opposite of an unknown is always a known, never rewritten
    unroll<L::Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        const CT cu = (CT)L::c[I][0] * u[0] + (CT)L::c[I][1] * u[1] + (CT)L::c[I][2] * u[2];
        CT v = h[O] + (CT)(6.0 * weight<L>(I)) * rho * cu;
        unroll<3>([&](auto T) {
            if constexpr (L::c[I][T] != 0) v -= (CT)L::c[I][T] * Nt[T];
        });
        h[I] = (cn[I] == 1) ? v : h[I];
    });
}

// Regularized velocity / pressure face (Latt et al. 2008, one of the boundary
// conditions of Sec. 3.5), applied where zouhe() would be: rho and u as for
// Zou-He; the unknown populations take the non-equilibrium part of their
// opposite; then every population becomes
//   feq_i(rho, u) + 4.5 w_i (c_i c_i - I/3) : Pi_neq,  Pi_neq = sum_i c_i c_i (f_i - feq_i).
// In deviation variables f_i - feq_i = h_i - heq_i.
template <class L, class CT>
__device__ __forceinline__ void regularize(CT *h, const Params<CT> &p, int face) {
    const int ax = face >> 1;
    const int sg = (face & 1) ? -1 : 1;
    int cn[L::Q];
    unroll<L::Q>([&](auto I) {
        const int ca = (ax == 0) ? L::c[I][0] : ((ax == 1) ? L::c[I][1] : L::c[I][2]);
        cn[I] = sg * ca;
    });
    CT SZ = 0, SO = 0;
    unroll<L::Q>([&](auto I) {
        SZ += (cn[I] == 0) ? h[I] : (CT)0;
        SO += (cn[I] == -1) ? h[I] : (CT)0;
    });
    const CT known = SZ + (CT)2 * SO;
    const FaceTab<CT> &F = *p.ft;
    CT rho, u[3];
    if (F.type[face] == F_REG_VEL) {
        u[0] = F.uw[face][0];
        u[1] = F.uw[face][1];
        u[2] = F.uw[face][2];
        const CT un = (CT)sg * ((ax == 0) ? u[0] : ((ax == 1) ? u[1] : u[2]));
        rho = p.rho0 + (known + p.rho0 * un) / ((CT)1 - un);
    } else {
        rho = F.rho[face];
        const CT un = (rho - p.rho0 - known) / rho;
        u[0] = (ax == 0) ? (CT)sg * un : (CT)0;
        u[1] = (ax == 1) ? (CT)sg * un : (CT)0;
        u[2] = (ax == 2) ? (CT)sg * un : (CT)0;
    }
    const CT drho = rho - p.rho0;
    const CT usq15 = (CT)1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    // non-equilibrium parts, in place; unknowns from their (known) opposites
    unroll<L::Q>([&](auto I) { h[I] -= heq<L, I>(drho, rho, u[0], u[1], u[2], usq15); });
    unroll<L::Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        h[I] = (cn[I] == 1) ? h[O] : h[I];
    });
    CT P00 = 0, P11 = 0, P22 = 0, P01 = 0, P02 = 0, P12 = 0;
    unroll<L::Q>([&](auto I) {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        if constexpr (cx != 0) P00 += h[I];
        if constexpr (cy != 0) P11 += h[I];
        if constexpr (cz != 0) P22 += h[I];
        if constexpr (cx * cy != 0) P01 += (CT)(cx * cy) * h[I];
        if constexpr (cx * cz != 0) P02 += (CT)(cx * cz) * h[I];
        if constexpr (cy * cz != 0) P12 += (CT)(cy * cz) * h[I];
    });
    const CT tr3 = (P00 + P11 + P22) * (CT)(1.0 / 3.0);
    unroll<L::Q>([&](auto I) {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        CT qp = -tr3;
        if constexpr (cx != 0) qp += P00;
        if constexpr (cy != 0) qp += P11;
        if constexpr (cz != 0) qp += P22;
        if constexpr (cx * cy != 0) qp += (CT)(2 * cx * cy) * P01;
        if constexpr (cx * cz != 0) qp += (CT)(2 * cx * cz) * P02;
        if constexpr (cy * cz != 0) qp += (CT)(2 * cy * cz) * P12;
        h[I] = heq<L, I>(drho, rho, u[0], u[1], u[2], usq15) + (CT)(4.5 * weight<L>(I)) * qp;
    });
}

// Edge bits of a cell: which box faces it sits on (bits 0-5), and with split
// pairs the seam (bit 6: X = nX/2 - 1, whose +X neighbour is in the high half;
// bit 7: X = nX/2, whose -X neighbour is in the low half).
template <class CT>
__device__ __forceinline__ uint32_t edge_bits(const Params<CT> &p, int X, int Y, int Z) {
    return (uint32_t)(X == 0) | ((uint32_t)(X == p.nX - 1) << 1) | ((uint32_t)(Y == 0) << 2) |
           ((uint32_t)(Y == p.nY - 1) << 3) | ((uint32_t)(Z == 0) << 4) | ((uint32_t)(Z == p.nZ - 1) << 5);
}
// the same with the seam bits of split pairs, for kernels that address
// populations of storage type ST by neighbour offsets
template <class ST, class CT>
__device__ __forceinline__ uint32_t edge_bits_st(const Params<CT> &p, int X, int Y, int Z) {
    uint32_t e = edge_bits(p, X, Y, Z);
    if constexpr (sizeof(ST) == 2)
        if (p.spk) e |= ((uint32_t)(2 * X + 2 == p.nX) << 6) | ((uint32_t)(2 * X == p.nX) << 7);
    return e;
}
constexpr uint32_t kSeams = 0xC0u;

// Periodic Z faces in the select paths.  A wavefront spans Z, so only its
// lanes at Z = 0 or nZ - 1 wrap: the Z step of a neighbour address is -1 / +1
// in the box and nZ - 1 / 1 - nZ across a periodic face.  zl: the step to
// Z - 1, zh: the step to Z + 1 (pe: the cell's periodic face bits).
struct ZWrap {
    int zl, zh;
};
template <class CT>
__device__ __forceinline__ ZWrap z_wrap(const Params<CT> &p, uint32_t pe) {
    return ZWrap{(pe & 16u) ? p.nZ - 1 : -1, (pe & 32u) ? 1 - p.nZ : 1};
}
// address offset of the source x - c_i
template <class L, int I, class CT>
__device__ __forceinline__ int64_t src_off(const Params<CT> &p, const ZWrap &w) {
    const int dz = (L::c[I][2] > 0) ? w.zl : ((L::c[I][2] < 0) ? w.zh : 0);
    return -((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY) + dz;
}
constexpr uint32_t kZFaces = 48u;

// Which directions have a source that is not a plain in-box fluid neighbour
// of the same split-pair half (a seam counts like the X face it mirrors).
template <class L>
__device__ __forceinline__ uint32_t irregular_mask(uint32_t e, uint32_t nbm) {
    e |= ((e >> 6) & 1u) << 1 | ((e >> 7) & 1u);
    uint32_t m = nbm;
    unroll<L::Q>([&](auto I) {
        constexpr uint32_t dm = src_face_bits<L>(I);
        if constexpr (dm != 0)
            if (e & dm) m |= 1u << I;
    });
    return m;
}

// Zou-He face of a cell (-1 if none): on an open Zou-He face and not on a wall face.
template <class CT>
__device__ __forceinline__ int zh_face_of(const Params<CT> &p, uint32_t e) {
    const uint32_t z = e & p.zhmask;
    if (!z || (e & p.wallmask)) return -1;
    return (int)__builtin_ctz(z);
}

// Body force by the exact-difference method (Sec. 4.4 and 6.1, after Kupershtokh):
// hp_i += feq_i(rho, u + du) - feq_i(rho, u), du = F / rho, written as
// w_i rho [3 c.du + 4.5 (c.du)(c.(u + u')) - 1.5 du.(u + u')] with
// u' = u + du, which has no cancellation between two equilibria.
template <class CT>
__device__ __forceinline__ void load_body_force(const Params<CT> &p, int64_t cell, CT &fx, CT &fy, CT &fz) {
    fx = p.fu[0];
    fy = p.fu[1];
    fz = p.fu[2];
    if (p.fld[0]) fx += p.feps * p.fld[0][cell];
    if (p.fld[1]) fy += p.feps * p.fld[1][cell];
    if (p.fld[2]) fz += p.feps * p.fld[2][cell];
}

template <class L, class CT>
__device__ __forceinline__ void add_body_force(CT *hp, CT fx, CT fy, CT fz, CT rho, CT inv, CT ux, CT uy, CT uz) {
    const CT dx = fx * inv, dy = fy * inv, dz = fz * inv;
    const CT sx = (CT)2 * ux + dx, sy = (CT)2 * uy + dy, sz = (CT)2 * uz + dz;
    const CT b = (CT)1.5 * (dx * sx + dy * sy + dz * sz);
    unroll<L::Q>([&](auto I) {
        CT cd = 0, cs = 0;
        if constexpr (L::c[I][0] != 0) { cd += (CT)L::c[I][0] * dx; cs += (CT)L::c[I][0] * sx; }
        if constexpr (L::c[I][1] != 0) { cd += (CT)L::c[I][1] * dy; cs += (CT)L::c[I][1] * sy; }
        if constexpr (L::c[I][2] != 0) { cd += (CT)L::c[I][2] * dz; cs += (CT)L::c[I][2] * sz; }
        hp[I] += (CT)weight<L>(I) * rho * ((CT)3 * cd + (CT)4.5 * cd * cs - b);
    });
}

// KBC collision (Karlin, Bosch & Chikatamarla 2014), D2Q9 / D3Q27: the
// non-equilibrium part n = f - feq splits into a shear part ds -- the
// deviatoric non-equilibrium momentum flux P carried by the axis velocities
// ((P_aa - tr P / D) / 2 each) and the face diagonals (c_a c_b P_ab / 4) -- and
// the rest dh = n - ds; then
//   f*_i = f_i - beta (2 ds_i + gamma dh_i),  beta = omega / 2,
//   gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>,  <x|y> = sum x_i y_i / feq_i
// (gamma = 2, i.e. BGK, when dh = 0).  In deviation variables n_i = h_i - heq_i.
template <class L, class CT>
__device__ __forceinline__ void kbc_relax(const CT *h, CT *hp, const Params<CT> &p, CT drho, CT rho, CT ux, CT uy,
                                          CT uz, CT usq15) {
    constexpr int Q = L::Q;
    // equilibria of opposite directions together: with cu = 3 c_i.u,
    // heq_i = sym + anti and heq_opp(i) = sym - anti, sym = w_i (drho + rho (cu^2/2 - 1.5 u^2)),
    // anti = w_i rho cu
    CT e[Q];
    const CT tx = (CT)3 * ux, ty = (CT)3 * uy, tz = (CT)3 * uz;
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        if constexpr (I == 0) {
            e[0] = (CT)weight<L>(0) * (drho - rho * usq15);
        } else if constexpr (I < O) {
            const CT cu = cdot<L, I>(tx, ty, tz);
            const CT wr = (CT)weight<L>(I) * rho;
            const CT sym = wr * ((CT)0.5 * cu * cu - usq15) + (CT)weight<L>(I) * drho;
            const CT anti = wr * cu;
            e[I] = sym + anti;
            e[O] = sym - anti;
        }
    });
    CT P00 = 0, P11 = 0, P22 = 0, P01 = 0, P02 = 0, P12 = 0;
    unroll<Q>([&](auto I) {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        const CT n = h[I] - e[I];
        if constexpr (cx != 0) P00 += n;
        if constexpr (cy != 0) P11 += n;
        if constexpr (cz != 0) P22 += n;
        if constexpr (cx * cy != 0) P01 += (cx * cy > 0) ? n : -n;
        if constexpr (cx * cz != 0) P02 += (cx * cz > 0) ? n : -n;
        if constexpr (cy * cz != 0) P12 += (cy * cz > 0) ? n : -n;
    });
    const CT trD = (P00 + P11 + P22) * (CT)(1.0 / L::D);
    // shear part: the deviatoric flux on the axis directions ((P_aa - tr P / D) / 2)
    // and the face diagonals (c_a c_b P_ab / 4); zero on rest and corner directions
    const CT sa0 = (CT)0.5 * (P00 - trD), sa1 = (CT)0.5 * (P11 - trD), sa2 = (CT)0.5 * (P22 - trD);
    const CT sb01 = (CT)0.25 * P01, sb02 = (CT)0.25 * P02, sb12 = (CT)0.25 * P12;
    auto has_shear = [](auto I) constexpr {
        constexpr int nzc = (L::c[I][0] != 0) + (L::c[I][1] != 0) + (L::c[I][2] != 0);
        return nzc == 1 || nzc == 2;
    };
    auto shear = [&](auto I) -> CT {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        constexpr int nzc = (cx != 0) + (cy != 0) + (cz != 0);
        if constexpr (nzc == 1) {
            return (cx != 0) ? sa0 : ((cy != 0) ? sa1 : sa2);
        } else {
            constexpr int sgn = (cz == 0) ? cx * cy : ((cy == 0) ? cx * cz : cy * cz);
            const CT b = (cz == 0) ? sb01 : ((cy == 0) ? sb02 : sb12);
            return (sgn > 0) ? b : -b;
        }
    };
    // entropic scalar products <s|dh> and <dh|dh> with weights 1 / feq_i
    CT sh = 0, hh = 0;
    unroll<Q>([&](auto I) {
        const CT n = h[I] - e[I];
        // the hardware reciprocal in FP32 (the weights only scale the two products)
        const CT feq = e[I] + (CT)weight<L>(I) * p.rho0;
        CT inv_feq;
        if constexpr (sizeof(CT) == 4) inv_feq = __builtin_amdgcn_rcpf(feq);
        else inv_feq = (CT)1 / feq;
        if constexpr (has_shear(I)) {
            const CT v = shear(I);
            const CT dh = n - v;
            const CT wd = dh * inv_feq;
            sh += wd * v;
            hh += wd * dh;
        } else {
            hh += n * inv_feq * n;
        }
    });
    const CT beta = (CT)0.5 * p.omega;
    const CT ib = (CT)1 / beta;
    const CT gamma = (hh > (CT)0) ? ib - ((CT)2 - ib) * sh / hh : (CT)2;
    // hp = h - beta (2 s + gamma dh) = h - beta gamma n - beta (2 - gamma) s
    const CT bg = beta * gamma, bs = beta * ((CT)2 - gamma);
    unroll<Q>([&](auto I) {
        const CT t = h[I] - bg * (h[I] - e[I]);
        if constexpr (has_shear(I)) hp[I] = t - bs * shear(I);
        else hp[I] = t;
    });
}

// Collision (eq. LBM-BGK; KB: the KBC collision above) of the deviations h ->
// post-collision hp, returning the moments (u without the force).  FRC: add
// the body force (fx, fy, fz) before the partial bounce-back mix
// hp_i = (1 - s) h*_i + s h_opp(i).
template <class L, bool FRC = false, bool KB = false, class CT>
__device__ __forceinline__ void collide(const CT *h, CT *hp, const Params<CT> &p, CT s, bool has_s,
                                        CT &rho_out, CT &ux, CT &uy, CT &uz, CT fx = 0, CT fy = 0, CT fz = 0) {
    CT drho = 0, jx = 0, jy = 0, jz = 0;
    unroll<L::Q>([&](auto I) {
        drho += h[I];
        if constexpr (L::c[I][0] != 0) jx += (CT)L::c[I][0] * h[I];
        if constexpr (L::c[I][1] != 0) jy += (CT)L::c[I][1] * h[I];
        if constexpr (L::c[I][2] != 0) jz += (CT)L::c[I][2] * h[I];
    });
    const CT rho = p.rho0 + drho;
    const CT inv = (CT)1 / rho;
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
    const CT usq15 = (CT)1.5 * (ux * ux + uy * uy + uz * uz);
    const CT om = p.omega;
    if constexpr (KB) {
        kbc_relax<L>(h, hp, p, drho, rho, ux, uy, uz, usq15);
    } else {
        unroll<L::Q>([&](auto I) {
            const CT e = heq<L, I>(drho, rho, ux, uy, uz, usq15);
            hp[I] = h[I] - om * (h[I] - e);
        });
    }
    if constexpr (FRC) add_body_force<L>(hp, fx, fy, fz, rho, inv, ux, uy, uz);
    if (has_s) {
        CT t[L::Q];
        unroll<L::Q>([&](auto I) { t[I] = ((CT)1 - s) * hp[I] + s * h[opp<L>(I)]; });
        unroll<L::Q>([&](auto I) { hp[I] = t[I]; });
    }
    rho_out = rho;
}

// Boundary value of population k = opp(i) at this cell when its source
// x - c_k = x + c_i is not fluid (nb = classification of that source).
//   wall / solid : hp_i + 6 w_k rho0 (c_k . u_w)          (halfway bounce-back)
//   outflow      : feq_k(rho_face, u(x,t)) - w_k rho0
//   Zou-He face, perimeter cell : equilibrium with (rho0, u_in) or (rho_w, u(x,t))
//   Zou-He face, otherwise      : hp_i (unused: the closure replaces it)
template <class L, int I, class CT>
__device__ __forceinline__ CT fill_value(const Params<CT> &p, const Nb &nb, CT hpi, bool perimeter,
                                         CT rho, CT ux, CT uy, CT uz) {
    constexpr int K = opp<L>(I);
    if (nb.kind == NB_WALL) {
        if (nb.face < 0) return hpi;
        const FaceTab<CT> &F = *p.ft;
        const CT cu = (CT)L::c[K][0] * F.uw[nb.face][0] + (CT)L::c[K][1] * F.uw[nb.face][1] +
                      (CT)L::c[K][2] * F.uw[nb.face][2];
        return hpi + (CT)(6.0 * weight<L>(K)) * p.rho0 * cu;
    }
    if (nb.kind == NB_OUT || (nb.kind == NB_ZH && perimeter)) {
        const FaceTab<CT> &F = *p.ft;
        CT r, vx, vy, vz;
        if (nb.kind == NB_ZH && (F.type[nb.face] == F_ZH_VEL || F.type[nb.face] == F_REG_VEL)) {
            r = p.rho0;
            vx = F.uw[nb.face][0];
            vy = F.uw[nb.face][1];
            vz = F.uw[nb.face][2];
        } else {
            r = F.rho[nb.face];
            vx = ux;
            vy = uy;
            vz = uz;
        }
        const CT usq15 = (CT)1.5 * (vx * vx + vy * vy + vz * vz);
        return heq<L, K>(r - p.rho0, r, vx, vy, vz, usq15);
    }
    return hpi;
    (void)rho;
}

}  // namespace lbm
