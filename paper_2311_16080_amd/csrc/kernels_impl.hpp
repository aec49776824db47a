// kernels_impl.hpp -- kernel templates of the single-domain forward path,
// instantiated per lattice by kernels_d2q9.hip / kernels_d3q19.hip /
// kernels_d3q27.hip.
#pragma once
//
//
//   k_step      fused stream + collide + boundary fill, one pass per step
//               (MODE 0: in-place even step, MODE 1: in-place odd step,
//                MODE 2: double-buffer push step, MODE 3: double-buffer
//                pull step)
//   k_init      f = feq(rho, u) in the storage format          (eq. feq)
//   k_moments   rho, u of the current state + FP64 block sums  (eqs. density, velocity)
//   k_reduce    fixed-order reduction of the block sums
//   k_solid     solid flags -> per-cell flag byte + solid-neighbour mask
//   k_copy      streaming copy (achievable-bandwidth probe)
//
// In-place streaming uses the AA access pattern (Bailey, Myre, Walsh, Lilja &
// Saar 2009): the even step reads a cell's populations and writes the
// post-collision values back into the same cell's opposite slots; the odd step
// gathers from the neighbours' opposite slots and pushes to the neighbours'
// natural slots.  Each cell reads and writes the same address set within a
// step, so one buffer suffices and there is no race.  Every step moves exactly
// 2 Q values per cell.
#include "kernels.hpp"



namespace lbm {

// Block -> (X, Y, Z-chunk).  Workgroups are handed to the 8 XCDs round robin;
// remapping makes each XCD process one contiguous range of rows, so the rows
// a block's neighbours touch mostly sit in the same XCD's L2.
// Optionally (LBM_ZROT=1) lanes are rotated by p.zrot = 32 within a row of
// >= 64 cells, so the row's two end cells share one wavefront; since the wall
// path made boundary wavefronts cheap, aligned rows measure as fast or faster.
// block_cell_at: the same for block b of a G-block covering (a launch that
// covers blocks [b0, b0 + gridDim.x) of it).
// With p.flat, the lanes of a block cover consecutive cells of the whole grid
// (X, Y, Z from the flat index), so rows whose length is not a multiple of 64
// cells still give aligned, fully occupied wavefronts; a wavefront may then
// hold the end of one row and the start of the next.
// PK (2-byte storage): with split pairs the lanes follow storage order, the
// cells of the two X-halves alternating, so that one-cell-per-lane kernels
// touch whole 32-bit words.
template <bool PK = false, class CT>
__device__ __forceinline__ bool block_cell_at(const Params<CT> &p, int b, int G, int &X, int &Y, int &Z) {
    if (PK && p.spk) {
        const uint32_t v = (uint32_t)b * blockDim.x + threadIdx.x;
        const uint32_t c = v >> 1;
        const uint32_t nz = (uint32_t)p.nZ, ny = (uint32_t)p.nY, hx = (uint32_t)(p.nX >> 1);
        const uint32_t r = c / nz;
        Z = (int)(c - r * nz);
        Y = (int)(r % ny);
        const uint32_t xh = r / ny;
        X = (int)(xh + (v & 1u) * hx);
        return xh < hx;
    }
    if (p.flat) {
        const uint32_t cell = (uint32_t)b * blockDim.x + threadIdx.x;
        const uint32_t nz = (uint32_t)p.nZ, ny = (uint32_t)p.nY;
        const uint32_t r = cell / nz;
        Z = (int)(cell - r * nz);
        Y = (int)(r % ny);
        X = (int)(r / ny);
        return X < p.nX;
    }
    if (p.xcd_remap && (G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3);
    const int zc = b % p.zblocks;
    const int r = b / p.zblocks;
    Y = r % p.nY;
    X = r / p.nY;
    const int lin = zc * (int)blockDim.x + (int)threadIdx.x;
    Z = (lin >= p.zrot) ? lin - p.zrot : lin - p.zrot + p.nZ;
    return lin < p.nZ;
}
template <bool PK = false, class CT>
__device__ __forceinline__ bool block_cell(const Params<CT> &p, int &X, int &Y, int &Z) {
    return block_cell_at<PK>(p, (int)blockIdx.x, (int)gridDim.x, X, Y, Z);
}

// One cell of one step.  p: the domain's parameters; A (and B for the push
// step) the domain's state; pending: the state read needs the Zou-He closure.
// XF bit 0: partial bounce-back field; bit 1: body force; bit 3: KBC
// collision (D2Q9 / D3Q27, without the partial bounce-back field); bit 4:
// walls on every lattice face (no general path: measured, the D3Q27 even step
// drops from 181 to 97 VGPRs); bit 2: periodic
// faces on the select path (a variant of its own, so that walls-only domains
// keep the leaner kernel): any periodic face in the local even step, which has
// no neighbour addresses, and periodic Z faces in the odd / push steps.
template <class L, class ST, int MODE, int XF, int NT>
__device__ __forceinline__ void step_cell(const Params<typename Store<ST>::CT> &p, ST *__restrict__ A,
                                          ST *__restrict__ B, int X, int Y, int Z, int pending) {
    // NT 0: plain accesses.  NT 1: non-temporal loads and stores wherever the
    // access is aligned with the wavefront (the local even step; directions
    // without a Z component in the odd / push steps); Z-shifted accesses stay
    // cached, since neighbouring wavefronts share their boundary cache lines.
    // NT 2: non-temporal everywhere.  NT 3: as 1 plus non-temporal Z-shifted
    // stores.  NT 4: as 1 plus non-temporal Z-shifted loads.
    constexpr bool HAS_S = (XF & 1) != 0;
    constexpr bool FRC = (XF & 2) != 0;
    constexpr bool PZ = (XF & 4) != 0;
    constexpr bool KB = (XF & 8) != 0;   // KBC collision
    constexpr bool WALLS_ONLY = (XF & 16) != 0;   // every lattice face is a wall
    // Reads gather from the neighbours (in-place odd step, pull step) or read
    // the cell's own slots (even step, push step); writes go to the cell's own
    // opposite slots (even step, pull step) or to the neighbours.  The pull
    // step reads A and writes B: A holds what an in-place even step leaves
    // (f*_i(x) in slot opp(i) of x), and so does B afterwards.
    constexpr bool GATHER = (MODE == 1 || MODE == 3);
    constexpr bool LOCAL_W = (MODE == 0 || MODE == 3);
    constexpr bool NTA = (NT >= 1);
    constexpr bool NTZL = (NT == 2) || (NT == 4);
    constexpr bool NTZS = (NT == 2) || (NT == 3);
    using CT = typename Store<ST>::CT;
    constexpr int Q = L::Q;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    // populations are addressed by storage index: sc for this cell, sm per cell step
    const int64_t sc = sidx<ST>(p, cell);
    const int64_t sm = smul<ST>(p);
    uint32_t nbm = 0;
    if (p.flags) {
        const uint8_t fl = p.flags[cell];
        if (fl & 1) return;                 // solid cells carry no state
        if (fl & 2) nbm = p.nbm[cell];
    }
    CT fx = 0, fy = 0, fz = 0;
    if constexpr (FRC) load_body_force(p, cell, fx, fy, fz);   // issued with the population loads
    const uint32_t e = edge_bits_st<ST>(p, X, Y, Z);
    const uint32_t irr = irregular_mask<L>(e, nbm);

    // Wavefronts of interior cells only (no face, no solid neighbour): plain
    // loads and stores, no per-direction boundary tests.
    if (__all(irr == 0)) {
        CT h[Q];
        if constexpr (GATHER) {
            unroll<Q>([&](auto I) {
                constexpr int O = opp<L>(I);
                const int64_t src = sc - sm * ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]);
                h[I] = ldh<L, ST, O, (L::c[I][2] == 0) ? NTA : NTZL>(A, src);
            });
        } else {
            unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I, NTA>(A, sc); });
        }
        CT hp[Q];
        CT rho, ux, uy, uz;
        CT s = 0;
        if constexpr (HAS_S) s = (CT)p.s[cell];
        collide<L, FRC, KB>(h, hp, p, s, HAS_S, rho, ux, uy, uz, fx, fy, fz);
        ST *W = (MODE >= 2) ? B : A;
        unroll<Q>([&](auto I) {
            constexpr int O = opp<L>(I);
            if constexpr (LOCAL_W) {
                sth<L, ST, O, NTA>(W, sc, hp[I]);
            } else {
                const int64_t dst = sc + sm * ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]);
                sth<L, ST, I, (L::c[I][2] == 0) ? NTA : NTZS>(W, dst, hp[I]);
            }
        });
        return;
    }

    // Wavefronts whose only non-regular directions meet wall faces, solid
    // cells or (PZ) periodic faces: halfway bounce-back with the moving-wall
    // term and periodic images, chosen per lane by selects.  Same values as
    // the general path below (classify_src, fill_value), without the
    // per-direction classification; a direction across a wall face and a
    // periodic face bounces back, as there.
    constexpr uint32_t kFaces = all_face_bits<L>();
    const uint32_t sel_faces = p.wallmask | (PZ ? (MODE == 0 ? p.permask : (p.permask & kZFaces)) : 0u);
    if (__all((e & (kFaces | kSeams) & ~sel_faces) == 0)) {
        const ZWrap zw = (PZ && MODE != 0) ? z_wrap(p, e & p.permask) : ZWrap{-1, 1};
        // wall faces of this cell (without PZ, e's lattice faces are all walls here)
        const uint32_t we = PZ ? (e & p.wallmask) : e;
        CT h[Q];
        if constexpr (GATHER) {
            unroll<Q>([&](auto I) {
                constexpr int O = opp<L>(I);
                // x - c_i is across a wall or solid
                const bool wall = ((we & src_face_bits<L>(I)) | (nbm & (1u << I))) != 0;
                const ST *nb = pop_ptr<L, O>(A, sc + sm * src_off<L, I>(p, zw));
                const ST *ptr = wall ? pop_ptr<L, I>(A, sc) : nb;
                h[I] = ldp<L, ST, O, (L::c[I][2] == 0) ? NTA : NTZL>(ptr);  // w_O = w_I
            });
        } else {
            unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I, NTA>(A, sc); });
        }
        CT hp[Q];
        CT rho, ux, uy, uz;
        CT s = 0;
        if constexpr (HAS_S) s = (CT)p.s[cell];
        collide<L, FRC, KB>(h, hp, p, s, HAS_S, rho, ux, uy, uz, fx, fy, fz);
        ST *W = (MODE >= 2) ? B : A;
        unroll<Q>([&](auto I) {
            constexpr int O = opp<L>(I);
            constexpr uint32_t fb = src_face_bits<L>(O);     // faces x + c_i can lie across
            constexpr bool NTW = (LOCAL_W || L::c[I][2] == 0) ? NTA : NTZS;
            const uint32_t cr = we & fb;
            const bool wall = (cr | (nbm & (1u << O))) != 0;  // x + c_i is across a wall or solid
            ST *own = pop_ptr<L, O>(W, sc);
            ST *ptr = own;
            if constexpr (!LOCAL_W)
                ptr = wall ? own : pop_ptr<L, I>(W, sc + sm * src_off<L, O>(p, zw));  // x + c_i = x - c_opp(i)
            CT v = hp[I];
            if (cr && !(cr & p.staticmask)) {
                // moving wall: the lowest-index face crossed (static walls win);
                // its velocity from the device face table, as in fill_value
                const int f = (int)__builtin_ctz(cr);
                const FaceTab<CT> &F = *p.ft;
                const CT cu = (CT)L::c[O][0] * F.uw[f][0] + (CT)L::c[O][1] * F.uw[f][1] + (CT)L::c[O][2] * F.uw[f][2];
                v = hp[I] + (CT)(6.0 * weight<L>(O)) * p.rho0 * cu;
            }
            stp<L, ST, I, NTW>(ptr, v);  // w_O = w_I
        });
        return;
    }

    // With walls on every lattice face the select path above takes every
    // wavefront that is not interior; the variant drops the general path and
    // the registers it needs.
    if constexpr (WALLS_ONLY) return;

    // Every direction issues exactly one load and one store: the address (and,
    // for a boundary fill, the value) is chosen per lane, so wavefronts that
    // hold a few boundary cells do not run extra memory instructions.
    CT h[Q];
    if constexpr (GATHER) {
        unroll<Q>([&](auto I) {
            constexpr int O = opp<L>(I);
            const ST *ptr;
            if (!((irr >> I) & 1u)) {
                ptr = pop_ptr<L, O>(A, sc - sm * ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]));
            } else {
                const Nb nb = classify_src<L>(p, X, Y, Z, I, nbm);
                ptr = (nb.kind == NB_FLUID) ? pop_ptr<L, O>(A, sidx<ST>(p, nb.cell)) : pop_ptr<L, I>(A, sc);
            }
            h[I] = ldp<L, ST, O, (L::c[I][2] == 0) ? NTA : NTZL>(ptr);  // w_O = w_I
        });
    } else {
        unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I, NTA>(A, sc); });
    }

    const int zf = zh_face_of(p, e);
    if (zf >= 0 && (GATHER || pending)) zouhe<L>(h, p, zf);

    CT hp[Q];
    CT rho, ux, uy, uz;
    CT s = 0;
    if constexpr (HAS_S) s = (CT)p.s[cell];
    collide<L, FRC, KB>(h, hp, p, s, HAS_S, rho, ux, uy, uz, fx, fy, fz);
    const bool perim = (e & p.wallmask) != 0;

    ST *W = (MODE >= 2) ? B : A;
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        constexpr bool NTW = (LOCAL_W || L::c[I][2] == 0) ? NTA : NTZS;
        ST *ptr;
        CT v = hp[I];
        if (!((irr >> O) & 1u)) {
            if constexpr (LOCAL_W) ptr = pop_ptr<L, O>(W, sc);
            else ptr = pop_ptr<L, I>(W, sc + sm * ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]));
        } else {
            const Nb nb = classify_src<L>(p, X, Y, Z, O, nbm);   // the cell x + c_i
            if (nb.kind == NB_FLUID) {
                if constexpr (LOCAL_W) ptr = pop_ptr<L, O>(W, sc);
                else ptr = pop_ptr<L, I>(W, sidx<ST>(p, nb.cell));
            } else {
                ptr = pop_ptr<L, O>(W, sc);
                v = fill_value<L, I>(p, nb, hp[I], perim, rho, ux, uy, uz);
            }
        }
        stp<L, ST, I, NTW>(ptr, v);  // w_O = w_I
    });
}

// Waves per SIMD the register allocation leaves room for: the compiler's
// choice, except the walls-only KBC variant on D3Q27 in FP32, held at 3
// (<= 168 VGPRs; its steps need 151-167 without spilling).  At 2 waves its
// local step ran 774 us on the 256^3 cavity against 636 us at 3; at 4 waves
// (128 VGPRs) every step spills 30-44 registers.  FP64 and the 2-byte storages
// would spill at 3.
template <class L, class ST, int MODE, int XF>
struct StepWaves {
    static constexpr int value = (L::Q == 27 && (XF & 24) == 24 && std::is_same<ST, float>::value) ? 3 : 1;
};

template <class L, class ST, int MODE, int XF, int NT>
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(StepWaves<L, ST, MODE, XF>::value)))
k_step(const Params<typename Store<ST>::CT> p, ST *__restrict__ A, ST *__restrict__ B) {
    int X, Y, Z;
    if (!block_cell<sizeof(ST) == 2>(p, X, Y, Z)) return;
    step_cell<L, ST, MODE, XF, NT>(p, A, B, X, Y, Z, p.zh_pending);
}

}  // namespace lbm

#include "pair_impl.hpp"

namespace lbm {

// f = feq(rho, u) written in natural order.  rho: N, u: D planes of N in the
// caller's axes; IT = float or double.
template <class L, class ST, class IT>
__global__ void __launch_bounds__(kMaxBlock) k_init(const Params<typename Store<ST>::CT> p, ST *__restrict__ A,
                                                    const IT *__restrict__ rho_in, const IT *__restrict__ u_in,
                                                    int64_t N) {
    using CT = typename Store<ST>::CT;
    int X, Y, Z;
    if (!block_cell<sizeof(ST) == 2>(p, X, Y, Z)) return;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    const bool solid = p.flags && (p.flags[cell] & 1);
    CT rho = rho_in ? (CT)rho_in[cell] : p.rho0;
    CT u[3] = {0, 0, 0};
    if (u_in) {
        if constexpr (L::D == 2) {
            u[1] = (CT)u_in[cell];
            u[2] = (CT)u_in[N + cell];
        } else {
            u[0] = (CT)u_in[cell];
            u[1] = (CT)u_in[N + cell];
            u[2] = (CT)u_in[2 * N + cell];
        }
    }
    const CT usq15 = (CT)1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const CT drho = rho - p.rho0;
    const int64_t sc = sidx<ST>(p, cell);
    unroll<L::Q>([&](auto I) {
        CT v = solid ? (CT)0 : heq<L, I>(drho, rho, u[0], u[1], u[2], usq15);
        sth<L, ST, I>(A, sc, v);
    });
}

// Moments of one cell of the current state.  ODD = the state is the AA buffer
// after an even step (post-collision values in swapped slots): the
// populations are gathered as the odd step would.  Returns false for a solid
// cell (rho0, u = 0).
template <class L, class ST, bool ODD>
__device__ __forceinline__ bool moments_cell(const Params<typename Store<ST>::CT> &p, const ST *__restrict__ A,
                                             int X, int Y, int Z, int pending, typename Store<ST>::CT &rho,
                                             typename Store<ST>::CT &ux, typename Store<ST>::CT &uy,
                                             typename Store<ST>::CT &uz) {
    using CT = typename Store<ST>::CT;
    constexpr int Q = L::Q;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    uint32_t nbm = 0;
    rho = p.rho0;
    ux = uy = uz = 0;
    if (p.flags) {
        const uint8_t fl = p.flags[cell];
        if (fl & 1) return false;
        if (fl & 2) nbm = p.nbm[cell];
    }
    const uint32_t e = edge_bits_st<ST>(p, X, Y, Z);
    const uint32_t irr = irregular_mask<L>(e, nbm);
    const int64_t sc = sidx<ST>(p, cell);
    const int64_t sm = smul<ST>(p);
    CT h[Q];
    if constexpr (ODD) {
        unroll<Q>([&](auto I) {
            constexpr int O = opp<L>(I);
            if (!((irr >> I) & 1u)) {
                const int64_t src = sc - sm * ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]);
                h[I] = ldh<L, ST, O>(A, src);
            } else {
                const Nb nb = classify_src<L>(p, X, Y, Z, I, nbm);
                h[I] = (nb.kind == NB_FLUID) ? ldh<L, ST, O>(A, sidx<ST>(p, nb.cell)) : ldh<L, ST, I>(A, sc);
            }
        });
    } else {
        unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I>(A, sc); });
    }
    const int zf = zh_face_of(p, e);
    if (zf >= 0 && (ODD || pending)) zouhe<L>(h, p, zf);
    CT drho = 0, jx = 0, jy = 0, jz = 0;
    unroll<Q>([&](auto I) {
        drho += h[I];
        if constexpr (L::c[I][0] != 0) jx += (CT)L::c[I][0] * h[I];
        if constexpr (L::c[I][1] != 0) jy += (CT)L::c[I][1] * h[I];
        if constexpr (L::c[I][2] != 0) jz += (CT)L::c[I][2] * h[I];
    });
    rho = p.rho0 + drho;
    const CT inv = (CT)1 / rho;
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
    return true;
}

// Block sum of the five moment sums into partial[row * 5 ..]: a butterfly
// within each wavefront, then the wavefront totals in wavefront order.  Any
// block of whole wavefronts (64, 128, 192 or 256 lanes) is summed completely,
// and the order is fixed, so the result is deterministic.
__device__ __forceinline__ void block_sums(const double (&m)[5], double *partial, int64_t row) {
    __shared__ double red[5][kMaxBlock / 64];
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    unroll<5>([&](auto K) {
        double v = m[K];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[K][wv] = v;
    });
    __syncthreads();
    if ((int)threadIdx.x < 5) {
        const int nw = ((int)blockDim.x + 63) / 64;
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[threadIdx.x][w];
        partial[row * 5 + threadIdx.x] = t;
    }
}

template <class L, class CT, class OT>
__device__ __forceinline__ void store_moments(OT *rho_out, OT *u_out, int64_t gcell, int64_t N, CT rho, CT ux, CT uy,
                                              CT uz) {
    if (rho_out) rho_out[gcell] = (OT)rho;
    if (u_out) {
        if constexpr (L::D == 2) {
            u_out[gcell] = (OT)uy;
            u_out[N + gcell] = (OT)uz;
        } else {
            u_out[gcell] = (OT)ux;
            u_out[N + gcell] = (OT)uy;
            u_out[2 * N + gcell] = (OT)uz;
        }
    }
}

// rho, u of the current state in the caller's axes (OT) and one row of FP64
// partial sums per block: mass, P_X, P_Y, P_Z, kinetic energy.
template <class L, class ST, class OT, bool ODD>
__global__ void __launch_bounds__(kMaxBlock) k_moments(const Params<typename Store<ST>::CT> p,
                                                       const ST *__restrict__ A, OT *__restrict__ rho_out,
                                                       OT *__restrict__ u_out, double *__restrict__ partial,
                                                       int64_t N) {
    using CT = typename Store<ST>::CT;
    int X, Y, Z;
    const bool inside = block_cell<sizeof(ST) == 2>(p, X, Y, Z);
    double m[5] = {0, 0, 0, 0, 0};
    if (inside) {
        CT rho, ux, uy, uz;
        if (moments_cell<L, ST, ODD>(p, A, X, Y, Z, p.zh_pending, rho, ux, uy, uz)) {
            const double r = (double)rho, vx = (double)ux, vy = (double)uy, vz = (double)uz;
            m[0] = r;
            m[1] = r * vx;
            m[2] = r * vy;
            m[3] = r * vz;
            m[4] = 0.5 * r * (vx * vx + vy * vy + vz * vz);
        }
        store_moments<L>(rho_out, u_out, ((int64_t)X * p.nY + Y) * p.nZ + Z, N, rho, ux, uy, uz);
    }
    if (partial) block_sums(m, partial, blockIdx.x);
}

// Per-cell flag byte (bit0 solid, bit1 some source x - c_k is solid) and the
// solid-neighbour mask, from N solid bytes.  Periodic faces wrap.
template <class L>
__global__ void __launch_bounds__(kMaxBlock) k_solid(const Params<float> p, const uint8_t *__restrict__ solid,
                                                     uint8_t *__restrict__ flags, uint32_t *__restrict__ nbm) {
    int X, Y, Z;
    if (!block_cell(p, X, Y, Z)) return;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    if (solid[cell]) {
        flags[cell] = 1;
        nbm[cell] = 0;
        return;
    }
    uint32_t m = 0;
    for (int k = 1; k < L::Q; ++k) {
        int y[3] = {X - L::c[k][0], Y - L::c[k][1], Z - L::c[k][2]};
        const int n[3] = {p.nX, p.nY, p.nZ};
        bool in = true;
        for (int a = 0; a < 3; ++a) {
            if (y[a] < 0) {
                if (p.ftype[2 * a] == F_PERIODIC) y[a] += n[a];
                else in = false;
            } else if (y[a] >= n[a]) {
                if (p.ftype[2 * a + 1] == F_PERIODIC) y[a] -= n[a];
                else in = false;
            }
        }
        if (in && solid[((int64_t)y[0] * p.nY + y[1]) * p.nZ + y[2]]) m |= 1u << k;
    }
    nbm[cell] = m;
    flags[cell] = m ? 2 : 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers (dispatch on lattice and storage type).
// ---------------------------------------------------------------------------
template <class L, class ST>
hipError_t step_t(const Launch &g, int mode, bool has_s) {
    using CT = typename Store<ST>::CT;
    const Params<CT> &p = *static_cast<const Params<CT> *>(g.params);
    ST *A = static_cast<ST *>(g.A);
    ST *B = static_cast<ST *>(g.B);
    if constexpr (sizeof(ST) == 2) {
        // split pairs: every step but the push step on the two-cell kernel
        if (p.spk && g.pair && !g.force && !g.kbc && mode != 2) {
            // no solid cells and walls on every lattice face: the kernel without the
            // per-cell fallback
            const bool nofb = !p.flags && (p.wallmask & all_face_bits<L>()) == all_face_bits<L>();
#define LBM_SPLIT_CASE(M, S, NF) \
    if (mode == M && has_s == S && nofb == NF) hipLaunchKernelGGL((k_step_split<L, ST, M, S, NF>), dim3(g.pgrid), dim3(g.pblock), 0, g.stream, p, A, B);
            LBM_SPLIT_CASE(0, false, false)
            LBM_SPLIT_CASE(1, false, false)
            LBM_SPLIT_CASE(3, false, false)
            LBM_SPLIT_CASE(0, true, false)
            LBM_SPLIT_CASE(1, true, false)
            LBM_SPLIT_CASE(3, true, false)
            LBM_SPLIT_CASE(0, false, true)
            LBM_SPLIT_CASE(1, false, true)
            LBM_SPLIT_CASE(3, false, true)
            LBM_SPLIT_CASE(0, true, true)
            LBM_SPLIT_CASE(1, true, true)
            LBM_SPLIT_CASE(3, true, true)
#undef LBM_SPLIT_CASE
            return hipGetLastError();
        }
        // two cells per lane (walls and, in the even step, periodic faces on its
        // own path); not with a body force or the KBC collision.  pair 1: even
        // and pull steps; 2: odd steps too (measurement).
        if (!g.force && !g.kbc && g.pair && mode != 2 && (mode != 1 || g.pair == 2)) {
            // no solid cells and walls on every lattice face: the variant without
            // the per-cell fallback (D3Q19 even step 99 vs 109 VGPRs; 2% faster)
            const bool walls = !p.flags && (p.wallmask & all_face_bits<L>()) == all_face_bits<L>();
#define LBM_PAIR_CASE(M, S, NF)                                                                                     \
    if (mode == M && has_s == S && walls == NF)                                                                     \
        hipLaunchKernelGGL((k_step_pair<L, ST, M, S, NF>), dim3(g.pgrid), dim3(g.pblock), 0, g.stream, p, A, B);
            LBM_PAIR_CASE(0, false, false)
            LBM_PAIR_CASE(1, false, false)
            LBM_PAIR_CASE(0, true, false)
            LBM_PAIR_CASE(1, true, false)
            LBM_PAIR_CASE(0, false, true)
            LBM_PAIR_CASE(1, false, true)
            LBM_PAIR_CASE(0, true, true)
            LBM_PAIR_CASE(1, true, true)
            LBM_PAIR_CASE(3, false, false)
            LBM_PAIR_CASE(3, true, false)
            LBM_PAIR_CASE(3, false, true)
            LBM_PAIR_CASE(3, true, true)
#undef LBM_PAIR_CASE
            return hipGetLastError();
        }
    }
    // walls on every lattice face, nothing else: the variant without the general
    // path.  Measured on 256^3 / 4096^2 cavities: D3Q27 FP32 +7.7%, D2Q9 FP32
    // +1.2%, D3Q27 FP16 +2.5%; D3Q19 FP32 -1.7% (its higher occupancy costs
    // bandwidth there), so D3Q19 keeps the full kernel.
    if constexpr (L::Q != 19) {
        constexpr int NTD0 = sizeof(ST) == 2 ? 0 : 1;
        // (not with split pairs: their seam planes need the general path)
        if ((p.wallmask & all_face_bits<L>()) == all_face_bits<L>() && !has_s && !g.force && !g.kbc &&
            g.nt == NTD0 && g.walls_only && !p.spk) {
            if (mode == 0)
                hipLaunchKernelGGL((k_step<L, ST, 0, 16, NTD0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
            else if (mode == 1)
                hipLaunchKernelGGL((k_step<L, ST, 1, 16, NTD0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
            else if (mode == 2)
                hipLaunchKernelGGL((k_step<L, ST, 2, 16, NTD0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
            else
                hipLaunchKernelGGL((k_step<L, ST, 3, 16, NTD0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
            return hipGetLastError();
        }
    }
    // periodic faces of the lattice's own axes (2-D: not the dummy X axis)
    const uint32_t per = p.permask & all_face_bits<L>();
    const bool pz = (mode == 0) ? per != 0 : (per & kZFaces) != 0;
    if (g.force || pz || g.kbc) {
        // body force, periodic faces and / or KBC: the one-cell-per-lane kernel
        // with the storage type's default memory hints (plain for 2-byte
        // storage, non-temporal where aligned otherwise)
        constexpr int NTD = sizeof(ST) == 2 ? 0 : 1;
        // KBC with walls on every lattice face: the variant without the general
        // path (D3Q27 FP32 local step 254 -> 179 VGPRs; 256^3 cavity 19.2k ->
        // 21.8k MLUPS with the local step at 3 waves; D2Q9 4096^2 76.4k -> 85.0k)
        const bool kwo = g.kbc && !has_s && !g.force && g.walls_only && !p.spk &&
                         (p.wallmask & all_face_bits<L>()) == all_face_bits<L>();
        const int xf = (has_s ? 1 : 0) | (g.force ? 2 : 0) | (pz ? 4 : 0) | (g.kbc ? 8 : 0) | (kwo ? 16 : 0);
#define LBM_XF_CASE(M, X)                                                                                    \
    if (mode == M && xf == X) {                                                                              \
        hipLaunchKernelGGL((k_step<L, ST, M, X, NTD>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B); \
        return hipGetLastError();                                                                            \
    }
        LBM_XF_CASE(0, 2)
        LBM_XF_CASE(0, 3)
        LBM_XF_CASE(0, 4)
        LBM_XF_CASE(0, 5)
        LBM_XF_CASE(0, 6)
        LBM_XF_CASE(0, 7)
        LBM_XF_CASE(1, 2)
        LBM_XF_CASE(1, 3)
        LBM_XF_CASE(1, 4)
        LBM_XF_CASE(1, 5)
        LBM_XF_CASE(1, 6)
        LBM_XF_CASE(1, 7)
        LBM_XF_CASE(2, 2)
        LBM_XF_CASE(2, 3)
        LBM_XF_CASE(2, 4)
        LBM_XF_CASE(2, 5)
        LBM_XF_CASE(2, 6)
        LBM_XF_CASE(2, 7)
        LBM_XF_CASE(3, 2)
        LBM_XF_CASE(3, 3)
        LBM_XF_CASE(3, 4)
        LBM_XF_CASE(3, 5)
        LBM_XF_CASE(3, 6)
        LBM_XF_CASE(3, 7)
        if constexpr (L::Q != 19) {
            LBM_XF_CASE(0, 8)
            LBM_XF_CASE(0, 10)
            LBM_XF_CASE(0, 12)
            LBM_XF_CASE(0, 14)
            LBM_XF_CASE(1, 8)
            LBM_XF_CASE(1, 10)
            LBM_XF_CASE(1, 12)
            LBM_XF_CASE(1, 14)
            LBM_XF_CASE(2, 8)
            LBM_XF_CASE(2, 10)
            LBM_XF_CASE(2, 12)
            LBM_XF_CASE(2, 14)
            LBM_XF_CASE(3, 8)
            LBM_XF_CASE(3, 10)
            LBM_XF_CASE(3, 12)
            LBM_XF_CASE(3, 14)
            LBM_XF_CASE(0, 24)
            LBM_XF_CASE(1, 24)
            LBM_XF_CASE(2, 24)
            LBM_XF_CASE(3, 24)
        }
#undef LBM_XF_CASE
        return hipErrorInvalidValue;
    }
#define LBM_STEP_CASE(M, S)                                                                            \
    if (mode == M && has_s == S) {                                                                     \
        switch (g.nt) {                                                                                \
            case 0: hipLaunchKernelGGL((k_step<L, ST, M, S, 0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B); break; \
            case 2: hipLaunchKernelGGL((k_step<L, ST, M, S, 2>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B); break; \
            case 3: hipLaunchKernelGGL((k_step<L, ST, M, S, 3>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B); break; \
            case 4: hipLaunchKernelGGL((k_step<L, ST, M, S, 4>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B); break; \
            default: hipLaunchKernelGGL((k_step<L, ST, M, S, 1>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B); break; \
        }                                                                                              \
        return hipGetLastError();                                                                      \
    }
    LBM_STEP_CASE(0, false)
    LBM_STEP_CASE(1, false)
    LBM_STEP_CASE(2, false)
    LBM_STEP_CASE(0, true)
    LBM_STEP_CASE(1, true)
    LBM_STEP_CASE(2, true)
#undef LBM_STEP_CASE
    // pull step: the default memory hints, or plain accesses (LBM_NT=0)
    if (mode == 3) {
        if (g.nt == 0) {
            if (has_s) hipLaunchKernelGGL((k_step<L, ST, 3, 1, 0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
            else hipLaunchKernelGGL((k_step<L, ST, 3, 0, 0>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
        } else {
            if (has_s) hipLaunchKernelGGL((k_step<L, ST, 3, 1, 1>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
            else hipLaunchKernelGGL((k_step<L, ST, 3, 0, 1>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A, B);
        }
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <class L, class ST>
hipError_t init_t(const Launch &g, const void *rho, const void *u, int in_f64, int64_t N) {
    using CT = typename Store<ST>::CT;
    const Params<CT> &p = *static_cast<const Params<CT> *>(g.params);
    ST *A = static_cast<ST *>(g.A);
    if (in_f64)
        hipLaunchKernelGGL((k_init<L, ST, double>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A,
                           static_cast<const double *>(rho), static_cast<const double *>(u), N);
    else
        hipLaunchKernelGGL((k_init<L, ST, float>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A,
                           static_cast<const float *>(rho), static_cast<const float *>(u), N);
    return hipGetLastError();
}

template <class L, class ST>
hipError_t moments_t(const Launch &g, bool odd, void *rho, void *u, int out_f64, double *partial, int64_t N) {
    using CT = typename Store<ST>::CT;
    const Params<CT> &p = *static_cast<const Params<CT> *>(g.params);
    const ST *A = static_cast<const ST *>(g.A);
#define LBM_MOM_CASE(OT, ODD)                                                                                  \
    hipLaunchKernelGGL((k_moments<L, ST, OT, ODD>), dim3(g.grid), dim3(g.block), 0, g.stream, p, A,           \
                       static_cast<OT *>(rho), static_cast<OT *>(u), partial, N);
    if (out_f64) {
        if (odd) { LBM_MOM_CASE(double, true) } else { LBM_MOM_CASE(double, false) }
    } else {
        if (odd) { LBM_MOM_CASE(float, true) } else { LBM_MOM_CASE(float, false) }
    }
#undef LBM_MOM_CASE
    return hipGetLastError();
}

// Momentum-exchange force (Ladd) of the step that produced the current state.
// For a fluid cell x and a direction i whose neighbour x + c_i is a solid
// cell or lies across a wall face, the population that left along c_i came
// back as f_opp(i)(x, t + 1) = f°_i + 6 w_opp rho0 (c_opp . u_w), stored in the
// cell's own slot opp(i) in either AA parity; the link hands
// (2 f_opp(i) - 6 w_opp rho0 c_opp . u_w) c_i of momentum to the solid / wall.
// rows: one row of kForceSlots FP64 sums per block: [0..2] solids,
// [3 + 3 f + a] wall face f (internal faces and axes; a link across several
// wall faces counts for the lowest-index one).
constexpr int kForceSlots = 21;

// This launch covers blocks [b0, b0 + gridDim.x) of the step grid of G blocks
// and writes its rows at rows[0 ..).
template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_forces(const Params<typename Store<ST>::CT> p, const ST *__restrict__ A,
                                                      double *__restrict__ rows, int64_t b0, int64_t G) {
    constexpr int Q = L::Q;
    __shared__ double red[kForceSlots][kMaxBlock / 64];
    int X, Y, Z;
    double part[kForceSlots];
#pragma unroll
    for (int k = 0; k < kForceSlots; ++k) part[k] = 0.0;
    bool links = false;
    if (block_cell_at<sizeof(ST) == 2>(p, (int)(b0 + (int64_t)blockIdx.x), (int)G, X, Y, Z)) {
        const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
        uint32_t nbm = 0;
        bool solid = false;
        if (p.flags) {
            const uint8_t fl = p.flags[cell];
            solid = fl & 1;
            if (fl & 2) nbm = p.nbm[cell];
        }
        const uint32_t e = edge_bits(p, X, Y, Z);
        if (!solid && (nbm || (e & p.wallmask))) {
            unroll<Q>([&](auto I) {
                constexpr int O = opp<L>(I);
                if constexpr (I != 0) {
                    const uint32_t cr = e & src_face_bits<L>(O) & p.wallmask;  // x + c_i across wall faces
                    const bool wall = cr != 0;
                    if (wall || ((nbm >> O) & 1u)) {
                        links = true;
                        const double back = (double)ldh<L, ST, O>(A, sidx<ST>(p, cell)) + weight<L>(O) * (double)p.rho0;
                        double term = 0.0;
                        int base = 0;
                        if (wall) {
                            const int f = (int)__builtin_ctz(cr);
                            base = 3 + 3 * f;
                            if (!(cr & p.staticmask)) {
                                const FaceTab<typename Store<ST>::CT> &F = *p.ft;
                                term = 6.0 * weight<L>(O) * (double)p.rho0 *
                                       ((double)L::c[O][0] * (double)F.uw[f][0] + (double)L::c[O][1] * (double)F.uw[f][1] +
                                        (double)L::c[O][2] * (double)F.uw[f][2]);
                            }
                        }
                        const double ex = 2.0 * back - term;
                        for (int k = 0; k < kForceSlots; k += 3)
                            if (k == base) {
                                part[k] += ex * L::c[I][0];
                                part[k + 1] += ex * L::c[I][1];
                                part[k + 2] += ex * L::c[I][2];
                            }
                    }
                }
            });
        }
    }
    // fixed-order block sums (wavefronts without links contribute zeros)
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    if (__any(links)) {
        for (int k = 0; k < kForceSlots; ++k) {
            double v = part[k];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) red[k][wv] = v;
        }
    } else if (lane == 0) {
        for (int k = 0; k < kForceSlots; ++k) red[k][wv] = 0.0;
    }
    __syncthreads();
    if ((int)threadIdx.x < kForceSlots) {
        const int nw = ((int)blockDim.x + 63) / 64;
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[threadIdx.x][w];
        rows[(int64_t)blockIdx.x * kForceSlots + threadIdx.x] = t;
    }
}

// blocks [b0, b0 + nb) of the step grid (nb = 0: all of it)
template <class L, class ST>
hipError_t forces_t(const Launch &g, double *rows, int64_t b0, int64_t nb) {
    using CT = typename Store<ST>::CT;
    const Params<CT> &p = *static_cast<const Params<CT> *>(g.params);
    if (nb <= 0) nb = (int64_t)g.grid - b0;
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_forces<L, ST>), dim3((unsigned)nb), dim3(g.block), 0, g.stream, p,
                       static_cast<const ST *>(g.A), rows, b0, (int64_t)g.grid);
    return hipGetLastError();
}

// Interpolated bounce-back (Bouzidi, Firdaouss & Lallemand 2001) on the curved
// links, after the step kernel has written halfway bounce-back.  With s along
// c_i (cell x_b at 0, wall at q, x_ff = x_b - c_i at -1, x_fff at -2):
//   q <  1/2: f_opp(x_b, t+1) = the post-collision field f*_i at s = 2q - 1
//             (Lagrange weights through s = 0, -1 (, -2));
//   q >= 1/2: f_opp(x_b, t+1) = the opp-field at t+1 at s = 0 through the
//             turned f*_i(x_b) at s = 2q - 1 and f*_opp(x_b), f*_opp(x_ff)
//             at s = -1, -2.
// Every value needed is in the state after the step:
//   f*_i(x_b)    the halfway value, own slot opp (either layout);
//   f*_i(x_ff)   = f_i(x_b, t+1):  natural: slot i of x_b;    else slot opp of x_ff
//   f*_i(x_fff)  = f_i(x_ff, t+1): natural: slot i of x_ff;   else slot opp of x_fff
//   f*_opp(x_b)  = f_opp(x_ff, t+1): natural: slot opp of x_ff; else slot i of x_b
//   f*_opp(x_ff) = f_opp(x_fff, t+1): natural: slot opp of x_fff; else slot i of x_ff
// (else = after an in-place even step, where f_j(y, t+1) sits in slot opp(j)
// of y - c_j).  None of these slots is the halfway slot of another link (the
// link list holds only links whose x_ff -- and x_fff for quadratic weights --
// are fluid), so the links are independent.  The interpolation is linear with
// weights summing to one and w_i = w_opp, so it runs on the stored values
// directly (FP16 / BF16: on h / w).
template <class L, class ST>
__global__ void __launch_bounds__(256) k_bouzidi(const Params<typename Store<ST>::CT> p, ST *__restrict__ A,
                                                 const LinkTab<typename Store<ST>::CT> lt, int natural) {
    using CT = typename Store<ST>::CT;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= lt.n) return;
    const int i = lt.dir[k];
    const int kind = lt.kind[k];
    const int64_t xb = lt.cell[k], xf = lt.cff[k];
    int o = 0;
    CT w = 0;
    unroll<L::Q>([&](auto I) {
        if ((int)I == i) {
            o = opp<L>(I);
            w = (CT)weight<L>(I);
        }
    });
    auto ld = [&](int d, int64_t cell) -> CT { return Store<ST>::ld(A + pidx<L::Q>(d, sidx<ST>(p, cell))); };
    const CT q = lt.q[k];
    const CT a = ld(o, xb);
    CT r;
    if (!(kind & 1)) {
        const CT b = natural ? ld(i, xb) : ld(o, xf);
        if (!(kind & 2)) {
            r = (CT)2 * q * a + ((CT)1 - (CT)2 * q) * b;
        } else {
            const int64_t x3 = lt.cfff[k];
            const CT c = natural ? ld(i, xf) : ld(o, x3);
            r = q * ((CT)1 + (CT)2 * q) * a + ((CT)1 - (CT)4 * q * q) * b - q * ((CT)1 - (CT)2 * q) * c;
        }
    } else {
        const CT d = natural ? ld(o, xf) : ld(i, xb);
        if (!(kind & 2)) {
            r = a / ((CT)2 * q) + ((CT)2 * q - (CT)1) / ((CT)2 * q) * d;
        } else {
            const int64_t x3 = lt.cfff[k];
            const CT e = natural ? ld(o, x3) : ld(i, xf);
            r = a / (q * ((CT)2 * q + (CT)1)) + ((CT)2 * q - (CT)1) / q * d + ((CT)1 - (CT)2 * q) / ((CT)1 + (CT)2 * q) * e;
        }
    }
    Store<ST>::st(A + pidx<L::Q>(o, sidx<ST>(p, xb)), r);
    lt.dlt[k] = Store<ST>::scaled ? (a - r) * w : (a - r);
}

// The curved links' share of the momentum exchange on the solids: over the
// links, (f*_i + f_opp(t+1)) c_i = 2 f_opp(t+1) c_i (what k_forces counts from
// the state) + dlt c_i.  One row of kForceSlots FP64 sums per block (slots
// 0..2, internal axes), wavefront sums then wavefronts in order.
// This launch covers links [l0, ..) (l0 a multiple of 256) and writes its
// rows at rows[0 ..).
template <class L, class CT>
__global__ void __launch_bounds__(256) k_link_forces(const LinkTab<CT> lt, double *__restrict__ rows, int64_t l0) {
    __shared__ double red[3][4];
    const int64_t k = l0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (k < lt.n) {
        const int i = lt.dir[k];
        const double d = (double)lt.dlt[k];
        unroll<L::Q>([&](auto I) {
            if ((int)I == i) {
                v[0] = d * L::c[I][0];
                v[1] = d * L::c[I][1];
                v[2] = d * L::c[I][2];
            }
        });
    }
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    for (int a = 0; a < 3; ++a) {
        double t = v[a];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) red[a][wv] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < kForceSlots) {
        double t = 0.0;
        if (threadIdx.x < 3) {
            const int nw = ((int)blockDim.x + 63) / 64;
            for (int w = 0; w < nw; ++w) t += red[threadIdx.x][w];
        }
        rows[(int64_t)blockIdx.x * kForceSlots + threadIdx.x] = t;
    }
}

template <class L, class ST>
hipError_t bouzidi_t(const Launch &g, const void *links, bool natural) {
    using CT = typename Store<ST>::CT;
    const Params<CT> &p = *static_cast<const Params<CT> *>(g.params);
    const LinkTab<CT> &lt = *static_cast<const LinkTab<CT> *>(links);
    if (lt.n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((lt.n + 255) / 256);
    hipLaunchKernelGGL((k_bouzidi<L, ST>), dim3(nb), dim3(256), 0, g.stream, p, static_cast<ST *>(g.A), lt,
                       natural ? 1 : 0);
    return hipGetLastError();
}

// row blocks [r0, r0 + nr) of 256 links each (nr = 0: all)
template <class L, class ST>
hipError_t link_forces_t(const Launch &g, const void *links, double *rows, int64_t r0, int64_t nr) {
    using CT = typename Store<ST>::CT;
    const LinkTab<CT> &lt = *static_cast<const LinkTab<CT> *>(links);
    const int64_t all = (lt.n + 255) / 256;
    if (nr <= 0) nr = all - r0;
    if (lt.n <= 0 || nr <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_link_forces<L, CT>), dim3((unsigned)nr), dim3(256), 0, g.stream, lt, rows, r0 * 256);
    return hipGetLastError();
}

// Launches for one (lattice, storage) pair; instantiated in kernels_<lat>_<st>.hip.
template <class L, class ST>
hipError_t dispatch_one(const Launch &g, int op, int a0, bool b0, const void *p0, const void *p1, void *q0, void *q1,
                        double *partial, int64_t N) {
    if (op == OP_STEP) return step_t<L, ST>(g, a0, b0);
    if (op == OP_INIT) return init_t<L, ST>(g, p0, p1, a0, N);
    if (op == OP_MOMENTS) return moments_t<L, ST>(g, b0, q0, q1, a0, partial, N);
    // OP_FORCES / OP_LINK_FORCES: N = first block (row) << 32 | count of this launch
    if (op == OP_FORCES) return forces_t<L, ST>(g, partial, N >> 32, N & 0xffffffff);
    if (op == OP_BOUZIDI) return bouzidi_t<L, ST>(g, p0, a0 != 0);
    if (op == OP_LINK_FORCES) return link_forces_t<L, ST>(g, p0, partial, N >> 32, N & 0xffffffff);
    return hipErrorInvalidValue;
}

template <class L>
hipError_t solid_t(const Launch &g, const uint8_t *solid, uint8_t *flags, uint32_t *nbm) {
    const Params<float> &p = *static_cast<const Params<float> *>(g.params);
    hipLaunchKernelGGL(k_solid<L>, dim3(g.grid), dim3(g.block), 0, g.stream, p, solid, flags, nbm);
    return hipGetLastError();
}

}  // namespace lbm
