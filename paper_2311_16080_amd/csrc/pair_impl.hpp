// pair_impl.hpp -- in-place step for 2-byte storage (FP16 / BF16) with two
// cells per lane.
//
// With one cell per lane a 2-byte population moves 128 B per wavefront
// instruction, and the kernel runs out of memory instructions long before it
// runs out of bandwidth.  Here lane t of a Z row owns the cell pair
// (z0, z0 + 1) = (2t, 2t + 1): every population plane of the local even step
// is read and written as aligned 32-bit pairs.  In the odd step the Z-shifted
// planes are read and written as 32-bit pairs at 2-byte-aligned addresses; a
// pair that would leave the row (Z wall) or straddle a 4096-cell tile goes
// through 16-bit accesses.  Rows of nZ % 128 == 0 cells only, so no wavefront
// straddles two rows: lane 0 of a row's first wavefront holds z = 0, lane 63
// of its last wavefront holds z = nZ - 1.
//
// Wavefronts whose cells meet only wall faces take this path; anything else
// (solid cells, periodic / open faces) runs step_cell once per cell of the
// pair.  Per cell the arithmetic is step_cell's (same collide, same rounding
// to storage), so both paths give bitwise-equal states.
//
// Measured on the D3Q19 FP16 256^3 cavity: the even (local) step drops from
// 305 to 224 us (202 us for the variant without the per-cell fallback that
// walls-only domains without solids use).  For the odd step two cells per lane
// measured slower than one: 330 us with the 2-byte-aligned 32-bit accesses
// (a plain copy at a 2-byte offset runs 8% below an aligned one, and the
// odd-step pattern with 10 of 19 planes at that offset 28% below), 400-590 us
// with wavefront-wide DPP shifts (~134 VGPRs), ~400 us with the Z-shifted planes
// staged through LDS behind block barriers, against 290 us with one cell per
// lane; so by default only even steps use this kernel (LBM_PAIR=2 selects it
// for odd steps too, for measurement).
#pragma once

namespace lbm {

template <class ST>
struct HalfBits;
template <>
struct HalfBits<_Float16> {
    __device__ static float val(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)b); }
    __device__ static uint32_t bits(float v) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v); }
};
template <>
struct HalfBits<bf16_t> {
    __device__ static float val(uint32_t b) { return __uint_as_float((b & 0xffffu) << 16); }
    __device__ static uint32_t bits(float v) { return (uint32_t)Store<bf16_t>::round(v); }
};

// population value of direction I (storage scale undone) from 16 stored bits
template <class L, class ST, int I>
__device__ __forceinline__ float hval(uint32_t b) {
    return HalfBits<ST>::val(b) * (float)weight<L>(I);
}
template <class L, class ST, int I>
__device__ __forceinline__ uint32_t hbits(float v) {
    return HalfBits<ST>::bits(v * (float)(1.0 / weight<L>(I)));
}

template <bool NT>
__device__ __forceinline__ uint32_t ld32(const uint32_t *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st32(uint32_t *p, uint32_t v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// 32-bit access at a 2-byte-aligned address: gfx9 runs global memory in
// unaligned mode, and the compiler emits one dword access for it
typedef uint32_t u32_a2 __attribute__((aligned(2)));
__device__ __forceinline__ uint32_t ld32u(const uint16_t *p) { return *reinterpret_cast<const u32_a2 *>(p); }
__device__ __forceinline__ void st32u(uint16_t *p, uint32_t v) { *reinterpret_cast<u32_a2 *>(p) = v; }

// The Z-shifted pair of source row rs that the pair (z0, z0 + 1) reads in the
// odd step -- (z0 - 1, z0) for c_z = 1, (z0 + 1, z0 + 2) for c_z = -1 -- leaves
// the row (Z wall) or straddles a tile boundary, so it is not one 32-bit access
template <int CZ>
__device__ __forceinline__ bool src_pair_edge(const Params<float> &p, int64_t rs, int z0) {
    if constexpr (CZ == 1) return z0 == 0 || ((rs + z0) & (kTile - 1)) == 0;
    else return z0 + 2 == p.nZ || ((rs + z0 + 2) & (kTile - 1)) == 0;
}
// the same for the pair of destination row rd that the odd step writes:
// (z0 + 1, z0 + 2) for c_z = 1, (z0 - 1, z0) for c_z = -1
template <int CZ>
__device__ __forceinline__ bool dst_pair_edge(const Params<float> &p, int64_t rd, int z0) {
    if constexpr (CZ == 1) return z0 + 2 == p.nZ || ((rd + z0 + 2) & (kTile - 1)) == 0;
    else return z0 == 0 || ((rd + z0) & (kTile - 1)) == 0;
}

// moving-wall term of the population bounced into slot O (= opp(I)) of a
// cell whose destination x + c_i lies across the faces cr (static walls win)
template <class L, int O>
__device__ __forceinline__ float wall_term(const Params<float> &p, uint32_t cr, float hpi) {
    if (cr && !(cr & p.staticmask)) {
        const int f = (int)__builtin_ctz(cr);
        const FaceTab<float> &F = *p.ft;
        const float cu = (float)L::c[O][0] * F.uw[f][0] + (float)L::c[O][1] * F.uw[f][1] + (float)L::c[O][2] * F.uw[f][2];
        return hpi + (float)(6.0 * weight<L>(O)) * p.rho0 * cu;
    }
    return hpi;
}

// NOFB: the domain has no solid cells and walls on every lattice face (the host
// checks), so the per-cell fallback is never needed and is left out -- it
// would otherwise set the kernel's register allocation (109 vs 64 VGPRs for
// the D3Q19 FP16 even step).
template <class L, class ST, int MODE, bool HAS_S, bool NOFB = false>
__device__ __forceinline__ void step_pair(const Params<float> &p, ST *__restrict__ A, ST *__restrict__ B, int X,
                                          int Y, int z0, int pending) {
    constexpr int Q = L::Q;
    constexpr uint32_t kFaces = all_face_bits<L>();
    constexpr uint32_t kXY = 0xFu;  // faces of the X and Y axes
    const int64_t row = ((int64_t)X * p.nY + Y) * p.nZ;
    const int64_t cell0 = row + z0;
    bool plain = true;
    if (p.flags) plain = (p.flags[cell0] | p.flags[cell0 + 1]) == 0;
    const uint32_t e0 = edge_bits(p, X, Y, z0);
    const uint32_t e1 = edge_bits(p, X, Y, z0 + 1);
    // walls, and in the local even step periodic faces too (no neighbour addresses)
    const uint32_t sel_faces = p.wallmask | (MODE == 0 ? p.permask : 0u);
    if (!NOFB && !__all(plain && ((e0 | e1) & kFaces & ~sel_faces) == 0)) {
        // (the even step's select path takes periodic faces too)
        constexpr int XF = (HAS_S ? 1 : 0) | (MODE == 0 ? 4 : 0);
        step_cell<L, ST, MODE, XF, 1>(p, A, B, X, Y, z0, pending);
        step_cell<L, ST, MODE, XF, 1>(p, A, B, X, Y, z0 + 1, pending);
        return;
    }
    uint32_t *W = reinterpret_cast<uint32_t *>(A);            // pairs: element index / 2
    uint16_t *H = reinterpret_cast<uint16_t *>(A);
    // the pull step (MODE 3) gathers from A like the odd step and stores the
    // cell's own opposite slots into B like the even step
    uint32_t *WO = reinterpret_cast<uint32_t *>(MODE == 3 ? B : A);
    const uint32_t exy = e0 & kXY;                              // X / Y faces: the same for the whole row
    // ---- read: pairs of h_i(z0), h_i(z0 + 1) -------------------------------------
    uint32_t u[Q];
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        constexpr int cz = L::c[I][2];
        if constexpr (MODE == 0) {
            u[I] = ld32<true>(W + (pidx<Q>(I, cell0) >> 1));
        } else {
            // Addresses are selected, not branched on, so the loads of all
            // directions stay in flight together.  A source row across an X / Y
            // wall means both cells bounce back (own slot I).  Z-shifted planes are
            // read as one 32-bit access at a 2-byte-aligned address (elements
            // z0 - 1, z0 for c_z = 1; z0 + 1, z0 + 2 for c_z = -1); a pair that
            // would cross the row's end (Z wall) or a tile boundary is read aligned
            // here and completed below.
            const bool wxy = (exy & src_face_bits<L>(I)) != 0;
            const int64_t rs = row - ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY);
            const int64_t own = pidx<Q>(I, cell0);
            const int64_t src = pidx<Q>(O, rs + z0);
            if constexpr (cz == 0) {
                u[I] = ld32<true>(W + ((wxy ? own : src) >> 1));
            } else {
                const bool edge = src_pair_edge<cz>(p, rs, z0);
                u[I] = ld32u(H + (wxy ? own : (edge ? src : src - cz)));
            }
        }
    });
    if constexpr (MODE != 0) {
        unroll<Q>([&](auto I) {
            constexpr int O = opp<L>(I);
            constexpr int cz = L::c[I][2];
            if constexpr (cz != 0) {
                const bool wxy = (exy & src_face_bits<L>(I)) != 0;
                const int64_t rs = row - ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY);
                if (!wxy && src_pair_edge<cz>(p, rs, z0)) {
                    if constexpr (cz == 1) {
                        // low half: element z0 - 1 (end of the previous tile), or own
                        // slot I at the z = 0 wall
                        const int64_t at = z0 == 0 ? pidx<Q>(I, cell0) : pidx<Q>(O, rs + z0 - 1);
                        u[I] = (u[I] << 16) | (uint32_t)H[at];
                    } else {
                        // high half: element z0 + 2 (start of the next tile), or own
                        // slot I of cell z0 + 1 at the z = nZ - 1 wall
                        const int64_t at = z0 + 2 == p.nZ ? pidx<Q>(I, cell0 + 1) : pidx<Q>(O, rs + z0 + 2);
                        u[I] = (u[I] >> 16) | ((uint32_t)H[at] << 16);
                    }
                }
            }
        });
    }
    // ---- collide the two cells one after the other (step_cell's arithmetic) -------------
    // out[i] packs the value each cell writes for direction i: the post-collision
    // value, or, where x + c_i lies across a wall, the bounced value with the
    // moving-wall term (only the bounce stores below use those).
    uint32_t out[Q];
    {
        float h[Q], hp[Q];
        float r, ux, uy, uz;
        unroll<Q>([&](auto I) { h[I] = hval<L, ST, I>(u[I]); });
        const float s0 = HAS_S ? p.s[cell0] : 0.f;
        collide<L>(h, hp, p, s0, HAS_S, r, ux, uy, uz);
        unroll<Q>([&](auto I) {
            out[I] = hbits<L, ST, I>(wall_term<L, opp<L>(I)>(p, e0 & p.wallmask & src_face_bits<L>(opp<L>(I)), hp[I]));
        });
    }
    {
        float h[Q], hp[Q];
        float r, ux, uy, uz;
        unroll<Q>([&](auto I) { h[I] = hval<L, ST, I>(u[I] >> 16); });
        const float s1 = HAS_S ? p.s[cell0 + 1] : 0.f;
        collide<L>(h, hp, p, s1, HAS_S, r, ux, uy, uz);
        unroll<Q>([&](auto I) {
            out[I] |= hbits<L, ST, I>(wall_term<L, opp<L>(I)>(p, e1 & p.wallmask & src_face_bits<L>(opp<L>(I)), hp[I])) << 16;
        });
    }
    // ---- write ------------------------------------------------------------------------
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        constexpr int cz = L::c[I][2];
        constexpr uint32_t fb = src_face_bits<L>(O);  // faces x + c_i can lie across
        const uint32_t v = out[I];
        if constexpr (MODE == 0 || MODE == 3) {
            st32<true>(WO + (pidx<Q>(O, cell0) >> 1), v);
        } else if (exy & fb) {
            // destination row across an X / Y wall: both values bounce into own slot O
            st32<true>(W + (pidx<Q>(O, cell0) >> 1), v);
        } else {
            const int64_t rd = row + ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY);
            const int64_t dst = pidx<Q>(I, rd + z0);
            if constexpr (cz == 0) {
                st32<true>(W + (dst >> 1), v);
            } else if (!dst_pair_edge<cz>(p, rd, z0)) {
                // one 32-bit store at a 2-byte-aligned address: elements z0 + 1, z0 + 2
                // (c_z = 1) or z0 - 1, z0 (c_z = -1)
                st32u(H + dst + cz, v);
            } else if constexpr (cz == 1) {
                // cell z0's value to element z0 + 1; cell z0 + 1's to element z0 + 2
                // (start of the next tile), or bounced into its own slot O off the
                // z = nZ - 1 wall
                H[dst + 1] = (uint16_t)v;
                H[z0 + 2 == p.nZ ? pidx<Q>(O, cell0 + 1) : pidx<Q>(I, rd + z0 + 2)] = (uint16_t)(v >> 16);
            } else {
                // cell z0 + 1's value to element z0; cell z0's to element z0 - 1 (end of
                // the previous tile), or bounced into its own slot O off the z = 0 wall
                H[dst] = (uint16_t)(v >> 16);
                H[z0 == 0 ? pidx<Q>(O, cell0) : pidx<Q>(I, rd + z0 - 1)] = (uint16_t)v;
            }
        }
    });
}

// one lane per cell pair; grid: rows x (nZ / 2 / blockDim.x)
template <class L, class ST, int MODE, bool HAS_S, bool NOFB = false>
__global__ void __launch_bounds__(kMaxBlock) k_step_pair(const Params<float> p, ST *__restrict__ A,
                                                         ST *__restrict__ B) {
    const int per_row = (p.nZ >> 1) / (int)blockDim.x;
    const int b = (int)blockIdx.x;
    const int r = b / per_row;
    const int z0 = 2 * ((b - r * per_row) * (int)blockDim.x + (int)threadIdx.x);
    step_pair<L, ST, MODE, HAS_S, NOFB>(p, A, B, r / p.nY, r % p.nY, z0, p.zh_pending);
}

}  // namespace lbm

namespace lbm {

// ---- split pairs -----------------------------------------------------------
// 2-byte storage with the box's two X-halves sharing each 32-bit word (core.hpp,
// sidx): lane t owns the pair c' = t, the cell (X', Y, Z) of the low half and
// (X' + nX/2, Y, Z) of the high half.  Every lattice shift moves both cells of a
// pair to the same neighbouring pair, so the step reads and writes aligned
// 32-bit words in every direction -- the Z-shifted ones one word apart, as a
// 4-byte population would be.  Wavefronts whose cells meet only wall faces (and
// in the local steps periodic faces) take this path; any other wavefront
// (solids, open faces) runs step_cell once per cell.  Per cell the arithmetic is
// step_cell's, so both give bitwise-equal states.
//
// The planes X' = 0 and X' = nX/2 - 1 hold an X face in one half and the seam
// in the other.  NOFB (no solid cells, walls on every lattice face; the host
// checks) keeps them on this path: there the directions that cross the X face
// in one half and the seam in the other move each half on its own -- the
// bounced half from or into the cell's own slot, the other half from or into
// the cell across the seam, in the other half -- with 16-bit accesses.
// Without NOFB those planes take the per-cell fallback in gathering steps.
template <class L, class ST, int MODE, bool HAS_S, bool NOFB = false>
__device__ __forceinline__ void step_split(const Params<float> &p, ST *__restrict__ A, ST *__restrict__ B, int Xh,
                                           int Y, int Z, int pending) {
    constexpr int Q = L::Q;
    constexpr uint32_t kFaces = all_face_bits<L>();
    constexpr bool GATHER = (MODE == 1 || MODE == 3);
    const int hx = p.nX >> 1;
    const int64_t c0 = ((int64_t)Xh * p.nY + Y) * p.nZ + Z;   // low-half cell; its pair index
    const uint32_t e0 = edge_bits(p, Xh, Y, Z);
    const uint32_t e1 = edge_bits(p, Xh + hx, Y, Z);
    const bool xlo = Xh == 0, xhi = Xh == hx - 1;              // X' edge planes
    if constexpr (!NOFB) {
        bool plain = true;
        if (p.flags) plain = (p.flags[c0] | p.flags[c0 + p.nh]) == 0;
        const uint32_t sel_faces = p.wallmask | (MODE == 0 ? p.permask : 0u);
        const bool xedge = GATHER && (xlo || xhi);
        if (!__all(plain && !xedge && ((e0 | e1) & kFaces & ~sel_faces) == 0)) {
            constexpr int XF = (HAS_S ? 1 : 0) | (MODE == 0 ? 4 : 0);
            step_cell<L, ST, MODE, XF, 1>(p, A, B, Xh, Y, Z, pending);
            step_cell<L, ST, MODE, XF, 1>(p, A, B, Xh + hx, Y, Z, pending);
            return;
        }
    }
    const uint32_t *WA = reinterpret_cast<const uint32_t *>(A);
    const uint16_t *HA = reinterpret_cast<const uint16_t *>(A);
    uint32_t *WO = reinterpret_cast<uint32_t *>(MODE == 3 ? B : A);
    uint16_t *HO = reinterpret_cast<uint16_t *>(MODE == 3 ? B : A);
    const int64_t s0 = 2 * c0;                     // storage index of the pair's low cell
    const uint32_t eyz = e0 & ~3u;                 // Y / Z faces, the same for both cells
    const int64_t hsx = (int64_t)hx * p.sX;        // pair-index step between the X' edge planes
    // ---- read ---------------------------------------------------------------------
    uint32_t u[Q];
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        constexpr int cx = L::c[I][0], cz = L::c[I][2];
        if constexpr (!GATHER) {
            u[I] = ld32<true>(WA + (pidx<Q>(I, s0) >> 1));
        } else {
            // x - c_i across a Y / Z wall: both cells bounce back (own slot I);
            // across the X face / seam of an edge plane: own slot here, the seam
            // half below
            const bool wall = (eyz & src_face_bits<L>(I)) != 0;
            const bool split = NOFB && ((cx == 1 && xlo) || (cx == -1 && xhi));
            const int64_t off = (int64_t)cx * p.sX + (int64_t)L::c[I][1] * p.sY + cz;
            const int64_t a = (wall || split) ? pidx<Q>(I, s0) : pidx<Q>(O, s0 - 2 * off);
            u[I] = ld32<cz == 0>(WA + (a >> 1));
        }
    });
    if constexpr (NOFB && GATHER) {
        if (__any(xlo || xhi)) {
            unroll<Q>([&](auto I) {
                constexpr int O = opp<L>(I);
                constexpr int cx = L::c[I][0];
                if constexpr (cx != 0) {
                    const bool wall = (eyz & src_face_bits<L>(I)) != 0;
                    const int64_t off = (int64_t)cx * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2];
                    if (!wall && cx == 1 && xlo) {
                        // low cell (X = 0): bounced, own low half; high cell (X = nX/2):
                        // from X = nX/2 - 1, the low half of pair X' = nX/2 - 1
                        const uint32_t v = HA[pidx<Q>(O, 2 * (c0 - off + hsx))];
                        u[I] = (u[I] & 0xffffu) | (v << 16);
                    } else if (!wall && cx == -1 && xhi) {
                        // low cell (X = nX/2 - 1): from X = nX/2, the high half of pair
                        // X' = 0; high cell (X = nX - 1): bounced, own high half
                        const uint32_t v = HA[pidx<Q>(O, 2 * (c0 - off - hsx) + 1)];
                        u[I] = (u[I] & 0xffff0000u) | v;
                    }
                }
            });
        }
    }
    // ---- collide the two cells (step_cell's arithmetic) ------------------------------
    uint32_t out[Q];
    {
        float h[Q], hp[Q];
        float r, ux, uy, uz;
        unroll<Q>([&](auto I) { h[I] = hval<L, ST, I>(u[I]); });
        const float sv = HAS_S ? p.s[c0] : 0.f;
        collide<L>(h, hp, p, sv, HAS_S, r, ux, uy, uz);
        unroll<Q>([&](auto I) {
            out[I] = hbits<L, ST, I>(wall_term<L, opp<L>(I)>(p, e0 & p.wallmask & src_face_bits<L>(opp<L>(I)), hp[I]));
        });
    }
    {
        float h[Q], hp[Q];
        float r, ux, uy, uz;
        unroll<Q>([&](auto I) { h[I] = hval<L, ST, I>(u[I] >> 16); });
        const float sv = HAS_S ? p.s[c0 + p.nh] : 0.f;
        collide<L>(h, hp, p, sv, HAS_S, r, ux, uy, uz);
        unroll<Q>([&](auto I) {
            out[I] |= hbits<L, ST, I>(wall_term<L, opp<L>(I)>(p, e1 & p.wallmask & src_face_bits<L>(opp<L>(I)), hp[I])) << 16;
        });
    }
    // ---- write ----------------------------------------------------------------------
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        constexpr int cx = L::c[I][0], cz = L::c[I][2];
        if constexpr (MODE == 0 || MODE == 3) {
            st32<true>(WO + (pidx<Q>(O, s0) >> 1), out[I]);
        } else {
            // x + c_i across a Y / Z wall: both values bounce into own slot O
            const bool wall = (eyz & src_face_bits<L>(O)) != 0;
            const int64_t off = (int64_t)cx * p.sX + (int64_t)L::c[I][1] * p.sY + cz;
            if (NOFB && !wall && cx == -1 && xlo) {
                // low cell (X = 0) bounces into its own slot O; the high cell (X = nX/2)
                // writes X = nX/2 - 1, the low half of pair X' = nX/2 - 1
                HO[pidx<Q>(O, s0)] = (uint16_t)out[I];
                HO[pidx<Q>(I, 2 * (c0 + off + hsx))] = (uint16_t)(out[I] >> 16);
            } else if (NOFB && !wall && cx == 1 && xhi) {
                // the low cell (X = nX/2 - 1) writes X = nX/2, the high half of pair
                // X' = 0; the high cell (X = nX - 1) bounces into its own slot O
                HO[pidx<Q>(I, 2 * (c0 + off - hsx) + 1)] = (uint16_t)out[I];
                HO[pidx<Q>(O, s0) + 1] = (uint16_t)(out[I] >> 16);
            } else {
                const int64_t a = wall ? pidx<Q>(O, s0) : pidx<Q>(I, s0 + 2 * off);
                st32<cz == 0>(WO + (a >> 1), out[I]);
            }
        }
    });
}

// one lane per pair; grid: ceil(N / 2 / blockDim.x)
template <class L, class ST, int MODE, bool HAS_S, bool NOFB>
__global__ void __launch_bounds__(kMaxBlock) k_step_split(const Params<float> p, ST *__restrict__ A,
                                                          ST *__restrict__ B) {
    const uint32_t c = (uint32_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nz = (uint32_t)p.nZ, ny = (uint32_t)p.nY;
    const uint32_t r = c / nz;
    const int Z = (int)(c - r * nz);
    const int Y = (int)(r % ny);
    const int Xh = (int)(r / ny);
    if (Xh >= (p.nX >> 1)) return;
    step_split<L, ST, MODE, HAS_S, NOFB>(p, A, B, Xh, Y, Z, p.zh_pending);
}

}  // namespace lbm
