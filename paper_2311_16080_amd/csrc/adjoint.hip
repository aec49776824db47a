// adjoint.hip -- discrete adjoint of the stream-collide step (gfx950).
//
// The paper obtains gradients of `step` with jax.grad (Sec. 3.6) and trains
// through unrolled steps with checkpointing (Sec. 6.1); here the transpose of
// one step is written out and run as one gather kernel per step.  With
// f(t+1) = Z(G(C(f(t)), f(t))) -- C collision (+ partial bounce-back), G
// streaming with the boundary fills, Z the Zou-He closure -- and
// a(t) = dL/df(t):
//   b_k(x)  = adjoint of the post-collision value f°_k(x): a_k(x + c_k) when
//             x + c_k is fluid, a_opp(k)(x) when it is a wall or solid cell
//             (bounce-back), 0 when it leaves through an open face;
//   PBB     : lambda = (1 - s) b, direct part s b_opp(j), dL/ds += sum b_i (f_opp(i) - f*_i);
//   BGK     : a_j = (1 - w) lambda_j + w (A + c_j . V),
//             A = sum_i lambda_i dfeq_i/drho, V = sum_i lambda_i dfeq_i/dj
//             (feq as a function of rho and j = rho u), dL/dtau += sum lambda (f - feq) / tau^2;
//   outflow : the equilibrium fills depend on u(x, t): a_j += e . (c_j - u) / rho;
//   Zou-He  : the unknowns are affine in the knowns at the same cell, so their
//             adjoints are folded into the knowns' (closure transpose);
//   walls   : dL/du_w += a_i(x) 6 w_i rho0 c_i for populations bounced off a moving wall.
// Per-block FP64 partial sums of dL/dtau and dL/du_w are added into the
// block's own slot (deterministic).
#include "adjoint.hpp"

namespace lbm {

template <class CT>
__device__ __forceinline__ bool adj_block_cell(const Params<CT> &p, int &X, int &Y, int &Z) {
    const int zc = (int)blockIdx.x % p.zblocks;
    const int r = (int)blockIdx.x / p.zblocks;
    Y = r % p.nY;
    X = r / p.nY;
    Z = zc * (int)blockDim.x + (int)threadIdx.x;
    return Z < p.nZ;
}

// Transpose of the Zou-He closure at a face cell: the adjoints of the
// unknowns a_i (i in U) are folded into the knowns; a_i (i in U) become 0.
//   velocity face: f_i = f_opp(i) + alpha_i rho - sum_t c_it N_t,
//                  rho = (sum_Z f + 2 sum_O f + rho0 u_n)/(1 - u_n) (deviation form),
//                  N_t = (Z_t - (2/3) rho u_t)/den, Z_t = sum_Z f_j c_jt, alpha_i = 6 w_i c_i.u
//   pressure face: f_i = f_opp(i) + 6 w_i rho_w u_n - sum_t c_it N_t,
//                  u_n = (rho_w - rho0 - sum_Z f - 2 sum_O f)/rho_w, N_t = Z_t/den
template <class L, class CT>
__device__ __forceinline__ void zouhe_transpose(CT *a, const Params<CT> &p, int face) {
    const int ax = face >> 1;
    const int sg = (face & 1) ? -1 : 1;
    int cn[L::Q];
    unroll<L::Q>([&](auto I) {
        const int ca = (ax == 0) ? L::c[I][0] : ((ax == 1) ? L::c[I][1] : L::c[I][2]);
        cn[I] = sg * ca;
    });
    const FaceTab<CT> &F = *p.ft;
    const bool vel = F.type[face] == F_ZH_VEL;
    CT u[3] = {0, 0, 0};
    CT un = 0;
    if (vel) {
        u[0] = F.uw[face][0];
        u[1] = F.uw[face][1];
        u[2] = F.uw[face][2];
        un = (CT)sg * ((ax == 0) ? u[0] : ((ax == 1) ? u[1] : u[2]));
    }
    const CT rhow = F.rho[face];
    // adjoints of the intermediate linear functionals
    CT g_scalar = 0;              // of rho (velocity face) or u_n (pressure face)
    CT g_t[3] = {0, 0, 0};        // of Z_t
    unroll<L::Q>([&](auto I) {
        const bool unk = cn[I] == 1;
        const CT ai = unk ? a[I] : (CT)0;
        if (vel) {
            const CT cu = (CT)L::c[I][0] * u[0] + (CT)L::c[I][1] * u[1] + (CT)L::c[I][2] * u[2];
            g_scalar += ai * (CT)(6.0 * weight<L>(I)) * cu;
        } else {
            g_scalar += ai * (CT)(6.0 * weight<L>(I)) * rhow;
        }
        unroll<3>([&](auto T) {
            if constexpr (L::c[I][T] != 0) g_t[T] -= ai * (CT)L::c[I][T] * (CT)(1.0 / L::den_t);
        });
    });
    unroll<3>([&](auto T) {
        if (T == ax) g_t[T] = 0;  // no normal-axis term
    });
    if (vel) {
        // N_t also depends on rho through -(2/3) rho u_t / den
        unroll<3>([&](auto T) { g_scalar += g_t[T] * (CT)(-2.0 / 3.0) * u[T]; });
    }
    // d(rho)/d(f_j) or d(u_n)/d(f_j) per known set: Z -> 1, O -> 2 (times the factor)
    const CT fac = vel ? (CT)1 / ((CT)1 - un) : (CT)(-1) / rhow;
    CT add[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        CT v = a[I];
        // direct term f_opp(unknown) : the unknown i = O of this known I
        if (cn[I] == -1) v += a[O];
        if (cn[I] == 0 || cn[I] == -1) v += g_scalar * fac * (CT)((cn[I] == 0) ? 1 : 2);
        if (cn[I] == 0) {
            unroll<3>([&](auto T) {
                if constexpr (L::c[I][T] != 0) v += g_t[T] * (CT)L::c[I][T];
            });
        }
        add[I] = v;
    });
    unroll<L::Q>([&](auto I) { a[I] = (cn[I] == 1) ? (CT)0 : add[I]; });
}

// Adjoint step at time t.  F: natural state f(t) (storage type ST); An: a(t+1)
// (CT planes); Ao: a(t).  ds: per-cell dL/ds accumulator (null without s).
// acc: per-block accumulator rows of kAdjSlots doubles (dL/dtau, dL/du_w[6][3]).
template <class L, class ST>
__device__ __forceinline__ void adjoint_cell(const Params<typename Store<ST>::CT> &p, const ST *__restrict__ F,
                                             const typename Store<ST>::CT *__restrict__ An,
                                             typename Store<ST>::CT *__restrict__ Ao,
                                             typename Store<ST>::CT *__restrict__ ds, int X, int Y, int Z,
                                             int pending, double inv_tau2, double (&part)[kAdjSlots]) {
    using CT = typename Store<ST>::CT;
    constexpr int Q = L::Q;
    const int64_t P = p.plane;
    {
        const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
        uint32_t nbm = 0;
        bool solid = false;
        if (p.flags) {
            const uint8_t fl = p.flags[cell];
            solid = fl & 1;
            if (fl & 2) nbm = p.nbm[cell];
        }
        if (solid) {
            unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = (CT)0; });
        } else {
            const uint32_t e = edge_bits(p, X, Y, Z);
            const uint32_t irr = irregular_mask<L>(e, nbm);
            const bool perim = (e & p.wallmask) != 0;
            CT h[Q];
            unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I>(F, P, cell); });
            const int zf = zh_face_of(p, e);
            if (zf >= 0 && pending) zouhe<L>(h, p, zf);
            // forward quantities
            CT drho = 0, jx = 0, jy = 0, jz = 0;
            unroll<Q>([&](auto I) {
                drho += h[I];
                if constexpr (L::c[I][0] != 0) jx += (CT)L::c[I][0] * h[I];
                if constexpr (L::c[I][1] != 0) jy += (CT)L::c[I][1] * h[I];
                if constexpr (L::c[I][2] != 0) jz += (CT)L::c[I][2] * h[I];
            });
            const CT rho = p.rho0 + drho;
            const CT inv = (CT)1 / rho;
            const CT ux = jx * inv, uy = jy * inv, uz = jz * inv;
            const CT usq15 = (CT)1.5 * (ux * ux + uy * uy + uz * uz);
            const CT om = p.omega;
            CT neq[Q];  // f - feq
            unroll<Q>([&](auto I) { neq[I] = h[I] - heq<L, I>(drho, rho, ux, uy, uz, usq15); });

            // b_k: adjoint of the post-collision value f°_k(x)
            CT b[Q];
            CT ex = 0, ey = 0, ez = 0;  // adjoint of u(x, t) through equilibrium fills
            unroll<Q>([&](auto K) {
                constexpr int O = opp<L>(K);
                if (!((irr >> O) & 1u)) {
                    const int64_t dst = cell + ((int64_t)L::c[K][0] * p.sX + (int64_t)L::c[K][1] * p.sY + L::c[K][2]);
                    b[K] = An[(int64_t)K * P + dst];
                } else {
                    const Nb nb = classify_src<L>(p, X, Y, Z, O, nbm);  // the cell x + c_k
                    if (nb.kind == NB_FLUID) b[K] = An[(int64_t)K * P + nb.cell];
                    else if (nb.kind == NB_WALL) b[K] = An[(int64_t)O * P + cell];
                    else b[K] = (CT)0;
                }
                // incoming population K at x from a non-fluid source: wall velocity /
                // equilibrium-fill dependencies
                if ((irr >> K) & 1u) {
                    const Nb ns = classify_src<L>(p, X, Y, Z, K, nbm);
                    if (ns.kind != NB_FLUID) {
                        const CT aK = An[(int64_t)K * P + cell];
                        const FaceTab<CT> &FT = *p.ft;
                        if (ns.kind == NB_WALL && ns.face >= 0) {
                            const double g = (double)aK * 6.0 * weight<L>(K) * (double)p.rho0;
                            unroll<3>([&](auto A3) {
                                if constexpr (L::c[K][A3] != 0) {
                                    const double v = g * (double)L::c[K][A3];
                                    // slot 1 + face*3 + axis (internal axes)
                                    for (int f = 0; f < 6; ++f)
                                        if (ns.face == f) part[1 + f * 3 + A3] += v;
                                }
                            });
                        } else if (ns.kind == NB_OUT ||
                                   (ns.kind == NB_ZH && perim && FT.type[ns.face] == F_ZH_PRES)) {
                            const CT rf = FT.rho[ns.face];
                            const CT cu = (CT)L::c[K][0] * ux + (CT)L::c[K][1] * uy + (CT)L::c[K][2] * uz;
                            const CT g = aK * (CT)weight<L>(K) * rf;
                            ex += g * ((CT)3 * (CT)L::c[K][0] + (CT)9 * cu * (CT)L::c[K][0] - (CT)3 * ux);
                            ey += g * ((CT)3 * (CT)L::c[K][1] + (CT)9 * cu * (CT)L::c[K][1] - (CT)3 * uy);
                            ez += g * ((CT)3 * (CT)L::c[K][2] + (CT)9 * cu * (CT)L::c[K][2] - (CT)3 * uz);
                        }
                    }
                }
            });

            CT s = 0;
            const bool has_s = p.s != nullptr;
            if (has_s) s = (CT)p.s[cell];
            CT lam[Q];
            unroll<Q>([&](auto I) { lam[I] = has_s ? ((CT)1 - s) * b[I] : b[I]; });
            if (has_s && ds) {
                CT g = 0;
                unroll<Q>([&](auto I) {
                    constexpr int O = opp<L>(I);
                    const CT fstar = h[I] - om * neq[I];
                    g += b[I] * (h[O] - fstar);
                });
                ds[cell] += g;
            }
            // dL/dtau: d f*_i / d tau = (f_i - feq_i) / tau^2
            {
                CT g = 0;
                unroll<Q>([&](auto I) { g += lam[I] * neq[I]; });
                part[0] += (double)g * inv_tau2;
            }
            // A and V
            CT Aa = 0, Vx = 0, Vy = 0, Vz = 0, Sw = 0;
            const CT uu = ux * ux + uy * uy + uz * uz;
            unroll<Q>([&](auto I) {
                const CT cu = (CT)L::c[I][0] * ux + (CT)L::c[I][1] * uy + (CT)L::c[I][2] * uz;
                const CT wl = (CT)weight<L>(I) * lam[I];
                Aa += wl * ((CT)1 - (CT)4.5 * cu * cu + (CT)1.5 * uu);
                Sw += wl;
                const CT t9 = (CT)3 + (CT)9 * cu;
                if constexpr (L::c[I][0] != 0) Vx += wl * t9 * (CT)L::c[I][0];
                if constexpr (L::c[I][1] != 0) Vy += wl * t9 * (CT)L::c[I][1];
                if constexpr (L::c[I][2] != 0) Vz += wl * t9 * (CT)L::c[I][2];
            });
            Vx -= (CT)3 * ux * Sw;
            Vy -= (CT)3 * uy * Sw;
            Vz -= (CT)3 * uz * Sw;
            const CT eu = ex * ux + ey * uy + ez * uz;
            CT a[Q];
            unroll<Q>([&](auto J) {
                constexpr int O = opp<L>(J);
                const CT cV = (CT)L::c[J][0] * Vx + (CT)L::c[J][1] * Vy + (CT)L::c[J][2] * Vz;
                const CT ce = (CT)L::c[J][0] * ex + (CT)L::c[J][1] * ey + (CT)L::c[J][2] * ez;
                CT v = ((CT)1 - om) * lam[J] + om * (Aa + cV) + (ce - eu) * inv;
                if (has_s) v += s * b[O];
                a[J] = v;
            });
            if (zf >= 0 && pending) zouhe_transpose<L>(a, p, zf);
            unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = a[I]; });
        }
    }
}

// block partial sums -> the block's own accumulator row
__device__ __forceinline__ void adj_block_reduce(const double (&part)[kAdjSlots], double *acc, int64_t row) {
    __shared__ double red[kAdjSlots][kMaxBlock / 64];
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kAdjSlots; ++k) {
        double v = part[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = ((int)blockDim.x + 63) / 64;
        for (int k = 0; k < kAdjSlots; ++k) {
            double v = 0.0;
            for (int w = 0; w < nw; ++w) v += red[k][w];
            acc[row * kAdjSlots + k] += v;
        }
    }
}

template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_adjoint(const Params<typename Store<ST>::CT> p, const ST *__restrict__ F,
                                                       const typename Store<ST>::CT *__restrict__ An,
                                                       typename Store<ST>::CT *__restrict__ Ao,
                                                       typename Store<ST>::CT *__restrict__ ds, double *__restrict__ acc,
                                                       double inv_tau2) {
    int X, Y, Z;
    const bool inside = adj_block_cell(p, X, Y, Z);
    double part[kAdjSlots];
#pragma unroll
    for (int k = 0; k < kAdjSlots; ++k) part[k] = 0.0;
    if (inside) adjoint_cell<L, ST>(p, F, An, Ao, ds, X, Y, Z, p.zh_pending, inv_tau2, part);
    adj_block_reduce(part, acc, blockIdx.x);
}

// a(n) = dL/df(n) from dL/drho, dL/du of the final moments (caller axes), with
// the Zou-He closure transpose on face cells.  IT = float or double.
// gcell / N: the cell's index in, and the length of, the caller's fields
template <class L, class ST, class IT>
__device__ __forceinline__ void seed_cell(const Params<typename Store<ST>::CT> &p, const ST *__restrict__ F,
                                          const IT *__restrict__ grho, const IT *__restrict__ gu,
                                          typename Store<ST>::CT *__restrict__ Ao, int X, int Y, int Z, int pending,
                                          int64_t gcell, int64_t N) {
    using CT = typename Store<ST>::CT;
    constexpr int Q = L::Q;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    const int64_t P = p.plane;
    if (p.flags && (p.flags[cell] & 1)) {
        unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = (CT)0; });
        return;
    }
    const uint32_t e = edge_bits(p, X, Y, Z);
    CT h[Q];
    unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I>(F, P, cell); });
    const int zf = zh_face_of(p, e);
    if (zf >= 0 && pending) zouhe<L>(h, p, zf);
    CT drho = 0, jx = 0, jy = 0, jz = 0;
    unroll<Q>([&](auto I) {
        drho += h[I];
        if constexpr (L::c[I][0] != 0) jx += (CT)L::c[I][0] * h[I];
        if constexpr (L::c[I][1] != 0) jy += (CT)L::c[I][1] * h[I];
        if constexpr (L::c[I][2] != 0) jz += (CT)L::c[I][2] * h[I];
    });
    const CT rho = p.rho0 + drho;
    const CT inv = (CT)1 / rho;
    const CT ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const CT gr = grho ? (CT)grho[gcell] : (CT)0;
    CT gx = 0, gy = 0, gz = 0;
    if (gu) {
        if constexpr (L::D == 2) {
            gy = (CT)gu[gcell];
            gz = (CT)gu[N + gcell];
        } else {
            gx = (CT)gu[gcell];
            gy = (CT)gu[N + gcell];
            gz = (CT)gu[2 * N + gcell];
        }
    }
    const CT gdotu = gx * ux + gy * uy + gz * uz;
    CT a[Q];
    unroll<Q>([&](auto I) {
        const CT gc = (CT)L::c[I][0] * gx + (CT)L::c[I][1] * gy + (CT)L::c[I][2] * gz;
        a[I] = gr + (gc - gdotu) * inv;
    });
    if (zf >= 0 && pending) zouhe_transpose<L>(a, p, zf);
    unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = a[I]; });
}

template <class L, class ST, class IT>
__global__ void __launch_bounds__(kMaxBlock) k_seed(const Params<typename Store<ST>::CT> p, const ST *__restrict__ F,
                                                    const IT *__restrict__ grho, const IT *__restrict__ gu,
                                                    typename Store<ST>::CT *__restrict__ Ao, int64_t N) {
    int X, Y, Z;
    if (!adj_block_cell(p, X, Y, Z)) return;
    seed_cell<L, ST, IT>(p, F, grho, gu, Ao, X, Y, Z, p.zh_pending, ((int64_t)X * p.nY + Y) * p.nZ + Z, N);
}

// Natural-order copy of the current in-place state: after an even step the
// AA buffer holds post-collision values in swapped slots; gather them as the
// odd step would (boundary slots from the cell itself), no closure.
template <class L, class ST>
__device__ __forceinline__ void materialize_cell(const Params<typename Store<ST>::CT> &p, const ST *__restrict__ A,
                                                 ST *__restrict__ D, int X, int Y, int Z) {
    constexpr int Q = L::Q;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    const int64_t P = p.plane;
    uint32_t nbm = 0;
    if (p.flags) {
        const uint8_t fl = p.flags[cell];
        if (fl & 1) return;
        if (fl & 2) nbm = p.nbm[cell];
    }
    const uint32_t e = edge_bits(p, X, Y, Z);
    const uint32_t irr = irregular_mask<L>(e, nbm);
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        ST v;
        if (!((irr >> I) & 1u)) {
            const int64_t src = cell - ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]);
            v = A[(int64_t)O * P + src];
        } else {
            const Nb nb = classify_src<L>(p, X, Y, Z, I, nbm);
            v = (nb.kind == NB_FLUID) ? A[(int64_t)O * P + nb.cell] : A[(int64_t)I * P + cell];
        }
        D[(int64_t)I * P + cell] = v;  // opposite slots share the storage scale
    });
}

template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_materialize(const Params<typename Store<ST>::CT> p,
                                                           const ST *__restrict__ A, ST *__restrict__ D) {
    int X, Y, Z;
    if (!adj_block_cell(p, X, Y, Z)) return;
    materialize_cell<L, ST>(p, A, D, X, Y, Z);
}

// acc rows [0, rows) summed in a fixed order into out[kAdjSlots]
__global__ void __launch_bounds__(256) k_adj_reduce(const double *__restrict__ acc, int64_t rows,
                                                    double *__restrict__ out) {
    __shared__ double red[256];
    const int k = (int)blockIdx.x;  // slot
    double v = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) v += acc[r * kAdjSlots + k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

template <class CT>
__global__ void __launch_bounds__(256) k_to_float(const CT *__restrict__ src, float *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// ---- batch variants ------------------------------------------------------------
template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_adjoint_batch(const BatchDev b, const ST *__restrict__ F,
                                                             const typename Store<ST>::CT *__restrict__ An,
                                                             typename Store<ST>::CT *__restrict__ Ao,
                                                             double *__restrict__ acc,
                                                             const double *__restrict__ inv_tau2, int pending) {
    using CT = typename Store<ST>::CT;
    const int tile = (int)blockIdx.x;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    double part[kAdjSlots];
#pragma unroll
    for (int k = 0; k < kAdjSlots; ++k) part[k] = 0.0;
    if (c < p.nX * p.nY * p.nZ) {
        int X, Y, Z;
        split_cell(c, p.nY, p.nZ, X, Y, Z);
        const int64_t o = b.stoff[d];
        adjoint_cell<L, ST>(p, F + o, An + o, Ao + o, nullptr, X, Y, Z, pending, inv_tau2[d], part);
    }
    adj_block_reduce(part, acc, tile);
}

template <class L, class ST, class IT>
__global__ void __launch_bounds__(kMaxBlock) k_seed_batch(const BatchDev b, const ST *__restrict__ F,
                                                          const IT *__restrict__ grho, const IT *__restrict__ gu,
                                                          typename Store<ST>::CT *__restrict__ Ao, int pending) {
    using CT = typename Store<ST>::CT;
    const int tile = (int)blockIdx.x;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    if (c >= p.nX * p.nY * p.nZ) return;
    int X, Y, Z;
    split_cell(c, p.nY, p.nZ, X, Y, Z);
    const int64_t o = b.stoff[d];
    seed_cell<L, ST, IT>(p, F + o, grho, gu, Ao + o, X, Y, Z, pending, b.cell0[d] + c, b.ncells);
}

template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_materialize_batch(const BatchDev b, const ST *__restrict__ A,
                                                                 ST *__restrict__ D) {
    using CT = typename Store<ST>::CT;
    const int tile = (int)blockIdx.x;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    if (c >= p.nX * p.nY * p.nZ) return;
    int X, Y, Z;
    split_cell(c, p.nY, p.nZ, X, Y, Z);
    const int64_t o = b.stoff[d];
    materialize_cell<L, ST>(p, A + o, D + o, X, Y, Z);
}

// one workgroup per domain; rows summed by a fixed thread/row assignment and
// a fixed tree, so the result is deterministic
__global__ void __launch_bounds__(256) k_adj_reduce_batch(const double *__restrict__ acc,
                                                          const int64_t *__restrict__ rbeg,
                                                          const int64_t *__restrict__ rend, double *__restrict__ out) {
    __shared__ double red[256];
    const int d = (int)blockIdx.x;
    const int64_t r0 = rbeg[d], r1 = rend[d];
    for (int k = 0; k < kAdjSlots; ++k) {
        double v = 0.0;
        for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) v += acc[r * kAdjSlots + k];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[(int64_t)d * kAdjSlots + k] = red[0];
        __syncthreads();
    }
}

template <class L, class ST>
static hipError_t adj_batch_dispatch(const BatchAdjLaunch &g) {
    using CT = typename Store<ST>::CT;
    const dim3 grid(g.grid), block(g.block);
    switch (g.op) {
        case ADJ_STEP:
            hipLaunchKernelGGL((k_adjoint_batch<L, ST>), grid, block, 0, g.stream, g.b, static_cast<const ST *>(g.F),
                               static_cast<const CT *>(g.An), static_cast<CT *>(g.Ao), g.acc, g.inv_tau2, g.pending);
            break;
        case ADJ_SEED:
            if (g.in_f64)
                hipLaunchKernelGGL((k_seed_batch<L, ST, double>), grid, block, 0, g.stream, g.b,
                                   static_cast<const ST *>(g.F), static_cast<const double *>(g.grho),
                                   static_cast<const double *>(g.gu), static_cast<CT *>(g.Ao), g.pending);
            else
                hipLaunchKernelGGL((k_seed_batch<L, ST, float>), grid, block, 0, g.stream, g.b,
                                   static_cast<const ST *>(g.F), static_cast<const float *>(g.grho),
                                   static_cast<const float *>(g.gu), static_cast<CT *>(g.Ao), g.pending);
            break;
        case ADJ_MATERIALIZE:
            hipLaunchKernelGGL((k_materialize_batch<L, ST>), grid, block, 0, g.stream, g.b,
                               static_cast<const ST *>(g.F), static_cast<ST *>(g.D));
            break;
        case ADJ_REDUCE:
            hipLaunchKernelGGL(k_adj_reduce_batch, dim3(g.b.ndom), dim3(256), 0, g.stream, g.acc, g.rbeg, g.rend,
                               g.out);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class L>
static hipError_t adj_batch_storage(const BatchAdjLaunch &g) {
    switch (g.storage) {
        case ST_F64: return adj_batch_dispatch<L, double>(g);
        case ST_F32: return adj_batch_dispatch<L, float>(g);
        case ST_F16: return adj_batch_dispatch<L, _Float16>(g);
        case ST_BF16: return adj_batch_dispatch<L, bf16_t>(g);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_batch(const BatchAdjLaunch &g) {
    switch (g.lattice) {
        case LAT_D2Q9: return adj_batch_storage<D2Q9>(g);
        case LAT_D3Q19: return adj_batch_storage<D3Q19>(g);
        case LAT_D3Q27: return adj_batch_storage<D3Q27>(g);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
template <class L, class ST>
static hipError_t adj_dispatch(const AdjLaunch &g) {
    using CT = typename Store<ST>::CT;
    const Params<CT> &p = *static_cast<const Params<CT> *>(g.params);
    const dim3 grid(g.grid), block(g.block);
    switch (g.op) {
        case ADJ_STEP:
            hipLaunchKernelGGL((k_adjoint<L, ST>), grid, block, 0, g.stream, p, static_cast<const ST *>(g.F),
                               static_cast<const CT *>(g.An), static_cast<CT *>(g.Ao), static_cast<CT *>(g.ds), g.acc,
                               g.inv_tau2);
            break;
        case ADJ_SEED:
            if (g.in_f64)
                hipLaunchKernelGGL((k_seed<L, ST, double>), grid, block, 0, g.stream, p, static_cast<const ST *>(g.F),
                                   static_cast<const double *>(g.grho), static_cast<const double *>(g.gu),
                                   static_cast<CT *>(g.Ao), g.N);
            else
                hipLaunchKernelGGL((k_seed<L, ST, float>), grid, block, 0, g.stream, p, static_cast<const ST *>(g.F),
                                   static_cast<const float *>(g.grho), static_cast<const float *>(g.gu),
                                   static_cast<CT *>(g.Ao), g.N);
            break;
        case ADJ_MATERIALIZE:
            hipLaunchKernelGGL((k_materialize<L, ST>), grid, block, 0, g.stream, p, static_cast<const ST *>(g.F),
                               static_cast<ST *>(g.D));
            break;
        case ADJ_DS_OUT: {
            const unsigned nb = (unsigned)((g.N + 255) / 256);
            hipLaunchKernelGGL((k_to_float<CT>), dim3(nb), dim3(256), 0, g.stream, static_cast<const CT *>(g.ds),
                               g.ds_out, g.N);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class L>
static hipError_t adj_storage(const AdjLaunch &g) {
    switch (g.storage) {
        case ST_F64: return adj_dispatch<L, double>(g);
        case ST_F32: return adj_dispatch<L, float>(g);
        case ST_F16: return adj_dispatch<L, _Float16>(g);
        case ST_BF16: return adj_dispatch<L, bf16_t>(g);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(const AdjLaunch &g) {
    switch (g.lattice) {
        case LAT_D2Q9: return adj_storage<D2Q9>(g);
        case LAT_D3Q19: return adj_storage<D3Q19>(g);
        case LAT_D3Q27: return adj_storage<D3Q27>(g);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_adj_reduce(const double *acc, int64_t rows, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_reduce, dim3(kAdjSlots), dim3(256), 0, s, acc, rows, out);
    return hipGetLastError();
}

}  // namespace lbm
