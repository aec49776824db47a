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
//   walls   : dL/du_w += a_i(x) 6 w_i rho0 c_i for populations bounced off a moving wall;
//   force   : the exact-difference term G_i = feq_i(rho, (j + F)/rho) - feq_i(rho, j/rho)
//             (inside the (1 - s) factor) adds a_j += A_F + c_j . V_F with
//             A_F = sum lambda_i dG_i/drho, V_F = sum lambda_i dG_i/dj, and
//             dL/dF(x) += sum lambda_i dfeq_i/dm at m = j + F (= V + V_F).
// The step kernel adds the block's FP64 sum of sum_i lambda_i (f_i - feq_i)
// into the block's own accumulator row (times 1/tau^2 on the host); a second,
// small kernel over the cells of the moving-wall faces adds the wall-velocity
// terms into one row of 3 per face tile.  Both are summed on the host in a
// fixed order (deterministic).
#include "adjoint.hpp"

namespace lbm {

template <class CT>
__device__ __forceinline__ bool adj_block_cell(const Params<CT> &p, int &X, int &Y, int &Z) {
    if (p.flat) {
        // consecutive cells of the whole grid (rows not a multiple of 64 cells)
        const uint32_t cell = (uint32_t)blockIdx.x * blockDim.x + threadIdx.x;
        const uint32_t nz = (uint32_t)p.nZ, ny = (uint32_t)p.nY;
        const uint32_t r = cell / nz;
        Z = (int)(cell - r * nz);
        Y = (int)(r % ny);
        X = (int)(r / ny);
        return X < p.nX;
    }
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

// Transpose of the regularized closure at a face cell (the forward is
// regularize() in core.hpp), taken at the cell's pre-closure populations g: the
// adjoints a of every post-closure population become the adjoints of the known
// g_j; those of the unknowns (overwritten) become 0.  Forward, in deviation
// variables:
//   known = sum_Z g + 2 sum_O g;  velocity face: rho = rho0 + (known + rho0 u_n)/(1 - u_n),
//   u = u_w;  pressure face: rho = rho_w, u_n = (rho_w - rho0 - known)/rho_w, u = u_n n;
//   n_i = g_i - heq_i(rho, u) (unknowns: n_opp(i));  P = sum_i c_i c_i n_i;
//   out_i = heq_i + 4.5 w_i (c_i c_i - I/3) : P.
// Reverse: dP from the out_i; dn_i = c_i c_i : dP; unknowns pass dn to their
// opposites; dg_j = dn_j; dheq_i = a_i - dn_i (knowns), a_i (unknowns); then
// rho (velocity) or u_n (pressure) carry sum_i dheq_i dheq_i/d(.) back to the
// knowns with weight 1 (Z) or 2 (O).
template <class L, class CT>
__device__ __forceinline__ void regularize_transpose(CT *a, const Params<CT> &p, int face, const CT *g) {
    constexpr int Q = L::Q;
    const int ax = face >> 1;
    const int sg = (face & 1) ? -1 : 1;
    int cn[Q];
    unroll<Q>([&](auto I) {
        const int ca = (ax == 0) ? L::c[I][0] : ((ax == 1) ? L::c[I][1] : L::c[I][2]);
        cn[I] = sg * ca;
    });
    const FaceTab<CT> &F = *p.ft;
    const bool vel = F.type[face] == F_REG_VEL;
    CT known = 0;
    unroll<Q>([&](auto I) { known += (cn[I] == 0) ? g[I] : ((cn[I] == -1) ? (CT)2 * g[I] : (CT)0); });
    CT rho, u[3], un;
    if (vel) {
        u[0] = F.uw[face][0];
        u[1] = F.uw[face][1];
        u[2] = F.uw[face][2];
        un = (CT)sg * ((ax == 0) ? u[0] : ((ax == 1) ? u[1] : u[2]));
        rho = p.rho0 + (known + p.rho0 * un) / ((CT)1 - un);
    } else {
        rho = F.rho[face];
        un = (rho - p.rho0 - known) / rho;
        u[0] = (ax == 0) ? (CT)sg * un : (CT)0;
        u[1] = (ax == 1) ? (CT)sg * un : (CT)0;
        u[2] = (ax == 2) ? (CT)sg * un : (CT)0;
    }
    const CT uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    // adjoint of the momentum flux P (symmetric; off-diagonal entries once)
    CT d00 = 0, d11 = 0, d22 = 0, d01 = 0, d02 = 0, d12 = 0;
    unroll<Q>([&](auto I) {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        const CT t = (CT)(4.5 * weight<L>(I)) * a[I];
        d00 += t * (CT)((cx != 0 ? 1.0 : 0.0) - 1.0 / 3.0);
        d11 += t * (CT)((cy != 0 ? 1.0 : 0.0) - 1.0 / 3.0);
        d22 += t * (CT)((cz != 0 ? 1.0 : 0.0) - 1.0 / 3.0);
        if constexpr (cx * cy != 0) d01 += t * (CT)(2 * cx * cy);
        if constexpr (cx * cz != 0) d02 += t * (CT)(2 * cx * cz);
        if constexpr (cy * cz != 0) d12 += t * (CT)(2 * cy * cz);
    });
    // adjoint of the non-equilibrium parts n_i (P00 = sum_{c_x != 0} n, P01 = sum c_x c_y n, ...)
    CT dn[Q];
    unroll<Q>([&](auto I) {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        CT v = 0;
        if constexpr (cx != 0) v += d00;
        if constexpr (cy != 0) v += d11;
        if constexpr (cz != 0) v += d22;
        if constexpr (cx * cy != 0) v += (CT)(cx * cy) * d01;
        if constexpr (cx * cz != 0) v += (CT)(cx * cz) * d02;
        if constexpr (cy * cz != 0) v += (CT)(cy * cz) * d12;
        dn[I] = v;
    });
    // unknowns copy their opposite's n
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        if (cn[I] == 1) dn[O] += dn[I];
    });
    // equilibrium: out_i = heq_i + ..., n_i = g_i - heq_i (knowns)
    CT drho = 0, du[3] = {0, 0, 0};
    unroll<Q>([&](auto I) {
        const CT dheq = a[I] - ((cn[I] == 1) ? (CT)0 : dn[I]);
        const CT cu = (CT)L::c[I][0] * u[0] + (CT)L::c[I][1] * u[1] + (CT)L::c[I][2] * u[2];
        drho += dheq * (CT)weight<L>(I) * ((CT)1 + (CT)3 * cu + (CT)4.5 * cu * cu - (CT)1.5 * uu);
        unroll<3>([&](auto A) {
            du[A] += dheq * (CT)weight<L>(I) * rho * ((CT)3 * (CT)L::c[I][A] + (CT)9 * cu * (CT)L::c[I][A] - (CT)3 * u[A]);
        });
    });
    // rho (velocity face) or u_n (pressure face) back to the knowns
    const CT dknown = vel ? drho / ((CT)1 - un) : -(CT)sg * ((ax == 0) ? du[0] : ((ax == 1) ? du[1] : du[2])) / rho;
    unroll<Q>([&](auto I) {
        const CT m = (cn[I] == 0) ? (CT)1 : ((cn[I] == -1) ? (CT)2 : (CT)0);
        a[I] = (cn[I] == 1) ? (CT)0 : dn[I] + m * dknown;
    });
}

// Shear part of direction I in the KBC collision (core.hpp, kbc_relax): the
// deviatoric flux (P_aa - tr P / D) / 2 on the axis directions, c_a c_b P_ab / 4
// on the face diagonals, zero on rest and corners.  sa[a] = (P_aa - tr P / D) / 2,
// sb = {P_xy, P_xz, P_yz} / 4.
template <class L, int I>
__device__ __forceinline__ constexpr bool kbc_has_shear() {
    constexpr int nzc = (L::c[I][0] != 0) + (L::c[I][1] != 0) + (L::c[I][2] != 0);
    return nzc == 1 || nzc == 2;
}

template <class L, int I, class CT>
__device__ __forceinline__ CT kbc_shear_of(const CT *sa, const CT *sb) {
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    constexpr int nzc = (cx != 0) + (cy != 0) + (cz != 0);
    if constexpr (nzc == 1) {
        return sa[(cx != 0) ? 0 : ((cy != 0) ? 1 : 2)];
    } else if constexpr (nzc == 2) {
        constexpr int sgn = (cz == 0) ? cx * cy : ((cy == 0) ? cx * cz : cy * cz);
        const CT v = sb[(cz == 0) ? 0 : ((cy == 0) ? 1 : 2)];
        return (sgn > 0) ? v : -v;
    } else {
        return (CT)0;
    }
}

// Transpose of the KBC collision at one cell.  Forward, in deviation variables
// (e_i = heq_i(rho(h), u(h)), n = h - e, P = sum c c n, s = shear(P),
// dh = n - s, feq = e + w rho0, sh = <s|dh>, hh = <dh|dh> with weights
// 1 / feq, gamma = 1/beta - (2 - 1/beta) sh / hh (2 when hh = 0)):
//   f*_i = h_i - beta (2 s_i + gamma dh_i).
// Given lam_i = dL/df*_i, writes dL/dh_j to a[] by reverse accumulation through
// gamma, sh, hh (and the feq in their weights), s(P), n and the equilibrium's
// rho and u; returns sum_i lam_i df*_i/dtau * tau^2 =
// sum lam s + (sum lam dh) (gamma - (1 + sh / hh) / beta) / 2.
template <class L, class CT>
__device__ __forceinline__ CT kbc_transpose(const CT *h, const CT *lam, CT *a, const Params<CT> &p, CT drho, CT rho,
                                            CT inv, CT ux, CT uy, CT uz, CT usq15) {
    constexpr int Q = L::Q;
    CT e[Q];
    unroll<Q>([&](auto I) { e[I] = heq<L, I>(drho, rho, ux, uy, uz, usq15); });
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
    const CT sa[3] = {(CT)0.5 * (P00 - trD), (CT)0.5 * (P11 - trD), (CT)0.5 * (P22 - trD)};
    const CT sb[3] = {(CT)0.25 * P01, (CT)0.25 * P02, (CT)0.25 * P12};
    auto inv_feq = [&](auto I) -> CT {
        const CT feq = e[I] + (CT)weight<L>(I) * p.rho0;
        if constexpr (sizeof(CT) == 4) return __builtin_amdgcn_rcpf(feq);   // as the forward step
        else return (CT)1 / feq;
    };
    CT sh = 0, hh = 0, A = 0, LS = 0;
    unroll<Q>([&](auto I) {
        const CT v = kbc_shear_of<L, I>(sa, sb);
        const CT dh = (h[I] - e[I]) - v;
        const CT wd = dh * inv_feq(I);
        sh += wd * v;
        hh += wd * dh;
        A += lam[I] * dh;
        LS += lam[I] * v;
    });
    const CT beta = (CT)0.5 * p.omega;
    const CT ib = (CT)1 / beta;
    const bool pos = hh > (CT)0;
    const CT r = pos ? sh / hh : (CT)0;
    const CT gamma = pos ? ib - ((CT)2 - ib) * r : (CT)2;
    const CT gt = LS + (CT)0.5 * A * (gamma - (pos ? ((CT)1 + r) * ib : (CT)0));
    // adjoints of sh and hh through gamma (zero when gamma is the constant 2)
    const CT bsh = pos ? beta * A * ((CT)2 - ib) / hh : (CT)0;
    const CT bhh = -bsh * r;
    const CT bg = -beta * gamma;
    // pass 1: adjoint of P through the shear parts
    CT bP00 = 0, bP11 = 0, bP22 = 0, bP01 = 0, bP02 = 0, bP12 = 0, btr = 0;
    unroll<Q>([&](auto I) {
        if constexpr (kbc_has_shear<L, I>()) {
            constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
            constexpr int nzc = (cx != 0) + (cy != 0) + (cz != 0);
            const CT v = kbc_shear_of<L, I>(sa, sb);
            const CT dh = (h[I] - e[I]) - v;
            const CT iv = inv_feq(I);
            const CT bdh = bg * lam[I] + bsh * v * iv + (CT)2 * bhh * dh * iv;
            const CT bs = (CT)(-2) * beta * lam[I] + bsh * dh * iv - bdh;
            if constexpr (nzc == 1) {
                if constexpr (cx != 0) bP00 += (CT)0.5 * bs;
                if constexpr (cy != 0) bP11 += (CT)0.5 * bs;
                if constexpr (cz != 0) bP22 += (CT)0.5 * bs;
                btr -= (CT)0.5 * bs;
            } else {
                constexpr int sgn = (cz == 0) ? cx * cy : ((cy == 0) ? cx * cz : cy * cz);
                const CT t = (sgn > 0) ? (CT)0.25 * bs : (CT)(-0.25) * bs;
                if constexpr (cz == 0) bP01 += t;
                else if constexpr (cy == 0) bP02 += t;
                else bP12 += t;
            }
        }
    });
    btr *= (CT)(1.0 / L::D);
    bP00 += btr;
    bP11 += btr;
    bP22 += btr;
    // pass 2: adjoint of n and of the equilibrium; the direct terms of h
    CT Ae = 0, Vx = 0, Vy = 0, Vz = 0;
    const CT uu = ux * ux + uy * uy + uz * uz;
    unroll<Q>([&](auto I) {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        const CT v = kbc_shear_of<L, I>(sa, sb);
        const CT dh = (h[I] - e[I]) - v;
        const CT iv = inv_feq(I);
        const CT bdh = bg * lam[I] + bsh * v * iv + (CT)2 * bhh * dh * iv;
        const CT bfeq = -(bsh * v + bhh * dh) * dh * iv * iv;
        CT bn = bdh;
        if constexpr (cx != 0) bn += bP00;
        if constexpr (cy != 0) bn += bP11;
        if constexpr (cz != 0) bn += bP22;
        if constexpr (cx * cy != 0) bn += (cx * cy > 0) ? bP01 : -bP01;
        if constexpr (cx * cz != 0) bn += (cx * cz > 0) ? bP02 : -bP02;
        if constexpr (cy * cz != 0) bn += (cy * cz > 0) ? bP12 : -bP12;
        a[I] = lam[I] + bn;
        const CT be = bfeq - bn;
        const CT cu = cdot<L, I>(ux, uy, uz);
        const CT wb = (CT)weight<L>(I) * be;
        Ae += wb * ((CT)1 + (CT)3 * cu + (CT)4.5 * cu * cu - (CT)1.5 * uu);
        const CT t9 = wb * rho * ((CT)3 + (CT)9 * cu);
        if constexpr (cx != 0) Vx += (cx > 0) ? t9 : -t9;
        if constexpr (cy != 0) Vy += (cy > 0) ? t9 : -t9;
        if constexpr (cz != 0) Vz += (cz > 0) ? t9 : -t9;
        const CT w3 = (CT)3 * wb * rho;
        Vx -= w3 * ux;
        Vy -= w3 * uy;
        Vz -= w3 * uz;
    });
    // pass 3: rho and u of the equilibrium back to every h_j (d rho / d h_j = 1,
    // d u / d h_j = (c_j - u) / rho)
    const CT uV = (ux * Vx + uy * Vy + uz * Vz) * inv;
    unroll<Q>([&](auto J) {
        const CT cV = cdot<L, J>(Vx, Vy, Vz);
        a[J] += Ae - uV + cV * inv;
    });
    return gt;
}

// Adjoint step at time t for one fluid cell.  F: natural state f(t) (storage
// type ST, the forward path's tiled layout); An: a(t+1); Ao: a(t).  The
// adjoint populations are compute-type planes, a_i(x) at i * plane + x: the
// gather over 19 or 27 neighbours then needs one address per cell plus
// per-direction constants, where the tiled index would hold a 64-bit address
// per direction and spill at the register budget the step runs at.  ds: per-cell dL/ds accumulator
// (HAS_S).  FRC: the body force is on; dF (or null): per-cell dL/dF
// accumulators, 3 planes of N (internal axes).  Returns
// sum_i lambda_i (f_i - feq_i), the cell's dL/dtau * tau^2.
// REG: regularized faces may occur (the pre-closure populations are kept for
// the closure's transpose).  KB: the KBC collision (no body force).
template <class L, class ST, bool HAS_S, bool FRC = false, bool REG = false, bool KB = false>
__device__ __forceinline__ typename Store<ST>::CT adjoint_cell(const Params<typename Store<ST>::CT> &p,
                                                               const ST *__restrict__ F,
                                                               const typename Store<ST>::CT *__restrict__ An,
                                                               typename Store<ST>::CT *__restrict__ Ao,
                                                               typename Store<ST>::CT *__restrict__ ds, int X, int Y,
                                                               int Z, int pending,
                                                               typename Store<ST>::CT *__restrict__ dF = nullptr,
                                                               int64_t N = 0) {
    using CT = typename Store<ST>::CT;
    constexpr int Q = L::Q;
    const int64_t P = p.plane;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    uint32_t nbm = 0;
    if (p.flags) {
        const uint8_t fl = p.flags[cell];
        if (fl & 1) {
            unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = (CT)0; });
            return (CT)0;
        }
        if (fl & 2) nbm = p.nbm[cell];
    }
    const uint32_t e = edge_bits(p, X, Y, Z);
    const uint32_t irr = irregular_mask<L>(e, nbm);
    CT h[Q];
    {
        const int64_t sc = sidx<ST>(p, cell);   // F is in the forward path's storage layout
        unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I>(F, sc); });
    }
    const int zf = zh_face_of(p, e);
    CT hpre[REG ? Q : 1];
    if constexpr (REG) unroll<Q>([&](auto I) { hpre[I] = h[I]; });
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
    const CT uu = ux * ux + uy * uy + uz * uz;
    const CT usq15 = (CT)1.5 * uu;
    const CT om = p.omega;

    // b_k: adjoint of the post-collision value f°_k(x): a_k(x + c_k) for a
    // fluid neighbour, a_opp(k)(x) off a wall or solid, 0 out of an open face.
    // Wavefronts of interior cells gather without tests; wavefronts whose
    // boundary cells only meet wall faces or solids choose the address per lane.
    CT b[Q];
    CT ex = 0, ey = 0, ez = 0;  // adjoint of u(x, t) through the equilibrium fills
    constexpr uint32_t kFaces = all_face_bits<L>();
    if (__all(irr == 0)) {
        unroll<Q>([&](auto K) {
            const int64_t dst = cell + ((int64_t)L::c[K][0] * p.sX + (int64_t)L::c[K][1] * p.sY + L::c[K][2]);
            b[K] = An[(int64_t)K * P + dst];
        });
    } else if (__all((e & kFaces & ~(p.wallmask | (p.permask & kZFaces))) == 0)) {
        const ZWrap zw = z_wrap(p, e & p.permask);
        unroll<Q>([&](auto K) {
            constexpr int O = opp<L>(K);
            // x + c_k is across a wall or solid (periodic Z faces wrap)
            const bool wall = ((e & p.wallmask & src_face_bits<L>(O)) | (nbm & (1u << O))) != 0;
            const int64_t dst = cell + src_off<L, O>(p, zw);
            b[K] = An[wall ? (int64_t)O * P + cell : (int64_t)K * P + dst];
        });
    } else {
        unroll<Q>([&](auto K) {
            constexpr int O = opp<L>(K);
            if (!((irr >> O) & 1u)) {
                const int64_t dst = cell + ((int64_t)L::c[K][0] * p.sX + (int64_t)L::c[K][1] * p.sY + L::c[K][2]);
                b[K] = An[(int64_t)K * P + dst];
            } else {
                const Nb nb = classify_src<L>(p, X, Y, Z, O, nbm);  // the cell x + c_k
                const int64_t idx = (nb.kind == NB_FLUID) ? (int64_t)K * P + nb.cell : (int64_t)O * P + cell;
                const CT v = An[idx];
                b[K] = (nb.kind == NB_FLUID || nb.kind == NB_WALL) ? v : (CT)0;
            }
        });
        if (irr) {
            const bool perim = (e & p.wallmask) != 0;
            unroll<Q>([&](auto K) {
                if ((irr >> K) & 1u) {
                    const Nb ns = classify_src<L>(p, X, Y, Z, K, nbm);
                    if (ns.kind == NB_OUT ||
                        (ns.kind == NB_ZH && perim && (p.ft->type[ns.face] == F_ZH_PRES || p.ft->type[ns.face] == F_REG_PRES))) {
                        const CT aK = An[(int64_t)K * P + cell];
                        const CT rf = p.ft->rho[ns.face];
                        const CT cu = (CT)L::c[K][0] * ux + (CT)L::c[K][1] * uy + (CT)L::c[K][2] * uz;
                        const CT g = aK * (CT)weight<L>(K) * rf;
                        ex += g * ((CT)3 * (CT)L::c[K][0] + (CT)9 * cu * (CT)L::c[K][0] - (CT)3 * ux);
                        ey += g * ((CT)3 * (CT)L::c[K][1] + (CT)9 * cu * (CT)L::c[K][1] - (CT)3 * uy);
                        ez += g * ((CT)3 * (CT)L::c[K][2] + (CT)9 * cu * (CT)L::c[K][2] - (CT)3 * uz);
                    }
                }
            });
        }
    }

    CT s = 0;
    if constexpr (HAS_S) s = (CT)p.s[cell];
    // body force: du = F / rho, bq = 1.5 du . (u + u'), u' = u + du
    CT dx = 0, dy = 0, dz = 0, bq = 0;
    if constexpr (FRC) {
        CT fx, fy, fz;
        load_body_force(p, cell, fx, fy, fz);
        dx = fx * inv;
        dy = fy * inv;
        dz = fz * inv;
        bq = (CT)1.5 * (dx * ((CT)2 * ux + dx) + dy * ((CT)2 * uy + dy) + dz * ((CT)2 * uz + dz));
    }
    const CT eu = ex * ux + ey * uy + ez * uz;
    CT a[Q];
    CT gt = 0;
    if constexpr (KB) {
        // lambda = (1 - s) b; the KBC collision's transpose; dL/ds against its output
        CT lam[Q];
        unroll<Q>([&](auto I) { lam[I] = HAS_S ? ((CT)1 - s) * b[I] : b[I]; });
        gt = kbc_transpose<L>(h, lam, a, p, drho, rho, inv, ux, uy, uz, usq15);
        if constexpr (HAS_S) {
            CT post[Q];
            kbc_relax<L>(h, post, p, drho, rho, ux, uy, uz, usq15);
            CT gs = 0;
            unroll<Q>([&](auto I) { gs += b[I] * (h[opp<L>(I)] - post[I]); });
            if (ds) ds[cell] += gs;
        }
        unroll<Q>([&](auto J) {
            constexpr int O = opp<L>(J);
            const CT ce = cdot<L, J>(ex, ey, ez);
            a[J] += (ce - eu) * inv;
            if constexpr (HAS_S) a[J] += s * b[O];
        });
    } else {
        // lambda = (1 - s) b (partial bounce-back), dL/ds, dL/dtau * tau^2, A, V
        // (force: AFs = sum w lambda cd (9 cu + 4.5 cd), T3 = sum w lambda cd c, cd = c . du)
        CT gs = 0, Aa = 0, Vx = 0, Vy = 0, Vz = 0, Sw = 0;
        CT AFs = 0, Tx = 0, Ty = 0, Tz = 0;
        unroll<Q>([&](auto I) {
            constexpr int O = opp<L>(I);
            const CT lam = HAS_S ? ((CT)1 - s) * b[I] : b[I];
            const CT neq = h[I] - heq<L, I>(drho, rho, ux, uy, uz, usq15);
            const CT cu = (CT)L::c[I][0] * ux + (CT)L::c[I][1] * uy + (CT)L::c[I][2] * uz;
            CT cd = 0;
            if constexpr (FRC) cd = (CT)L::c[I][0] * dx + (CT)L::c[I][1] * dy + (CT)L::c[I][2] * dz;
            if constexpr (HAS_S) {
                CT post = h[I] - om * neq;
                if constexpr (FRC)
                    post += (CT)weight<L>(I) * rho * ((CT)3 * cd + (CT)4.5 * cd * ((CT)2 * cu + cd) - bq);
                gs += b[I] * (h[O] - post);
            }
            gt += lam * neq;
            const CT wl = (CT)weight<L>(I) * lam;
            Aa += wl * ((CT)1 - (CT)4.5 * cu * cu + (CT)1.5 * uu);
            Sw += wl;
            const CT t9 = (CT)3 + (CT)9 * cu;
            if constexpr (L::c[I][0] != 0) Vx += wl * t9 * (CT)L::c[I][0];
            if constexpr (L::c[I][1] != 0) Vy += wl * t9 * (CT)L::c[I][1];
            if constexpr (L::c[I][2] != 0) Vz += wl * t9 * (CT)L::c[I][2];
            if constexpr (FRC) {
                const CT wcd = wl * cd;
                AFs += wcd * ((CT)9 * cu + (CT)4.5 * cd);
                if constexpr (L::c[I][0] != 0) Tx += wcd * (CT)L::c[I][0];
                if constexpr (L::c[I][1] != 0) Ty += wcd * (CT)L::c[I][1];
                if constexpr (L::c[I][2] != 0) Tz += wcd * (CT)L::c[I][2];
            }
        });
        if constexpr (HAS_S) {
            if (ds) ds[cell] += gs;
        }
        Vx -= (CT)3 * ux * Sw;
        Vy -= (CT)3 * uy * Sw;
        Vz -= (CT)3 * uz * Sw;
        // force: A_F = bq Sw - AFs, V_F = 9 T3 - 3 du Sw; dL/dF = V + V_F
        CT AF = 0, VFx = 0, VFy = 0, VFz = 0;
        if constexpr (FRC) {
            AF = bq * Sw - AFs;
            VFx = (CT)9 * Tx - (CT)3 * dx * Sw;
            VFy = (CT)9 * Ty - (CT)3 * dy * Sw;
            VFz = (CT)9 * Tz - (CT)3 * dz * Sw;
            if (dF) {
                dF[cell] += Vx + VFx;
                dF[N + cell] += Vy + VFy;
                dF[2 * N + cell] += Vz + VFz;
            }
        }
        unroll<Q>([&](auto J) {
            constexpr int O = opp<L>(J);
            const CT lam = HAS_S ? ((CT)1 - s) * b[J] : b[J];
            const CT cV = (CT)L::c[J][0] * Vx + (CT)L::c[J][1] * Vy + (CT)L::c[J][2] * Vz;
            const CT ce = (CT)L::c[J][0] * ex + (CT)L::c[J][1] * ey + (CT)L::c[J][2] * ez;
            CT v = ((CT)1 - om) * lam + om * (Aa + cV) + (ce - eu) * inv;
            if constexpr (FRC) v += AF + (CT)L::c[J][0] * VFx + (CT)L::c[J][1] * VFy + (CT)L::c[J][2] * VFz;
            if constexpr (HAS_S) v += s * b[O];
            a[J] = v;
        });
    }
    if (zf >= 0 && pending) {
        if constexpr (REG) {
            if (p.ft->type[zf] >= F_REG_VEL) regularize_transpose<L>(a, p, zf, hpre);
            else zouhe_transpose<L>(a, p, zf);
        } else {
            zouhe_transpose<L>(a, p, zf);
        }
    }
    unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = a[I]; });
    return gt;
}

// FP64 sum of v over the block, added to acc[row] (fixed order)
__device__ __forceinline__ void block_add(double v, double *acc, int64_t row) {
    __shared__ double red[kMaxBlock / 64];
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = ((int)blockDim.x + 63) / 64;
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[w];
        acc[row] += t;
    }
}

// Waves per SIMD the register allocation must leave room for.  The adjoint
// step is latency bound: measured on D3Q19 FP32 256^3, 4 waves (<= 128 VGPRs)
// run 15% faster than the compiler's 3, 5 waves spill.
// FP64 arithmetic keeps the compiler's choice.
// With the body force, regularized faces or KBC (more live values) D3Q19 FP32
// asks for 3 waves and D3Q27 for 2: one more spills.
template <class L, class ST, bool FRC = false, bool REG = false, bool KB = false>
struct AdjWaves {
    static constexpr bool f64 = sizeof(typename Store<ST>::CT) == 8;
    static constexpr int value = f64 ? 1
                                     : ((L::Q == 19) ? ((FRC || REG || KB) ? 3 : 4)
                                                     : ((L::Q == 27) ? ((FRC || REG || KB) ? 2 : 3) : 1));
};
#ifdef LBM_ADJ_WAVES
#define LBM_ADJ_ATTR __attribute__((amdgpu_waves_per_eu(LBM_ADJ_WAVES)))
#define LBM_ADJ_ATTR_F LBM_ADJ_ATTR
#else
#define LBM_ADJ_ATTR __attribute__((amdgpu_waves_per_eu(AdjWaves<L, ST>::value)))
#define LBM_ADJ_ATTR_F __attribute__((amdgpu_waves_per_eu(AdjWaves<L, ST, FRC, REG, KB>::value)))
#endif

template <class L, class ST, bool HAS_S, bool FRC, bool REG, bool KB>
__global__ void __launch_bounds__(kMaxBlock) LBM_ADJ_ATTR_F k_adjoint(const Params<typename Store<ST>::CT> p, const ST *__restrict__ F,
                                                       const typename Store<ST>::CT *__restrict__ An,
                                                       typename Store<ST>::CT *__restrict__ Ao,
                                                       typename Store<ST>::CT *__restrict__ ds, double *__restrict__ acc,
                                                       typename Store<ST>::CT *__restrict__ dF, int64_t N) {
    int X, Y, Z;
    double g = 0.0;
    if (adj_block_cell(p, X, Y, Z))
        g = (double)adjoint_cell<L, ST, HAS_S, FRC, REG, KB>(p, F, An, Ao, ds, X, Y, Z, p.zh_pending, dF, N);
    block_add(g, acc, blockIdx.x);
}

// dL/dF out: out[a N + cell] = eps dF[(a + off) N + cell] (caller axis a < D;
// off = 1 for 2-D, whose caller axes x, y are the internal Y, Z), and one row
// of D FP64 block sums per workgroup (for the uniform force's gradient).
template <class CT, class OT>
__global__ void __launch_bounds__(256) k_df_out(const CT *__restrict__ dF, OT *__restrict__ out, int64_t N, int D,
                                                int off, double eps, double *__restrict__ rows) {
    __shared__ double red[3][4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    for (int a = 0; a < D; ++a) {
        double v = 0.0;
        if (i < N) {
            v = eps * (double)dF[(int64_t)(a + off) * N + i];
            if (out) out[(int64_t)a * N + i] = (OT)v;
        }
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[a][wv] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < D) {
        const int nw = ((int)blockDim.x + 63) / 64;
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[threadIdx.x][w];
        rows[(int64_t)blockIdx.x * D + threadIdx.x] = t;
    }
}

// Wall-velocity gradient of one step: tile k covers `blockDim.x` cells of
// moving-wall face wt.face[k] of domain wt.dom[k] (face-local index from
// wt.start[k]); for each incoming population bounced off that face,
// dL/du_w += a_K(x, t+1) 6 w_K rho0 c_K.  accw: 3 rows per tile (internal axes).
template <class L, class CT, bool BATCH>
__global__ void __launch_bounds__(kMaxBlock) k_adj_walls(const Params<CT> p1, const BatchDev b, const WallTiles wt,
                                                         const CT *__restrict__ An, double *__restrict__ accw) {
    constexpr int Q = L::Q;
    __shared__ double red[3][kMaxBlock / 64];
    const int tile = (int)blockIdx.x;
    const int d = wt.dom[tile], f = wt.face[tile];
    const Params<CT> &p = BATCH ? dom_params<CT>(b, d) : p1;
    const CT *A = BATCH ? An + b.stoff[d] : An;
    const int ax = f >> 1;
    const int na = (ax == 0) ? p.nY : p.nX;
    const int nb = (ax == 2) ? p.nY : p.nZ;
    const int q = wt.start[tile] + (int)threadIdx.x;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    if (q < na * nb) {
        const int i = q / nb, j = q - (q / nb) * nb;
        const int fixed = (f & 1) ? ((ax == 0) ? p.nX : ((ax == 1) ? p.nY : p.nZ)) - 1 : 0;
        const int X = (ax == 0) ? fixed : i;
        const int Y = (ax == 0) ? i : ((ax == 1) ? fixed : j);
        const int Z = (ax == 2) ? fixed : j;
        const int64_t P = p.plane;
        const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
        uint32_t nbm = 0;
        bool solid = false;
        if (p.flags) {
            const uint8_t fl = p.flags[cell];
            solid = fl & 1;
            if (fl & 2) nbm = p.nbm[cell];
        }
        if (!solid) {
            const uint32_t irr = irregular_mask<L>(edge_bits(p, X, Y, Z), nbm);
            unroll<Q>([&](auto K) {
                if ((irr >> K) & 1u) {
                    const Nb ns = classify_src<L>(p, X, Y, Z, K, nbm);
                    if (ns.kind == NB_WALL && ns.face == f) {
                        const double v = (double)A[(int64_t)K * P + cell] * 6.0 * weight<L>(K) * (double)p.rho0;
                        g0 += v * L::c[K][0];
                        g1 += v * L::c[K][1];
                        g2 += v * L::c[K][2];
                    }
                }
            });
        }
    }
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        g0 += __shfl_xor(g0, o);
        g1 += __shfl_xor(g1, o);
        g2 += __shfl_xor(g2, o);
    }
    if (lane == 0) {
        red[0][wv] = g0;
        red[1][wv] = g1;
        red[2][wv] = g2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int nw = ((int)blockDim.x + 63) / 64;
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[threadIdx.x][w];
        accw[(int64_t)tile * 3 + threadIdx.x] += t;
    }
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
    const int64_t P = p.plane;
    const int64_t cell = ((int64_t)X * p.nY + Y) * p.nZ + Z;
    if (p.flags && (p.flags[cell] & 1)) {
        unroll<Q>([&](auto I) { Ao[(int64_t)I * P + cell] = (CT)0; });
        return;
    }
    const uint32_t e = edge_bits(p, X, Y, Z);
    CT h[Q];
    {
        const int64_t sc = sidx<ST>(p, cell);   // F is in the forward path's storage layout
        unroll<Q>([&](auto I) { h[I] = ldh<L, ST, I>(F, sc); });
    }
    const int zf = zh_face_of(p, e);
    CT hpre[Q];   // pre-closure populations (regularized faces)
    unroll<Q>([&](auto I) { hpre[I] = h[I]; });
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
    if (zf >= 0 && pending) {
        if (p.ft->type[zf] >= F_REG_VEL) regularize_transpose<L>(a, p, zf, hpre);
        else zouhe_transpose<L>(a, p, zf);
    }
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
    uint32_t nbm = 0;
    if (p.flags) {
        const uint8_t fl = p.flags[cell];
        if (fl & 1) return;
        if (fl & 2) nbm = p.nbm[cell];
    }
    const uint32_t e = edge_bits_st<ST>(p, X, Y, Z);
    const uint32_t irr = irregular_mask<L>(e, nbm);
    const int64_t sc = sidx<ST>(p, cell);
    const int64_t sm = smul<ST>(p);
    unroll<Q>([&](auto I) {
        constexpr int O = opp<L>(I);
        ST v;
        if (!((irr >> I) & 1u)) {
            const int64_t src = sc - sm * ((int64_t)L::c[I][0] * p.sX + (int64_t)L::c[I][1] * p.sY + L::c[I][2]);
            v = A[pidx<Q>(O, src)];
        } else {
            const Nb nb = classify_src<L>(p, X, Y, Z, I, nbm);
            v = (nb.kind == NB_FLUID) ? A[pidx<Q>(O, sidx<ST>(p, nb.cell))] : A[pidx<Q>(I, sc)];
        }
        D[pidx<Q>(I, sc)] = v;  // opposite slots share the storage scale
    });
}

template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) k_materialize(const Params<typename Store<ST>::CT> p,
                                                           const ST *__restrict__ A, ST *__restrict__ D) {
    int X, Y, Z;
    if (!adj_block_cell(p, X, Y, Z)) return;
    materialize_cell<L, ST>(p, A, D, X, Y, Z);
}

template <class CT>
__global__ void __launch_bounds__(256) k_to_float(const CT *__restrict__ src, float *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// ---- batch variants ------------------------------------------------------------
template <class L, class ST>
__global__ void __launch_bounds__(kMaxBlock) LBM_ADJ_ATTR k_adjoint_batch(const BatchDev b, const ST *__restrict__ F,
                                                             const typename Store<ST>::CT *__restrict__ An,
                                                             typename Store<ST>::CT *__restrict__ Ao,
                                                             double *__restrict__ acc, int pending) {
    using CT = typename Store<ST>::CT;
    const int tile = (int)blockIdx.x;
    const int d = b.tile_dom[tile];
    const Params<CT> &p = dom_params<CT>(b, d);
    const int c = b.tile_start[tile] + (int)threadIdx.x;
    double g = 0.0;
    if (c < p.nX * p.nY * p.nZ) {
        int X, Y, Z;
        split_cell(c, p.nY, p.nZ, X, Y, Z);
        const int64_t o = b.stoff[d];
        g = (double)adjoint_cell<L, ST, false>(p, F + o, An + o, Ao + o, nullptr, X, Y, Z, pending);
    }
    block_add(g, acc, tile);
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

// ---------------------------------------------------------------------------
template <class L, class ST>
static hipError_t adj_dispatch(const AdjLaunch &g) {
    using CT = typename Store<ST>::CT;
    const bool batch = g.batch != nullptr;
    const Params<CT> p = batch ? Params<CT>{} : *static_cast<const Params<CT> *>(g.params);
    const BatchDev bd = batch ? *g.batch : BatchDev{};
    const dim3 grid(g.grid), block(g.block);
    switch (g.op) {
        case ADJ_STEP:
            if (batch)
                hipLaunchKernelGGL((k_adjoint_batch<L, ST>), grid, block, 0, g.stream, bd, static_cast<const ST *>(g.F),
                                   static_cast<const CT *>(g.An), static_cast<CT *>(g.Ao), g.acc, g.pending);
            else {
#define LBM_ADJ(S, FR, RG, KB)                                                                                     \
    hipLaunchKernelGGL((k_adjoint<L, ST, S, FR, RG, KB>), grid, block, 0, g.stream, p,                             \
                       static_cast<const ST *>(g.F),                                                             \
                       static_cast<const CT *>(g.An), static_cast<CT *>(g.Ao), static_cast<CT *>(g.ds), g.acc,    \
                       static_cast<CT *>(g.dF), g.N);
                // (regularized faces or KBC with a body force, and KBC with
                // regularized faces, are refused by the host; KBC runs on D2Q9
                // and D3Q27)
                if (g.kbc) {
                    if constexpr (L::Q != 19) {
                        if (g.ds) LBM_ADJ(true, false, false, true)
                        else LBM_ADJ(false, false, false, true)
                    }
                } else if (g.reg && g.ds) LBM_ADJ(true, false, true, false)
                else if (g.reg) LBM_ADJ(false, false, true, false)
                else if (g.ds && g.force) LBM_ADJ(true, true, false, false)
                else if (g.ds) LBM_ADJ(true, false, false, false)
                else if (g.force) LBM_ADJ(false, true, false, false)
                else LBM_ADJ(false, false, false, false)
#undef LBM_ADJ
            }
            break;
        case ADJ_WALLS:
            if (g.walls.n == 0) break;
            if (batch)
                hipLaunchKernelGGL((k_adj_walls<L, CT, true>), dim3(g.walls.n), dim3(g.walls.block), 0, g.stream, p,
                                   bd, g.walls, static_cast<const CT *>(g.An), g.accw);
            else
                hipLaunchKernelGGL((k_adj_walls<L, CT, false>), dim3(g.walls.n), dim3(g.walls.block), 0, g.stream, p,
                                   bd, g.walls, static_cast<const CT *>(g.An), g.accw);
            break;
        case ADJ_SEED:
#define LBM_SEED(IT)                                                                                                \
    if (batch)                                                                                                      \
        hipLaunchKernelGGL((k_seed_batch<L, ST, IT>), grid, block, 0, g.stream, bd, static_cast<const ST *>(g.F),  \
                           static_cast<const IT *>(g.grho), static_cast<const IT *>(g.gu), static_cast<CT *>(g.Ao), \
                           g.pending);                                                                              \
    else                                                                                                            \
        hipLaunchKernelGGL((k_seed<L, ST, IT>), grid, block, 0, g.stream, p, static_cast<const ST *>(g.F),          \
                           static_cast<const IT *>(g.grho), static_cast<const IT *>(g.gu), static_cast<CT *>(g.Ao), \
                           g.N);
            if (g.in_f64) {
                LBM_SEED(double)
            } else {
                LBM_SEED(float)
            }
#undef LBM_SEED
            break;
        case ADJ_MATERIALIZE:
            if (batch)
                hipLaunchKernelGGL((k_materialize_batch<L, ST>), grid, block, 0, g.stream, bd,
                                   static_cast<const ST *>(g.F), static_cast<ST *>(g.D));
            else
                hipLaunchKernelGGL((k_materialize<L, ST>), grid, block, 0, g.stream, p, static_cast<const ST *>(g.F),
                                   static_cast<ST *>(g.D));
            break;
        case ADJ_DS_OUT: {
            const unsigned nb = (unsigned)((g.N + 255) / 256);
            hipLaunchKernelGGL((k_to_float<CT>), dim3(nb), dim3(256), 0, g.stream, static_cast<const CT *>(g.ds),
                               g.ds_out, g.N);
            break;
        }
        case ADJ_DF_OUT: {
            const unsigned nb = (unsigned)((g.N + 255) / 256);
            const int D = (g.lattice == LAT_D2Q9) ? 2 : 3;
            const int off = (D == 2) ? 1 : 0;
            if (g.in_f64)
                hipLaunchKernelGGL((k_df_out<CT, double>), dim3(nb), dim3(256), 0, g.stream,
                                   static_cast<const CT *>(g.dF), static_cast<double *>(g.df_out), g.N, D, off, g.eps,
                                   g.acc);
            else
                hipLaunchKernelGGL((k_df_out<CT, float>), dim3(nb), dim3(256), 0, g.stream,
                                   static_cast<const CT *>(g.dF), static_cast<float *>(g.df_out), g.N, D, off, g.eps,
                                   g.acc);
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

}  // namespace lbm
