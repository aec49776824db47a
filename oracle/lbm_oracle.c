/*
 * lbm_oracle.c -- plain FP64 CPU reference of the lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never does.  It shares
 * no code, header, table or helper with the GPU path.
 *
 * What it computes (paper: "XLB: a differentiable massively parallel lattice
 * Boltzmann library in Python", Sec. 2 and Sec. 3):
 *   - collision, eq. (collision) with the BGK operator, eq. (LBM-BGK), and the
 *     quadratic equilibrium, eq. (feq); units dx = dt = 1, cs^2 = 1/3, eq. (tau);
 *   - moments, eqs. (density) and (velocity);
 *   - streaming, eq. (streaming), periodic by default (Sec. 3.4);
 *   - boundary conditions applied after streaming (Sec. 3.5, Sec. 3.6):
 *     halfway bounce-back with an optional moving-wall term, Zou-He
 *     velocity / pressure faces, an equilibrium outflow face; interior solid
 *     cells bounce back; an optional partial bounce-back (solid fraction s).
 *
 * Layout: array of structures f[((x*ny + y)*nz + z)*q + i], as the paper's
 * (nx, ny, nz, q) arrays (Sec. 3.3).  Double buffered, literal formulas, no
 * blocking or fusion.  The state f(t) is the post-stream, post-boundary,
 * pre-collision population; one step maps f(t) to f(t+1).
 *
 * Readings of points the paper leaves open (lattice weights, wall position,
 * the 3-D Zou-He closure, the outflow velocity, the partial bounce-back
 * variant) are listed in the design notes; each is restated at its use below.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* face types */
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_ZOUHE_VEL = 2, ORC_ZOUHE_PRES = 3, ORC_OUTFLOW = 4,
       ORC_REG_VEL = 5, ORC_REG_PRES = 6 };
/* velocity / pressure faces (Zou-He or regularized) */
static int vel_face(int t) { return t == ORC_ZOUHE_VEL || t == ORC_REG_VEL; }
static int pres_face(int t) { return t == ORC_ZOUHE_PRES || t == ORC_REG_PRES; }

typedef struct {
    int type;
    double u[3];   /* wall / inlet velocity */
    double rho;    /* pressure-face or outflow density */
} orc_face;

typedef struct {
    int q;                      /* 9, 19 or 27 */
    int nx, ny, nz;             /* nz = 1 for D2Q9 */
    double tau;
    double rho0;                /* reference density of the moving-wall term */
    orc_face face[6];           /* -x, +x, -y, +y, -z, +z */
    const uint8_t *solid;       /* N bytes, 1 = solid; NULL = none */
    const double *s;            /* N solid fractions (partial bounce-back); NULL = none */
    double force[3];            /* body force, test hook only (Poiseuille pin) */
    const double *edm;          /* N*3 body force per cell, exact-difference method; NULL = none */
    int collision;              /* 0: BGK; 1: KBC entropic multi-relaxation (D2Q9, D3Q27) */
    const double *qlink;        /* N*q wall fractions of curved links (0 = halfway); NULL = none */
    int bouzidi_order;          /* 1: linear, 2: quadratic interpolated bounce-back */
} orc_sim;

/* ---------------------------------------------------------------------------
 * Lattice tables.  Direction order: rest vector first, then the order in which
 * the paper's lattice figure lists the vectors (Fig. "lattice").  Weights are
 * the textbook values by |c|^2 (Krueger et al., the paper's LBM reference);
 * the paper does not print them.
 * ------------------------------------------------------------------------- */
static const int C9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0}};
static const int C27[27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
    {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
    {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1},
    {-1, 1, 1}, {-1, 1, -1}, {-1, -1, 1}, {-1, -1, -1}};
/* D3Q19 is the first 19 entries of the D3Q27 list (rest, 6 faces, 12 edges). */

static const int *cvec(int q, int i)
{
    return q == 9 ? C9[i] : C27[i];
}

static double weight(int q, int i)
{
    const int *c = cvec(q, i);
    int n = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    if (q == 9) { const double w[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0}; return w[n]; }
    if (q == 19) { const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0}; return w[n]; }
    { const double w[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0}; return w[n]; }
}

static int opposite(int q, int i)
{
    const int *c = cvec(q, i);
    for (int j = 0; j < q; ++j) {
        const int *d = cvec(q, j);
        if (d[0] == -c[0] && d[1] == -c[1] && d[2] == -c[2]) return j;
    }
    return -1;
}

int orc_tables(int q, int *c_out, double *w_out, int *opp_out)
{
    if (q != 9 && q != 19 && q != 27) return -1;
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        for (int a = 0; a < 3; ++a) c_out[3 * i + a] = c[a];
        w_out[i] = weight(q, i);
        opp_out[i] = opposite(q, i);
    }
    return 0;
}

/* eq. (feq): w_i rho {1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - |u|^2/(2 cs^2)} */
static double feq_i(int q, int i, double rho, const double u[3])
{
    const int *c = cvec(q, i);
    const double cs2 = 1.0 / 3.0;
    double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return weight(q, i) * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

void orc_equilibrium(int q, double rho, const double *u, double *feq)
{
    for (int i = 0; i < q; ++i) feq[i] = feq_i(q, i, rho, u);
}

/* eqs. (density), (velocity) */
static void moments(int q, const double *f, double *rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        r += f[i];
        for (int a = 0; a < 3; ++a) j[a] += c[a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

void orc_cell_moments(int q, const double *f, double *rho, double *u)
{
    moments(q, f, rho, u);
}

/* eq. (LBM-BGK) with dt = 1: f* = f - (1/tau)(f - feq).  The force hook adds
 * 3 w_i (c_i . F) after relaxation (oracle test hook only).  A body force F
 * by the exact-difference method (Sec. 4.4 and 6.1, after Kupershtokh) adds
 * feq_i(rho, u + F/rho) - feq_i(rho, u) to the relaxed populations. */
/* KBC collision (Karlin, Bosch & Chikatamarla 2014; listed in Sec. 2, the
 * paper's collision for its D2Q9 / D3Q27 runs of Sec. 4).  f - feq splits into a shear part ds,
 * built from the deviatoric non-equilibrium momentum flux on the axis and
 * face-diagonal velocities only (zero mass, momentum and trace), and the rest
 * dh:
 *   D2Q9 : axis (+-1, 0): (P_xx - P_yy) / 4, axis (0, +-1): -(P_xx - P_yy) / 4,
 *          diagonal c: c_x c_y P_xy / 4;
 *   D3Q27: axis +-e_a: (2 P_aa - P_bb - P_cc) / 6, face diagonal in the (a, b)
 *          plane: c_a c_b P_ab / 4, corners and rest 0;
 * with P = sum_i c_i c_i (f_i - feq_i).  Then
 *   f*_i = f_i - beta (2 ds_i + gamma dh_i),  beta = 1 / (2 tau),
 *   gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>,  <x|y> = sum_i x_i y_i / feq_i,
 * the gamma that minimizes the quadratic entropy <f* - feq|f* - feq>; with
 * dh = 0 it is BGK. */
static void kbc_collide(int q, const double *f, const double *feq, double tau, double *fstar)
{
    double fneq[27], ds[27], dh[27];
    for (int i = 0; i < q; ++i) fneq[i] = f[i] - feq[i];
    double P[3][3] = {{0.0}};
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) P[a][b] += c[a] * c[b] * fneq[i];
    }
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        int nz = (c[0] != 0) + (c[1] != 0) + (c[2] != 0);
        double v = 0.0;
        if (nz == 1) {
            int a = (c[0] != 0) ? 0 : ((c[1] != 0) ? 1 : 2);
            if (q == 9) v = (a == 0 ? 1.0 : -1.0) * (P[0][0] - P[1][1]) / 4.0;
            else v = (2.0 * P[a][a] - P[(a + 1) % 3][(a + 1) % 3] - P[(a + 2) % 3][(a + 2) % 3]) / 6.0;
        } else if (nz == 2) {
            int a = (c[0] == 0) ? 1 : 0;
            int b = (c[2] != 0) ? 2 : 1;
            v = c[a] * c[b] * P[a][b] / 4.0;
        }
        ds[i] = v;
        dh[i] = fneq[i] - v;
    }
    double beta = 0.5 / tau, sh = 0.0, hh = 0.0;
    for (int i = 0; i < q; ++i) {
        sh += ds[i] * dh[i] / feq[i];
        hh += dh[i] * dh[i] / feq[i];
    }
    double gamma = (hh > 0.0) ? 1.0 / beta - (2.0 - 1.0 / beta) * sh / hh : 2.0;
    for (int i = 0; i < q; ++i) fstar[i] = f[i] - beta * (2.0 * ds[i] + gamma * dh[i]);
}

static void collide_f(const orc_sim *S, const double *f, double *fstar, double *rho, double u[3], const double *F)
{
    int q = S->q;
    double omega = 1.0 / S->tau;
    moments(q, f, rho, u);
    double w[3];
    if (F)
        for (int a = 0; a < 3; ++a) w[a] = u[a] + F[a] / *rho;
    if (S->collision == 1) {
        double feq[27];
        for (int i = 0; i < q; ++i) feq[i] = feq_i(q, i, *rho, u);
        kbc_collide(q, f, feq, S->tau, fstar);
    }
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        if (S->collision != 1) fstar[i] = f[i] - omega * (f[i] - feq_i(q, i, *rho, u));
        fstar[i] += 3.0 * weight(q, i) * (c[0] * S->force[0] + c[1] * S->force[1] + c[2] * S->force[2]);
        if (F) fstar[i] += feq_i(q, i, *rho, w) - feq_i(q, i, *rho, u);
    }
}

static void collide(const orc_sim *S, const double *f, double *fstar, double *rho, double u[3])
{
    collide_f(S, f, fstar, rho, u, NULL);
}

/* The KBC collision of one cell, moments and equilibrium included, in complex
 * arithmetic: the same operations as moments, feq_i and kbc_collide above,
 * for the complex-step derivative of the adjoint (Squire & Trapp 1998): for a
 * map g that is real-analytic at x, Im g(x + i h e_j) / h = dg/dx_j + O(h^2)
 * with no difference of nearby values, so h = 1e-30 gives the derivative to
 * rounding.  gamma's branch is taken on the real part. */
static void kbc_collide_cx(int q, const double complex *f, double complex tau, double complex *fstar)
{
    const double cs2 = 1.0 / 3.0;
    double complex rho = 0.0, j[3] = {0.0, 0.0, 0.0}, u[3];
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += c[a] * f[i];
    }
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    double complex feq[27], fneq[27], ds[27], dh[27];
    const double complex uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        double complex cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        feq[i] = weight(q, i) * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
        fneq[i] = f[i] - feq[i];
    }
    double complex P[3][3] = {{0.0}};
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) P[a][b] += c[a] * c[b] * fneq[i];
    }
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        int nz = (c[0] != 0) + (c[1] != 0) + (c[2] != 0);
        double complex v = 0.0;
        if (nz == 1) {
            int a = (c[0] != 0) ? 0 : ((c[1] != 0) ? 1 : 2);
            if (q == 9) v = (a == 0 ? 1.0 : -1.0) * (P[0][0] - P[1][1]) / 4.0;
            else v = (2.0 * P[a][a] - P[(a + 1) % 3][(a + 1) % 3] - P[(a + 2) % 3][(a + 2) % 3]) / 6.0;
        } else if (nz == 2) {
            int a = (c[0] == 0) ? 1 : 0;
            int b = (c[2] != 0) ? 2 : 1;
            v = c[a] * c[b] * P[a][b] / 4.0;
        }
        ds[i] = v;
        dh[i] = fneq[i] - v;
    }
    double complex beta = 0.5 / tau, sh = 0.0, hh = 0.0;
    for (int i = 0; i < q; ++i) {
        sh += ds[i] * dh[i] / feq[i];
        hh += dh[i] * dh[i] / feq[i];
    }
    double complex gamma = (creal(hh) > 0.0) ? 1.0 / beta - (2.0 - 1.0 / beta) * sh / hh : 2.0;
    for (int i = 0; i < q; ++i) fstar[i] = f[i] - beta * (2.0 * ds[i] + gamma * dh[i]);
}

/* d f*_i / d f_j (jac) and d f*_i / d tau (dtau) of the KBC collision at f,
 * by the complex step. */
static void kbc_jacobian(int q, const double *f, double tau, double jac[27][27], double dtau[27])
{
    const double hstep = 1e-30;
    double complex fc[27], out[27];
    for (int j = 0; j < q; ++j) {
        for (int i = 0; i < q; ++i) fc[i] = f[i];
        fc[j] += hstep * I;
        kbc_collide_cx(q, fc, tau, out);
        for (int i = 0; i < q; ++i) jac[i][j] = cimag(out[i]) / hstep;
    }
    for (int i = 0; i < q; ++i) fc[i] = f[i];
    kbc_collide_cx(q, fc, tau + hstep * I, out);
    for (int i = 0; i < q; ++i) dtau[i] = cimag(out[i]) / hstep;
}

void orc_collide_cell(const orc_sim *S, const double *f, double *fstar)
{
    double rho, u[3];
    collide(S, f, fstar, &rho, u);
}

/* ---------------------------------------------------------------------------
 * Geometry helpers.
 * ------------------------------------------------------------------------- */
static int dimn(const orc_sim *S, int a) { return a == 0 ? S->nx : (a == 1 ? S->ny : S->nz); }

static size_t cell_index(const orc_sim *S, const int x[3])
{
    return ((size_t)x[0] * S->ny + x[1]) * S->nz + x[2];
}

/* Classification of the source y = x - c_i of population i at fluid cell x. */
enum { SRC_FLUID, SRC_WALL, SRC_ZOUHE, SRC_OUTFLOW };

typedef struct {
    int kind;
    size_t cell;       /* SRC_FLUID: index of the (wrapped) source cell */
    double uw[3];      /* SRC_WALL: wall velocity (0 for solid cells, static walls) */
    int face;          /* face crossed (WALL with moving velocity / ZOUHE / OUTFLOW), else -1 */
    int wall_face;     /* SRC_WALL across the domain boundary: lowest-index wall face crossed, else -1 */
} orc_src;

/* Domain faces are halfway outside the outermost cell layer, so every cell of
 * the nx*ny*nz grid is a fluid node unless flagged solid.  If the source lies
 * across several faces and one of them is a wall, the direction bounces back;
 * a static wall among them wins over a moving one (u_w = 0). */
static orc_src classify(const orc_sim *S, const int x[3], const int *c)
{
    orc_src r;
    int y[3];
    int crossed[3], ncross = 0;
    r.kind = SRC_FLUID; r.cell = 0; r.face = -1; r.wall_face = -1;
    r.uw[0] = r.uw[1] = r.uw[2] = 0.0;
    for (int a = 0; a < 3; ++a) {
        int n = dimn(S, a);
        y[a] = x[a] - c[a];
        if (y[a] < 0 || y[a] >= n) {
            int f = 2 * a + (y[a] < 0 ? 0 : 1);
            if (S->face[f].type == ORC_PERIODIC) {
                y[a] = (y[a] + n) % n;
            } else {
                crossed[ncross++] = f;
            }
        }
    }
    if (ncross == 0) {
        r.cell = cell_index(S, y);
        if (S->solid && S->solid[r.cell]) r.kind = SRC_WALL;
        return r;
    }
    int nwall = 0, any_static = 0, first_wall = -1;
    for (int k = 0; k < ncross; ++k) {
        const orc_face *F = &S->face[crossed[k]];
        if (F->type == ORC_WALL) {
            ++nwall;
            if (first_wall < 0) first_wall = crossed[k];
            if (F->u[0] == 0.0 && F->u[1] == 0.0 && F->u[2] == 0.0) any_static = 1;
        }
    }
    if (nwall > 0) {
        r.kind = SRC_WALL;
        r.wall_face = first_wall;
        if (!any_static) {
            r.face = first_wall;
            for (int a = 0; a < 3; ++a) r.uw[a] = S->face[first_wall].u[a];
        }
        return r;
    }
    /* only one open (Zou-He or outflow) face can be crossed: they sit on one axis */
    r.face = crossed[0];
    r.kind = (S->face[r.face].type == ORC_OUTFLOW) ? SRC_OUTFLOW : SRC_ZOUHE;
    return r;
}

/*
 * Interpolated bounce-back at a curved wall (Bouzidi, Firdaouss & Lallemand
 * 2001; the paper's no-slip condition for curved geometries, Sec. 4.3).
 * Link (x_b, i): x_b is fluid, x_b + c_i is solid, and the wall cuts the link
 * at the fraction qv of its length from x_b (0 < qv <= 1).  The unknown after
 * streaming is f_opp(i)(x_b, t+1).  Measure s along c_i with x_b at s = 0, the
 * wall at s = qv and x_ff = x_b - c_i at s = -1, x_fff = x_b - 2 c_i at s = -2.
 * A population moving along c_i covers one unit per step and turns around at
 * the wall:
 *   qv <  1/2: the value that reaches x_b after the turn started at
 *              s_D = 2 qv - 1, between x_ff and x_b, so f_opp(i)(x_b, t+1) is
 *              the post-collision field f*_i(., t) interpolated at s_D from
 *              the nodes s = 0, -1 (linear) and -2 (quadratic);
 *   qv >= 1/2: f*_i(x_b, t) turns around and lands at s_P = 2 qv - 1, between
 *              x_b and the wall, so f_opp(i)(x_b, t+1) is the field of
 *              opp(i)-populations at t+1 interpolated at s = 0 from the point
 *              s_P (value f*_i(x_b, t)) and the nodes s = -1, -2, which hold
 *              f_opp(i)(x_ff, t+1) = f*_opp(i)(x_b, t) and
 *              f_opp(i)(x_fff, t+1) = f*_opp(i)(x_ff, t).
 * Lagrange interpolation through those points gives
 *   linear,    qv <  1/2: 2 qv f*_i(x_b) + (1 - 2 qv) f*_i(x_ff)
 *   linear,    qv >= 1/2: f*_i(x_b) / (2 qv) + (2 qv - 1) / (2 qv) f*_opp(x_b)
 *   quadratic, qv <  1/2: qv (1 + 2 qv) f*_i(x_b) + (1 - 4 qv^2) f*_i(x_ff)
 *                         - qv (1 - 2 qv) f*_i(x_fff)
 *   quadratic, qv >= 1/2: f*_i(x_b) / (qv (2 qv + 1)) + (2 qv - 1) / qv f*_opp(x_b)
 *                         + (1 - 2 qv) / (1 + 2 qv) f*_opp(x_ff)
 * (qv = 1/2 is halfway bounce-back in every case).  The walls are at rest.
 * Where x_ff is not a fluid node the link falls back to halfway bounce-back;
 * where the quadratic rule needs x_fff and it is not a fluid node, the linear
 * rule is used.  fpost: post-collision populations of every cell.
 */
static double bouzidi_fill(const orc_sim *S, const int xb[3], int i, double qv, const double *fpost)
{
    const int q = S->q;
    const int *c = cvec(q, i);
    const int o = opposite(q, i);
    const size_t kb = cell_index(S, xb);
    const double A = fpost[kb * q + i];
    const orc_src ff = classify(S, xb, c);          /* x_b - c_i */
    if (ff.kind != SRC_FLUID) return A;
    int xff[3];
    xff[0] = (int)(ff.cell / ((size_t)S->ny * S->nz));
    xff[1] = (int)((ff.cell / S->nz) % S->ny);
    xff[2] = (int)(ff.cell % S->nz);
    int order = S->bouzidi_order;
    orc_src fff = {0};
    if (order == 2) {
        fff = classify(S, xff, c);                   /* x_b - 2 c_i */
        if (fff.kind != SRC_FLUID) order = 1;
    }
    if (qv < 0.5) {
        const double B = fpost[ff.cell * q + i];
        if (order == 1) return 2.0 * qv * A + (1.0 - 2.0 * qv) * B;
        const double C = fpost[fff.cell * q + i];
        return qv * (1.0 + 2.0 * qv) * A + (1.0 - 4.0 * qv * qv) * B - qv * (1.0 - 2.0 * qv) * C;
    }
    const double D = fpost[kb * q + o];
    if (order == 1) return A / (2.0 * qv) + (2.0 * qv - 1.0) / (2.0 * qv) * D;
    const double E = fpost[ff.cell * q + o];
    return A / (qv * (2.0 * qv + 1.0)) + (2.0 * qv - 1.0) / qv * D + (1.0 - 2.0 * qv) / (1.0 + 2.0 * qv) * E;
}

/* Is cell x on a wall face (a perimeter cell of an open face)? */
static int on_wall_face(const orc_sim *S, const int x[3])
{
    for (int a = 0; a < 3; ++a) {
        if (x[a] == 0 && S->face[2 * a].type == ORC_WALL) return 1;
        if (x[a] == dimn(S, a) - 1 && S->face[2 * a + 1].type == ORC_WALL) return 1;
    }
    return 0;
}

/* Inward unit normal of face f (as integer vector). */
static void inward_normal(int f, int n[3])
{
    n[0] = n[1] = n[2] = 0;
    n[f / 2] = (f % 2 == 0) ? 1 : -1;
}

/*
 * Zou-He (non-equilibrium bounce-back) closure at a face cell with inward
 * normal n (the paper cites Zou & He for it in Sec. 4.3; the generic 2-D/3-D
 * form below reduces to their D2Q9 formulas).  U = {c.n = 1} are the unknown
 * populations, Z = {c.n = 0}, O = {c.n = -1} the known ones.
 *   velocity face: rho = (sum_Z f + 2 sum_O f) / (1 - u_w.n), u = u_w
 *   pressure face: rho = rho_w, u = u_n n with u_n = 1 - (sum_Z f + 2 sum_O f)/rho_w
 *   f_i = f_opp(i) + 6 w_i rho (c_i.u) - sum_t (c_i.t) N_t   (i in U)
 *   N_t = (sum_{j in Z} f_j (c_j.t) - (2/3) rho u_t) / sum_{k in U} (c_k.t)^2
 * where t runs over the two (one in 2-D) tangential axes.
 */
static void zouhe_closure(const orc_sim *S, int face, double *f)
{
    int q = S->q;
    int n[3];
    inward_normal(face, n);
    const orc_face *F = &S->face[face];
    double sumZ = 0.0, sumO = 0.0;
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        int cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
        if (cn == 0) sumZ += f[i];
        if (cn == -1) sumO += f[i];
    }
    double rho, u[3];
    if (vel_face(F->type)) {
        double un = F->u[0] * n[0] + F->u[1] * n[1] + F->u[2] * n[2];
        rho = (sumZ + 2.0 * sumO) / (1.0 - un);
        for (int a = 0; a < 3; ++a) u[a] = F->u[a];
    } else {
        rho = F->rho;
        double un = 1.0 - (sumZ + 2.0 * sumO) / rho;
        for (int a = 0; a < 3; ++a) u[a] = un * n[a];
    }
    double N[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < 3; ++t) {
        if (n[t] != 0) continue;               /* t tangential */
        double num = 0.0, den = 0.0;
        for (int j = 0; j < q; ++j) {
            const int *c = cvec(q, j);
            int cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
            if (cn == 0) num += f[j] * c[t];
            if (cn == 1) den += (double)(c[t] * c[t]);
        }
        if (den == 0.0) continue;               /* the z axis of D2Q9 */
        N[t] = (num - (2.0 / 3.0) * rho * u[t]) / den;
    }
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        int cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
        if (cn != 1) continue;
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double v = f[opposite(q, i)] + 6.0 * weight(q, i) * rho * cu;
        for (int t = 0; t < 3; ++t)
            if (n[t] == 0) v -= c[t] * N[t];
        f[i] = v;
    }
}


/* Regularized velocity / pressure face (Latt, Chopard, Malaspinas, Deville &
 * Michler 2008; the paper lists it among XLB's boundary conditions, Sec. 3.5).
 * rho and u as for Zou-He: a velocity face takes u_w and the density from the
 * known populations, a pressure face rho_w and the normal velocity from them.
 * The unknown populations get the non-equilibrium part of their opposite
 * (bounce-back of f - feq); then every population is rebuilt from the
 * equilibrium and the non-equilibrium momentum flux alone:
 *   f_i = feq_i(rho, u) + w_i / (2 cs^4) (c_i c_i - cs^2 I) : Pi_neq,
 *   Pi_neq = sum_i c_i c_i (f_i - feq_i),  cs^2 = 1/3. */
static void regularized_closure(const orc_sim *S, int face, double *f)
{
    int q = S->q;
    int n[3];
    inward_normal(face, n);
    const orc_face *F = &S->face[face];
    double sumZ = 0.0, sumO = 0.0;
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        int cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
        if (cn == 0) sumZ += f[i];
        if (cn == -1) sumO += f[i];
    }
    double rho, u[3];
    if (vel_face(F->type)) {
        double un = F->u[0] * n[0] + F->u[1] * n[1] + F->u[2] * n[2];
        rho = (sumZ + 2.0 * sumO) / (1.0 - un);
        for (int a = 0; a < 3; ++a) u[a] = F->u[a];
    } else {
        rho = F->rho;
        double un = 1.0 - (sumZ + 2.0 * sumO) / rho;
        for (int a = 0; a < 3; ++a) u[a] = un * n[a];
    }
    double fneq[27];
    for (int i = 0; i < q; ++i) fneq[i] = f[i] - feq_i(q, i, rho, u);
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        if (c[0] * n[0] + c[1] * n[1] + c[2] * n[2] == 1) fneq[i] = fneq[opposite(q, i)];
    }
    double Pi[3][3] = {{0.0}};
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi[a][b] += c[a] * c[b] * fneq[i];
    }
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        double qp = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) qp += (c[a] * c[b] - ((a == b) ? 1.0 / 3.0 : 0.0)) * Pi[a][b];
        f[i] = feq_i(q, i, rho, u) + 4.5 * weight(q, i) * qp;
    }
}

/* closure of an open velocity / pressure face, by its type */
static void open_closure(const orc_sim *S, int face, double *f)
{
    int t = S->face[face].type;
    if (t == ORC_REG_VEL || t == ORC_REG_PRES) regularized_closure(S, face, f);
    else zouhe_closure(S, face, f);
}

void orc_zouhe_closure(const orc_sim *S, int face, double *f) { open_closure(S, face, f); }

/* ---------------------------------------------------------------------------
 * One step f(t) -> f(t+1).
 *   1. moments and BGK collision at every fluid cell, then the optional partial
 *      bounce-back mix  f°_i = (1 - s) f*_i + s f_opp(i)  (pre-collision
 *      opposite population; Walsh, Burwinkle & Saar 2009 -- not in the paper);
 *   2. streaming by pull, f_i(x, t+1) = f°_i(x - c_i, t) for fluid sources;
 *   3. boundary fill for the other directions:
 *        wall / solid source : f_i = f°_opp(i)(x) + 6 w_i rho0 (c_i . u_w)
 *        outflow face        : f_i = feq_i(rho_face, u(x, t))
 *        Zou-He face         : closure above; on a perimeter cell (also on a
 *                              wall face) the equilibrium rule with
 *                              (rho0, u_in) or (rho_w, u(x, t)) instead.
 * work: caller-provided buffers of N*q (post-collision) and N*3 (velocity).
 * ------------------------------------------------------------------------- */
/* Streaming and boundary fill into fluid cell k (steps 2 and 3 up to the open-
 * face closure): out[i] = f_i(x, t+1) before the closure, with the unknowns of
 * an open face set to 0.  Returns the open face whose closure the cell takes,
 * or -1.  fpost: post-collision populations, vel: velocities of every cell. */
static int gather_cell(const orc_sim *S, long k, const double *fpost, const double *vel, double *out)
{
    const int q = S->q;
    int x[3];
    x[2] = (int)(k % S->nz);
    x[1] = (int)((k / S->nz) % S->ny);
    x[0] = (int)(k / ((long)S->nz * S->ny));
    const double *u_here = vel + (size_t)k * 3;
    int zh_face = -1;
    int perimeter = on_wall_face(S, x);
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        orc_src src = classify(S, x, c);
        switch (src.kind) {
        case SRC_FLUID:
            out[i] = fpost[src.cell * q + i];
            break;
        case SRC_WALL: {
            const int o = opposite(q, i);
            const double qv = S->qlink ? S->qlink[(size_t)k * q + o] : 0.0;
            if (src.wall_face < 0 && qv > 0.0) {
                /* a solid cell with a curved-wall link along c_o = -c_i */
                out[i] = bouzidi_fill(S, x, o, qv, fpost);
                break;
            }
            double cu = c[0] * src.uw[0] + c[1] * src.uw[1] + c[2] * src.uw[2];
            out[i] = fpost[(size_t)k * q + o] + 6.0 * weight(q, i) * S->rho0 * cu;
            break;
        }
        case SRC_OUTFLOW:
            out[i] = feq_i(q, i, S->face[src.face].rho, u_here);
            break;
        case SRC_ZOUHE: {
            const orc_face *F = &S->face[src.face];
            if (perimeter) {
                if (vel_face(F->type)) out[i] = feq_i(q, i, S->rho0, F->u);
                else out[i] = feq_i(q, i, F->rho, u_here);
            } else {
                out[i] = 0.0;          /* unknown: filled by the closure */
                zh_face = src.face;
            }
            break;
        }
        }
    }
    return zh_face;
}

static void step_impl(const orc_sim *S, const double *f, double *fn, double *fpost, double *vel)
{
    const int q = S->q;
    const long N = (long)S->nx * S->ny * S->nz;

#pragma omp parallel for schedule(static)
    for (long k = 0; k < N; ++k) {
        if (S->solid && S->solid[k]) continue;
        const double *fk = f + (size_t)k * q;
        double *fo = fpost + (size_t)k * q;
        double rho, u[3];
        collide_f(S, fk, fo, &rho, u, S->edm ? S->edm + (size_t)k * 3 : NULL);
        if (S->s) {
            double s = S->s[k];
            double mixed[27];
            for (int i = 0; i < q; ++i) mixed[i] = (1.0 - s) * fo[i] + s * fk[opposite(q, i)];
            for (int i = 0; i < q; ++i) fo[i] = mixed[i];
        }
        for (int a = 0; a < 3; ++a) vel[(size_t)k * 3 + a] = u[a];
    }

#pragma omp parallel for schedule(static)
    for (long k = 0; k < N; ++k) {
        double *out = fn + (size_t)k * q;
        if (S->solid && S->solid[k]) {
            for (int i = 0; i < q; ++i) out[i] = 0.0;   /* solid cells carry no state */
            continue;
        }
        int zh_face = gather_cell(S, k, fpost, vel, out);
        if (zh_face >= 0) open_closure(S, zh_face, out);
    }
}

int orc_run(const orc_sim *S, double *f, int nsteps)
{
    const long N = (long)S->nx * S->ny * S->nz;
    const size_t bytes = (size_t)N * S->q * sizeof(double);
    double *fn = (double *)malloc(bytes);
    double *fpost = (double *)malloc(bytes);
    double *vel = (double *)malloc((size_t)N * 3 * sizeof(double));
    if (!fn || !fpost || !vel) { free(fn); free(fpost); free(vel); return -1; }
    for (int t = 0; t < nsteps; ++t) {
        step_impl(S, f, fn, fpost, vel);
        memcpy(f, fn, bytes);
    }
    free(fn); free(fpost); free(vel);
    return 0;
}

/* f = feq(rho, u) at every cell; rho (N) and u (N*3, AoS) may be NULL for
 * rho = rho0, u = 0.  Solid cells are set to zero. */
void orc_init_equilibrium(const orc_sim *S, const double *rho, const double *u, double *f)
{
    const long N = (long)S->nx * S->ny * S->nz;
    for (long k = 0; k < N; ++k) {
        double r = rho ? rho[k] : S->rho0;
        double v[3] = {0.0, 0.0, 0.0};
        if (u) for (int a = 0; a < 3; ++a) v[a] = u[(size_t)k * 3 + a];
        for (int i = 0; i < S->q; ++i)
            f[(size_t)k * S->q + i] = (S->solid && S->solid[k]) ? 0.0 : feq_i(S->q, i, r, v);
    }
}

/* rho (N) and u (N*3, AoS) of the state f; solid cells report rho0 and 0. */
void orc_moments(const orc_sim *S, const double *f, double *rho, double *u)
{
    const long N = (long)S->nx * S->ny * S->nz;
    for (long k = 0; k < N; ++k) {
        double r, v[3];
        if (S->solid && S->solid[k]) { r = S->rho0; v[0] = v[1] = v[2] = 0.0; }
        else moments(S->q, f + (size_t)k * S->q, &r, v);
        rho[k] = r;
        for (int a = 0; a < 3; ++a) u[(size_t)k * 3 + a] = v[a];
    }
}

/* Kahan-summed mass, momentum (3) and kinetic energy 1/2 sum rho|u|^2 over
 * fluid cells: sums[5]. */
void orc_sums(const orc_sim *S, const double *f, double *sums)
{
    const long N = (long)S->nx * S->ny * S->nz;
    double s[5] = {0, 0, 0, 0, 0}, comp[5] = {0, 0, 0, 0, 0};
    for (long k = 0; k < N; ++k) {
        if (S->solid && S->solid[k]) continue;
        double r, v[3];
        moments(S->q, f + (size_t)k * S->q, &r, v);
        double term[5] = {r, r * v[0], r * v[1], r * v[2], 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2])};
        for (int m = 0; m < 5; ++m) {
            double yv = term[m] - comp[m];
            double tv = s[m] + yv;
            comp[m] = (tv - s[m]) - yv;
            s[m] = tv;
        }
    }
    for (int m = 0; m < 5; ++m) sums[m] = s[m];
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of one step (FP64).  Given the pre-collision state f(t) and
 * a_next = dL/df(t+1), accumulate a_out += dL/df(t) (through this step only)
 * and the parameter gradients:
 *   dLds[N]  += dL/ds(x)     (partial bounce-back fraction; needs S->s)
 *   *dLdtau  += dL/dtau
 *   dLduw[6*3] += dL/du_w for each face's wall velocity vector.
 *
 * Written as the literal transpose of step_impl, walked backwards and
 * scattered onto the sources:
 *   (3) closure: the Zou-He unknowns are an affine function of the known
 *       populations at the same cell; its coefficients are read off by
 *       evaluating the closure on unit vectors;
 *   (2) stream / fill: each destination slot sends its adjoint to the slot it
 *       was read from (fluid source, bounced own slot, or the velocity of the
 *       cell for equilibrium fills);
 *   (1) collision + mix: per cell, the explicit q x q Jacobian of
 *       f°(f) = (1-s)[f - (f - feq(rho(f), u(f)))/tau] + s f_opp
 *       (KBC: (1-s) f*(f) + s f_opp, f* the KBC collision, whose Jacobian
 *       and tau derivative are taken by the complex step).
 * work: N*q (adjoint of the gathered values), N*q (adjoint of f°), N*3
 * (adjoint of u(x,t)).
 * ------------------------------------------------------------------------- */
static void closure_matrix(const orc_sim *S, int face, double A[27][27], double b[27])
{
    /* column j: closure(e_j) - closure(0) for the unknown rows */
    int q = S->q;
    double base[27], e[27];
    for (int i = 0; i < q; ++i) base[i] = 0.0;
    zouhe_closure(S, face, base);
    for (int i = 0; i < q; ++i) b[i] = base[i];
    for (int j = 0; j < q; ++j) {
        for (int i = 0; i < q; ++i) e[i] = (i == j) ? 1.0 : 0.0;
        zouhe_closure(S, face, e);
        for (int i = 0; i < q; ++i) A[i][j] = e[i] - base[i];
    }
}

/* Jacobian d feq_i(rho(f), v(f)) / d f_j of the equilibrium at a cell whose
 * velocity argument is v = (j + F) / rho (F = 0: the cell's own velocity):
 * d feq_i / d rho at fixed v, plus d feq_i / d v . (c_j - v) / rho. */
static void feq_jacobian(int q, double rho, const double v[3], double out[27][27])
{
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int i = 0; i < q; ++i) {
        const int *c = cvec(q, i);
        double cv = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
        double d_rho = weight(q, i) * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
        double d_v[3];
        for (int a = 0; a < 3; ++a) d_v[a] = weight(q, i) * rho * (3.0 * c[a] + 9.0 * cv * c[a] - 3.0 * v[a]);
        for (int j = 0; j < q; ++j) {
            const int *cj = cvec(q, j);
            double x = d_rho;
            for (int a = 0; a < 3; ++a) x += d_v[a] * (cj[a] - v[a]) / rho;
            out[i][j] = x;
        }
    }
}

int orc_adjoint_step(const orc_sim *S, const double *f, const double *a_next, double *a_out,
                     double *dLds, double *dLdtau, double *dLduw, double *dLdF)
{
    const int q = S->q;
    const long N = (long)S->nx * S->ny * S->nz;
    double *ag = (double *)calloc((size_t)N * q, sizeof(double));
    double *apost = (double *)calloc((size_t)N * q, sizeof(double));
    double *au = (double *)calloc((size_t)N * 3, sizeof(double));
    double *fpost = (double *)malloc((size_t)N * q * sizeof(double));
    double *vel = (double *)malloc((size_t)N * 3 * sizeof(double));
    if (!ag || !apost || !au || !fpost || !vel) {
        free(ag); free(apost); free(au); free(fpost); free(vel); return -1;
    }
    double duw[18] = {0};

    /* recompute the forward quantities of this step */
    for (long k = 0; k < N; ++k) {
        if (S->solid && S->solid[k]) continue;
        double rho, u[3];
        collide(S, f + (size_t)k * q, fpost + (size_t)k * q, &rho, u);
        if (S->s) {
            double s = S->s[k], mixed[27];
            for (int i = 0; i < q; ++i)
                mixed[i] = (1.0 - s) * fpost[(size_t)k * q + i] + s * f[(size_t)k * q + opposite(q, i)];
            for (int i = 0; i < q; ++i) fpost[(size_t)k * q + i] = mixed[i];
        }
        for (int a = 0; a < 3; ++a) vel[(size_t)k * 3 + a] = u[a];
    }

    /* (3) transpose of the open-face closure.  Zou-He: unknowns i in U are
     * f_i = sum_j A_ij g_j + b_i over known j, so dL/dg_j += A_ij dL/df_i.
     * Regularized: every population is rewritten, f_i = R_i(g) over the known
     * g_j, and R is a polynomial of degree at most 2 in them (rho or u_n is
     * affine in g, the equilibrium quadratic in u, the rest linear), so the
     * central difference (R(g + e_j) - R(g - e_j)) / 2 is its exact derivative;
     * dL/dg_j = sum_i dR_i/dg_j dL/df_i, taken at this step's g (gather_cell
     * from the post-collision state). */
    for (long k = 0; k < N; ++k) {
        if (S->solid && S->solid[k]) continue;
        int x[3];
        x[2] = (int)(k % S->nz);
        x[1] = (int)((k / S->nz) % S->ny);
        x[0] = (int)(k / ((long)S->nz * S->ny));
        int perimeter = on_wall_face(S, x);
        int zh_face = -1, unknown[27];
        for (int i = 0; i < q; ++i) {
            orc_src src = classify(S, x, cvec(q, i));
            unknown[i] = (src.kind == SRC_ZOUHE && !perimeter);
            if (unknown[i]) zh_face = src.face;
        }
        const double *an = a_next + (size_t)k * q;
        double *g = ag + (size_t)k * q;
        for (int i = 0; i < q; ++i) g[i] = unknown[i] ? 0.0 : an[i];
        const int reg = zh_face >= 0 && (S->face[zh_face].type == ORC_REG_VEL || S->face[zh_face].type == ORC_REG_PRES);
        if (reg) {
            double g0[27], gp[27], gm[27];
            gather_cell(S, k, fpost, vel, g0);
            for (int j = 0; j < q; ++j) {
                if (unknown[j]) continue;
                for (int i = 0; i < q; ++i) gp[i] = gm[i] = g0[i];
                gp[j] += 1.0;
                gm[j] -= 1.0;
                open_closure(S, zh_face, gp);
                open_closure(S, zh_face, gm);
                double v = 0.0;
                for (int i = 0; i < q; ++i) v += 0.5 * (gp[i] - gm[i]) * an[i];
                g[j] = v;
            }
        } else if (zh_face >= 0) {
            double A[27][27], b[27];
            closure_matrix(S, zh_face, A, b);
            for (int i = 0; i < q; ++i) {
                if (!unknown[i]) continue;
                for (int j = 0; j < q; ++j)
                    if (!unknown[j]) g[j] += A[i][j] * an[i];
            }
        }
    }

    /* (2) transpose of stream + fill: scatter each destination's adjoint */
    for (long k = 0; k < N; ++k) {
        if (S->solid && S->solid[k]) continue;
        int x[3];
        x[2] = (int)(k % S->nz);
        x[1] = (int)((k / S->nz) % S->ny);
        x[0] = (int)(k / ((long)S->nz * S->ny));
        int perimeter = on_wall_face(S, x);
        const double *u_here = vel + (size_t)k * 3;
        for (int i = 0; i < q; ++i) {
            const int *c = cvec(q, i);
            double gi = ag[(size_t)k * q + i];
            orc_src src = classify(S, x, c);
            if (src.kind == SRC_FLUID) {
                apost[src.cell * q + i] += gi;
            } else if (src.kind == SRC_WALL) {
                apost[(size_t)k * q + opposite(q, i)] += gi;
                if (src.face >= 0)
                    for (int a = 0; a < 3; ++a) duw[3 * src.face + a] += gi * 6.0 * weight(q, i) * S->rho0 * c[a];
            } else {
                /* equilibrium fills depending on u(x,t): d feq_i / d u at fixed rho */
                int uses_u = 0;
                double rf = 0.0;
                if (src.kind == SRC_OUTFLOW) { uses_u = 1; rf = S->face[src.face].rho; }
                else if (perimeter && pres_face(S->face[src.face].type)) { uses_u = 1; rf = S->face[src.face].rho; }
                if (uses_u) {
                    double cu = c[0] * u_here[0] + c[1] * u_here[1] + c[2] * u_here[2];
                    for (int a = 0; a < 3; ++a) {
                        double d = weight(q, i) * rf * (3.0 * c[a] + 9.0 * cu * c[a] - 3.0 * u_here[a]);
                        au[(size_t)k * 3 + a] += gi * d;
                    }
                }
            }
        }
    }

    /* (1) transpose of collision + partial bounce-back, cell by cell */
    const double omega = 1.0 / S->tau;
    double dtau = 0.0;
    for (long k = 0; k < N; ++k) {
        if (S->solid && S->solid[k]) continue;
        const double *fk = f + (size_t)k * q;
        const double *ap = apost + (size_t)k * q;
        double rho, u[3];
        moments(q, fk, &rho, u);
        double s = S->s ? S->s[k] : 0.0;
        /* J_ij = d f°_i / d f_j; KBC: the collision's Jacobian jk and its
         * tau derivative dk by the complex step */
        double J[27][27];
        double dfeq[27][27], dfeqF[27][27], jk[27][27], dk[27];
        const int kbc = S->collision == 1;
        feq_jacobian(q, rho, u, dfeq);
        if (kbc) kbc_jacobian(q, fk, S->tau, jk, dk);
        /* body force (exact-difference method): f* gains feq(rho, u') - feq(rho, u),
         * u' = (j + F) / rho, whose Jacobian is that of feq at u' minus that at u */
        const double *F = S->edm ? S->edm + (size_t)k * 3 : NULL;
        double up[3] = {u[0], u[1], u[2]};
        if (F) {
            for (int a = 0; a < 3; ++a) up[a] = u[a] + F[a] / rho;
            feq_jacobian(q, rho, up, dfeqF);
        }
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j)
                J[i][j] = (1.0 - s) * ((kbc ? jk[i][j] : ((i == j) ? 1.0 : 0.0) * (1.0 - omega) + omega * dfeq[i][j])
                                       + (F ? dfeqF[i][j] - dfeq[i][j] : 0.0))
                          + s * ((j == opposite(q, i)) ? 1.0 : 0.0);
        double *ao = a_out + (size_t)k * q;
        for (int j = 0; j < q; ++j) {
            double v = 0.0;
            for (int i = 0; i < q; ++i) v += J[i][j] * ap[i];
            /* adjoint of u(x,t) used by equilibrium fills: du/df_j = (c_j - u)/rho */
            const int *cj = cvec(q, j);
            for (int a = 0; a < 3; ++a) v += au[(size_t)k * 3 + a] * (cj[a] - u[a]) / rho;
            ao[j] += v;
        }
        /* parameters */
        double fstar[27];
        if (kbc) {
            double feq[27];
            for (int i = 0; i < q; ++i) feq[i] = feq_i(q, i, rho, u);
            kbc_collide(q, fk, feq, S->tau, fstar);
        }
        for (int i = 0; i < q; ++i) {
            if (!kbc) fstar[i] = fk[i] - omega * (fk[i] - feq_i(q, i, rho, u));
            if (F) fstar[i] += feq_i(q, i, rho, up) - feq_i(q, i, rho, u);
        }
        /* d f°_i / d F = (1-s) d feq_i(rho, u') / d u' / rho */
        if (dLdF && F) {
            for (int i = 0; i < q; ++i) {
                const int *c = cvec(q, i);
                double cv = c[0] * up[0] + c[1] * up[1] + c[2] * up[2];
                for (int a = 0; a < 3; ++a)
                    dLdF[(size_t)k * 3 + a] += ap[i] * (1.0 - s) * weight(q, i) * (3.0 * c[a] + 9.0 * cv * c[a] - 3.0 * up[a]);
            }
        }
        if (dLds && S->s) {
            double g = 0.0;
            for (int i = 0; i < q; ++i) g += ap[i] * (fk[opposite(q, i)] - fstar[i]);
            dLds[k] += g;
        }
        /* d f°_i / d tau = (1-s) (f_i - feq_i) / tau^2 (BGK), (1-s) dk_i (KBC) */
        for (int i = 0; i < q; ++i)
            dtau += ap[i] * (1.0 - s) * (kbc ? dk[i] : (fk[i] - feq_i(q, i, rho, u)) / (S->tau * S->tau));
    }
    if (dLdtau) *dLdtau += dtau;
    if (dLduw) for (int m = 0; m < 18; ++m) dLduw[m] += duw[m];
    free(ag); free(apost); free(au); free(fpost); free(vel);
    return 0;
}

/*
 * Momentum-exchange force (Ladd 1994) of the step that produced f (= f(t+1)),
 * the drag / lift sums of the paper's obstacle flows (Sec. 4.3).  For every
 * fluid cell x and direction i whose neighbour x + c_i is a solid cell or
 * lies across a wall face, the post-collision population f°_i(x, t) left
 * along c_i and came back as f_opp(i)(x, t + 1) = f°_i + 6 w_opp rho0
 * (c_opp . u_w).  The fluid lost (f°_i + f_opp(i)(x, t + 1)) c_i of momentum
 * to that solid or wall; summed over links (Kahan, FP64):
 *   out[0..2]          force on the solid cells,
 *   out[3 + 3 f + a]   force on wall face f (a link across several wall faces
 *                      counts for the lowest-index one).
 */
void orc_forces(const orc_sim *S, const double *f, double *out)
{
    const int q = S->q;
    double s[21], comp[21];
    for (int k = 0; k < 21; ++k) s[k] = comp[k] = 0.0;
    int x[3];
    for (x[0] = 0; x[0] < S->nx; ++x[0])
        for (x[1] = 0; x[1] < S->ny; ++x[1])
            for (x[2] = 0; x[2] < S->nz; ++x[2]) {
                const size_t cell = cell_index(S, x);
                if (S->solid && S->solid[cell]) continue;
                for (int i = 1; i < q; ++i) {
                    const int *c = cvec(q, i);
                    const int o = opposite(q, i);
                    int mc[3] = {-c[0], -c[1], -c[2]};
                    const orc_src src = classify(S, x, mc);   /* the cell x + c_i */
                    if (src.kind != SRC_WALL) continue;
                    const int *co = cvec(q, o);
                    const double back = f[cell * q + o];       /* f_opp(i)(x, t + 1) */
                    const double term = 6.0 * weight(q, o) * S->rho0 *
                                        (co[0] * src.uw[0] + co[1] * src.uw[1] + co[2] * src.uw[2]);
                    const double ex = 2.0 * back - term;       /* f°_i + f_opp(i)(x, t + 1) */
                    const int base = (src.wall_face >= 0) ? 3 + 3 * src.wall_face : 0;
                    for (int a = 0; a < 3; ++a) {
                        const double y = ex * c[a] - comp[base + a];
                        const double t = s[base + a] + y;
                        comp[base + a] = (t - s[base + a]) - y;
                        s[base + a] = t;
                    }
                }
            }
    for (int k = 0; k < 21; ++k) out[k] = s[k];
}

/*
 * One step f(t) -> f(t+1), in place, and the momentum-exchange force of that
 * step in the form of Mei, Yu, Shyy & Luo (2002), which the paper cites for
 * its lift and drag (Sec. 4.3): over every link (x, i) from a fluid cell x to
 * a solid cell or across a wall face, the fluid loses (f°_i(x, t) +
 * f_opp(i)(x, t + 1)) c_i of momentum, where f° is the post-collision
 * population and f_opp(i)(x, t + 1) whatever the boundary rule filled in
 * (halfway or interpolated bounce-back).  out[21] as orc_forces.  With
 * halfway bounce-back only, this equals orc_forces of the new state.
 */
int orc_step_forces(const orc_sim *S, double *f, double *out)
{
    const int q = S->q;
    const long N = (long)S->nx * S->ny * S->nz;
    const size_t bytes = (size_t)N * q * sizeof(double);
    double *fn = (double *)malloc(bytes);
    double *fpost = (double *)malloc(bytes);
    double *vel = (double *)malloc((size_t)N * 3 * sizeof(double));
    if (!fn || !fpost || !vel) { free(fn); free(fpost); free(vel); return -1; }
    step_impl(S, f, fn, fpost, vel);
    double s[21], comp[21];
    for (int k = 0; k < 21; ++k) s[k] = comp[k] = 0.0;
    int x[3];
    for (x[0] = 0; x[0] < S->nx; ++x[0])
        for (x[1] = 0; x[1] < S->ny; ++x[1])
            for (x[2] = 0; x[2] < S->nz; ++x[2]) {
                const size_t cell = cell_index(S, x);
                if (S->solid && S->solid[cell]) continue;
                for (int i = 1; i < q; ++i) {
                    const int *c = cvec(q, i);
                    int mc[3] = {-c[0], -c[1], -c[2]};
                    const orc_src src = classify(S, x, mc);   /* the cell x + c_i */
                    if (src.kind != SRC_WALL) continue;
                    const double ex = fpost[cell * q + i] + fn[cell * q + opposite(q, i)];
                    const int base = (src.wall_face >= 0) ? 3 + 3 * src.wall_face : 0;
                    for (int a = 0; a < 3; ++a) {
                        const double y = ex * c[a] - comp[base + a];
                        const double t = s[base + a] + y;
                        comp[base + a] = (t - s[base + a]) - y;
                        s[base + a] = t;
                    }
                }
            }
    for (int k = 0; k < 21; ++k) out[k] = s[k];
    memcpy(f, fn, bytes);
    free(fn); free(fpost); free(vel);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the following calls use (timing of the oracle on one core and on
 * all cores; the result does not depend on it). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
