/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Plain FP64 CPU reference of one time step of the 16-velocity, third-order
 * isothermal lattice Boltzmann model with corner transport upwind advection of
 * Sofonea et al., arXiv:1802.01272.  Everything here is written for a reader
 * who checks it against the paper by eye: whole-field arrays, one quantity at
 * a time, in the order the paper introduces them, no blocking and no fusion.
 *
 * Readings of the paper taken here (the paper is silent, garbled or ambiguous):
 *  - A time step is the two-step split of Sec. II C: advection of f^n first
 *    (left-hand side of Eq. eBGK, by CTU1 or CTU2), then collision and force
 *    (right-hand side) evaluated on the advected state f*.  The apparent
 *    viscosities of Table apparentvisco, T (tau - dt/2) plus the numerical
 *    part, identify this order; an update with every term at level n would
 *    give T (tau + dt/2).
 *  - In the CTU2 limiter of S^y the printed ratio uses R^x; it is read as
 *    R^y_{i,j-s_y} / R^y_{i,j}, the symmetric counterpart of S^x.
 *  - In the transverse term of the x-flux the printed index pair of R^y is
 *    (i+(1-s_y)/2, j+(1-s_y)/2); it is read as (i+(1-s_x)/2, j+(1-s_y)/2), the
 *    pair used in the y-flux.  With the limiter switched off the flux form
 *    then reproduces Eq. (ctueq) exactly, which the tests check.
 *  - The limiter correction R*Psi(R_up/R) is taken as 0 when R = 0.
 *  - The 25-point stencils are not printed.  The gradient of (p^i - p^w) uses
 *    the fourth-order accurate isotropic gradient on the 5x5 block,
 *    grad phi = (1/ds) sum_e w(|e|^2) e phi(x + e) with w(1)=2/5, w(2)=7/45,
 *    w(4)=0, w(5)=-1/45, w(8)=1/720: the weights that make the stencil exact
 *    to fourth order, its fifth-order error isotropic and its seventh-order
 *    error free of the cos(4 theta) harmonic.  Along a lattice axis it is the
 *    classic fourth-order central difference (2/3, -1/12).  With it a relaxed
 *    flat interface at the parameters of Sec. III A has the printed surface
 *    tension and coexistence densities close to the Maxwell values (Sec. II E);
 *    second-order isotropic gradients leave the vapour density several percent
 *    low there.  kappa grad(lap rho) applies the 9-point isotropic gradient
 *    (w(1)=1/3, w(2)=1/12) to the 9-point isotropic Laplacian
 *    (4*sum_nn + sum_diag - 20*centre)/6, a 25-point composite.
 *  - a^(2) in the force term is the second Hermite moment of f itself.
 *  - Regularization replaces the advected f* by f^eq + fhat^neq at every node
 *    before the collision, so that f itself stays in the Hermite space of
 *    order <= 3.
 *  - Shear walls: ghost rows j = -2, -1 hold f^eq(rho_w, (-u_w, 0)) and rows
 *    j = Ly, Ly+1 hold f^eq(rho_w, (+u_w, 0)); x stays periodic.
 *  - The far-field clamp of Sec. III B is measured from the lattice centre
 *    ((Lx-1)/2, (Ly-1)/2), the centre of the bubbles, and applies to nodes
 *    strictly farther than the radius, after each step.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Velocity set: Table "roots".  The Cartesian components are the roots of the
 * Hermite polynomial He4(x) = x^4 - 6 x^2 + 3, i.e. +-sqrt(3 -+ sqrt(6)); the
 * weights are products of the 1D Gauss-Hermite weights (3 +- sqrt(6))/12,
 * which give (5 + 2 sqrt 6)/48, 1/48 and (5 - 2 sqrt 6)/48.                  */
void orc_velocity_set(double xi_x[16], double xi_y[16], double w[16])
{
    const double s6 = sqrt(6.0);
    const double q_small = sqrt(3.0 - s6), q_large = sqrt(3.0 + s6);
    /* group g: (|xi_x|, |xi_y|, weight) for k = 4g .. 4g+3 */
    const double gx[4] = {q_small, q_large, q_small, q_large};
    const double gy[4] = {q_small, q_small, q_large, q_large};
    const double gw[4] = {(5.0 + 2.0 * s6) / 48.0, 1.0 / 48.0, 1.0 / 48.0,
                          (5.0 - 2.0 * s6) / 48.0};
    /* sign pairs inside a group: (+,+), (-,+), (-,-), (+,-) */
    const double sx[4] = {1.0, -1.0, -1.0, 1.0};
    const double sy[4] = {1.0, 1.0, -1.0, -1.0};
    for (int g = 0; g < 4; ++g)
        for (int s = 0; s < 4; ++s) {
            int k = 4 * g + s;
            xi_x[k] = sx[s] * gx[g];
            xi_y[k] = sy[s] * gy[g];
            w[k] = gw[g];
        }
}

/* Eq. (herfeq): third-order Hermite equilibrium at reference temperature 1. */
void orc_feq(double T, double rho, double ux, double uy, double out[16])
{
    double xx[16], xy[16], w[16];
    orc_velocity_set(xx, xy, w);
    const double u2 = ux * ux + uy * uy;
    for (int k = 0; k < 16; ++k) {
        const double xu = xx[k] * ux + xy[k] * uy;
        const double xi2 = xx[k] * xx[k] + xy[k] * xy[k];
        const double second = 0.5 * (xu * xu - u2 + (T - 1.0) * (xi2 - 2.0));
        const double third = xu / 6.0 * (xu * xu - 3.0 * u2 + 3.0 * (T - 1.0) * (xi2 - 4.0));
        out[k] = w[k] * rho * (1.0 + xu + second + third);
    }
}

/* Eq. (herforce): w_k rho { xi.g + (xi.g)(xi.u) - g.u
 *                          + (1/(2 rho)) a2 : [ (xi.g) H2(xi) - 2 g xi ] }  */
void orc_force(double rho, double ux, double uy, double gx, double gy,
               const double a2[3], double out[16])
{
    double xx[16], xy[16], w[16];
    orc_velocity_set(xx, xy, w);
    /* a2 as a full symmetric 2x2 tensor */
    const double A[2][2] = {{a2[0], a2[1]}, {a2[1], a2[2]}};
    const double g[2] = {gx, gy};
    for (int k = 0; k < 16; ++k) {
        const double xi[2] = {xx[k], xy[k]};
        const double xg = xi[0] * gx + xi[1] * gy;
        const double xu = xi[0] * ux + xi[1] * uy;
        const double gu = gx * ux + gy * uy;
        double contraction = 0.0; /* a2_{ab} [ (xi.g) H2_{ab}(xi) - 2 g_a xi_b ] */
        for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) {
                const double H2 = xi[al] * xi[be] - (al == be ? 1.0 : 0.0);
                contraction += A[al][be] * (xg * H2 - 2.0 * g[al] * xi[be]);
            }
        out[k] = w[k] * rho * (xg + xg * xu - gu + contraction / (2.0 * rho));
    }
}

/* rho = sum f, u = sum f xi / rho (no force shift), a2 = sum f (xi xi - I). */
void orc_moments(const double f[16], double* rho, double* ux, double* uy,
                 double a2[3])
{
    double xx[16], xy[16], w[16];
    orc_velocity_set(xx, xy, w);
    double r = 0.0, jx = 0.0, jy = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0;
    for (int k = 0; k < 16; ++k) {
        r += f[k];
        jx += f[k] * xx[k];
        jy += f[k] * xy[k];
        pxx += f[k] * (xx[k] * xx[k] - 1.0);
        pxy += f[k] * (xx[k] * xy[k]);
        pyy += f[k] * (xy[k] * xy[k] - 1.0);
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
    if (a2) {
        a2[0] = pxx;
        a2[1] = pxy;
        a2[2] = pyy;
    }
}

/* Eq. (evdw) written for general constants: p^w = rho T / (1 - b rho) - a rho^2
 * (a = 9/8, b = 1/3 gives the paper's 3 rho T / (3 - rho) - 9/8 rho^2). */
double orc_pressure_vdw(double T, double a, double b, double rho)
{
    return rho * T / (1.0 - b * rho) - a * rho * rho;
}

/* Eq. (ereg): f <- f^eq + w_k [ (1/2!) H2(xi_k) : sum f^neq xi xi
 *                              + (1/3!) H3(xi_k) : sum f^neq xi xi xi ]      */
void orc_regularize_node(double T, double f[16])
{
    double xx[16], xy[16], w[16], feq[16], fneq[16];
    orc_velocity_set(xx, xy, w);
    double rho, ux, uy;
    orc_moments(f, &rho, &ux, &uy, NULL);
    orc_feq(T, rho, ux, uy, feq);
    for (int k = 0; k < 16; ++k) fneq[k] = f[k] - feq[k];

    double M2[2][2] = {{0}}, M3[2][2][2] = {{{0}}};
    for (int k = 0; k < 16; ++k) {
        const double xi[2] = {xx[k], xy[k]};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                M2[a][b] += fneq[k] * xi[a] * xi[b];
                for (int c = 0; c < 2; ++c) M3[a][b][c] += fneq[k] * xi[a] * xi[b] * xi[c];
            }
    }
    for (int k = 0; k < 16; ++k) {
        const double xi[2] = {xx[k], xy[k]};
        double h2 = 0.0, h3 = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const double dab = (a == b) ? 1.0 : 0.0;
                h2 += (xi[a] * xi[b] - dab) * M2[a][b];
                for (int c = 0; c < 2; ++c) {
                    const double dbc = (b == c) ? 1.0 : 0.0, dac = (a == c) ? 1.0 : 0.0;
                    const double H3 = xi[a] * xi[b] * xi[c] - (xi[a] * dbc + xi[b] * dac + xi[c] * dab);
                    h3 += H3 * M3[a][b][c];
                }
            }
        f[k] = feq[k] + w[k] * (h2 / 2.0 + h3 / 6.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Isotropic finite-difference stencils on an extended array.                */

/* weights of the fourth-order 5x5 gradient, indexed by |e|^2 (0 for unused):
 * sum w e_x^2 = 1, sum w e_x^4 = sum w e_x^2 e_y^2 = 0 (no third-order error),
 * sum w e_x^6 = 5 sum w e_x^4 e_y^2 (isotropic fifth-order error) and no
 * cos(4 theta) term in sum w |e|^8 cos^8(angle(e) - theta).                   */
static double w_grad5(int e2)
{
    switch (e2) {
    case 1: return 2.0 / 5.0;
    case 2: return 7.0 / 45.0;
    case 4: return 0.0;
    case 5: return -1.0 / 45.0;
    case 8: return 1.0 / 720.0;
    default: return 0.0;
    }
}
/* weights of the 8-neighbour gradient */
static double w_grad3(int e2)
{
    switch (e2) {
    case 1: return 1.0 / 3.0;
    case 2: return 1.0 / 12.0;
    default: return 0.0;
    }
}

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

void orc_grad5(int Lx, int Ly, double ds, const double* phi, double* gx, double* gy)
{
    for (int j = 0; j < Ly; ++j)
        for (int i = 0; i < Lx; ++i) {
            double sx = 0.0, sy = 0.0;
            for (int ey = -2; ey <= 2; ++ey)
                for (int ex = -2; ex <= 2; ++ex) {
                    const double wt = w_grad5(ex * ex + ey * ey);
                    const double v = phi[wrap(j + ey, Ly) * Lx + wrap(i + ex, Lx)];
                    sx += wt * ex * v;
                    sy += wt * ey * v;
                }
            gx[j * Lx + i] = sx / ds;
            gy[j * Lx + i] = sy / ds;
        }
}

void orc_grad3(int Lx, int Ly, double ds, const double* phi, double* gx, double* gy)
{
    for (int j = 0; j < Ly; ++j)
        for (int i = 0; i < Lx; ++i) {
            double sx = 0.0, sy = 0.0;
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex) {
                    const double wt = w_grad3(ex * ex + ey * ey);
                    const double v = phi[wrap(j + ey, Ly) * Lx + wrap(i + ex, Lx)];
                    sx += wt * ex * v;
                    sy += wt * ey * v;
                }
            gx[j * Lx + i] = sx / ds;
            gy[j * Lx + i] = sy / ds;
        }
}

void orc_lap3(int Lx, int Ly, double ds, const double* phi, double* lap)
{
    for (int j = 0; j < Ly; ++j)
        for (int i = 0; i < Lx; ++i) {
#define P(dx, dy) phi[wrap(j + (dy), Ly) * Lx + wrap(i + (dx), Lx)]
            const double nn = P(1, 0) + P(-1, 0) + P(0, 1) + P(0, -1);
            const double dg = P(1, 1) + P(-1, 1) + P(-1, -1) + P(1, -1);
            lap[j * Lx + i] = (4.0 * nn + dg - 20.0 * P(0, 0)) / (6.0 * ds * ds);
#undef P
        }
}

/* ------------------------------------------------------------------------ */
/* Advection of one velocity on an extended array.
 *
 * fE covers the extended box of nEx x nEy nodes; the output box is the inner
 * part [2, nEx-2) x [2, nEy-2).  A has (nEx-4)*(nEy-4) entries.            */

#define EIDX(ex, ey) ((size_t)(ey) * (size_t)nEx + (size_t)(ex))

static int sgn_of(double c) { return c >= 0.0 ? 1 : -1; } /* varsigma, with varsigma(0) = +1 */

/* Monotonized-centred limiter Psi(theta) = max(0, min((1+theta)/2, 2, 2 theta)) */
static double psi_mc(double theta)
{
    double m = (1.0 + theta) / 2.0;
    if (2.0 < m) m = 2.0;
    if (2.0 * theta < m) m = 2.0 * theta;
    return m > 0.0 ? m : 0.0;
}

/* R * Psi(R_up / R), taken as 0 for R = 0 */
static double limited(double R, double R_up)
{
    if (R == 0.0) return 0.0;
    return R * psi_mc(R_up / R);
}

/* Eq. (ctueq), literally. */
static void ctu1_literal(int nEx, int nEy, double ds, double dt, double cx, double cy,
                         const double* fE, double* A)
{
    const int sx = sgn_of(cx), sy = sgn_of(cy);
    const double ax = fabs(cx), ay = fabs(cy);
    const int nx = nEx - 4;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 2; ey < nEy - 2; ++ey)
        for (int ex = 2; ex < nEx - 2; ++ex) {
            const double v = fE[EIDX(ex, ey)] * (ds - ax * dt) * (ds - ay * dt)
                           + fE[EIDX(ex - sx, ey)] * ax * (ds - ay * dt) * dt
                           + fE[EIDX(ex, ey - sy)] * ay * (ds - ax * dt) * dt
                           + fE[EIDX(ex - sx, ey - sy)] * ax * ay * dt * dt;
            A[(size_t)(ey - 2) * nx + (ex - 2)] = v / (ds * ds);
        }
}

/* CTU2 in the flux form of Sec. II C 2 (with the readings listed above). */
static void ctu2_flux(int nEx, int nEy, double ds, double dt, double cx, double cy,
                      int use_limiter, const double* fE, double* A)
{
    const int sx = sgn_of(cx), sy = sgn_of(cy);
    const double nu = dt / ds;
    const size_t n = (size_t)nEx * nEy;
    double* Rx = calloc(n, sizeof(double));
    double* Ry = calloc(n, sizeof(double));
    double* Sx = calloc(n, sizeof(double));
    double* Sy = calloc(n, sizeof(double));
    double* Fx = calloc(n, sizeof(double)); /* F_{ex+1/2, ey} */
    double* Gy = calloc(n, sizeof(double)); /* G_{ex, ey+1/2} */

    /* R^x_{i,j} = f_{i,j} - f_{i-1,j},  R^y_{i,j} = f_{i,j} - f_{i,j-1} */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 0; ey < nEy; ++ey)
        for (int ex = 1; ex < nEx; ++ex) Rx[EIDX(ex, ey)] = fE[EIDX(ex, ey)] - fE[EIDX(ex - 1, ey)];
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 1; ey < nEy; ++ey)
        for (int ex = 0; ex < nEx; ++ex) Ry[EIDX(ex, ey)] = fE[EIDX(ex, ey)] - fE[EIDX(ex, ey - 1)];

    /* S^x_{i,j} = 1/2 |c_x| (1 - nu |c_x|) R^x_{i,j} Psi(R^x_{i-s_x,j} / R^x_{i,j}), same for y */
    const double kx = 0.5 * fabs(cx) * (1.0 - nu * fabs(cx));
    const double ky = 0.5 * fabs(cy) * (1.0 - nu * fabs(cy));
    if (use_limiter) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
        for (int ey = 0; ey < nEy; ++ey)
            for (int ex = 1; ex < nEx; ++ex) {
                const int eu = ex - sx;
                if (eu < 1 || eu >= nEx) continue;
                Sx[EIDX(ex, ey)] = kx * limited(Rx[EIDX(ex, ey)], Rx[EIDX(eu, ey)]);
            }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
        for (int ey = 1; ey < nEy; ++ey)
            for (int ex = 0; ex < nEx; ++ex) {
                const int eu = ey - sy;
                if (eu < 1 || eu >= nEy) continue;
                Sy[EIDX(ex, ey)] = ky * limited(Ry[EIDX(ex, ey)], Ry[EIDX(ex, eu)]);
            }
    }

    const int hx = (1 - sx) / 2, hy = (1 - sy) / 2; /* I = i + hx, J = j + hy */
    /* F_{i+1/2,j} = c_x f_{I,j} + S^x_{i+1,j} - 1/2 nu c_x c_y R^y_{I,J}
     *             + nu c_x (S^y_{I,j} - S^y_{I,j+1})                        */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 2; ey < nEy - 2; ++ey)
        for (int ex = 1; ex < nEx - 2; ++ex) {
            const int I = ex + hx, J = ey + hy;
            Fx[EIDX(ex, ey)] = cx * fE[EIDX(I, ey)] + Sx[EIDX(ex + 1, ey)]
                             - 0.5 * nu * cx * cy * Ry[EIDX(I, J)]
                             + nu * cx * (Sy[EIDX(I, ey)] - Sy[EIDX(I, ey + 1)]);
        }
    /* G_{i,j+1/2} = c_y f_{i,J} + S^y_{i,j+1} - 1/2 nu c_x c_y R^x_{I,J}
     *             + nu c_y (S^x_{i,J} - S^x_{i+1,J})                        */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 1; ey < nEy - 2; ++ey)
        for (int ex = 2; ex < nEx - 2; ++ex) {
            const int I = ex + hx, J = ey + hy;
            Gy[EIDX(ex, ey)] = cy * fE[EIDX(ex, J)] + Sy[EIDX(ex, ey + 1)]
                             - 0.5 * nu * cx * cy * Rx[EIDX(I, J)]
                             + nu * cy * (Sx[EIDX(ex, J)] - Sx[EIDX(ex + 1, J)]);
        }
    /* f - nu [F_{i+1/2} - F_{i-1/2} + G_{j+1/2} - G_{j-1/2}] */
    const int nx = nEx - 4;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 2; ey < nEy - 2; ++ey)
        for (int ex = 2; ex < nEx - 2; ++ex)
            A[(size_t)(ey - 2) * nx + (ex - 2)] =
                fE[EIDX(ex, ey)] - nu * (Fx[EIDX(ex, ey)] - Fx[EIDX(ex - 1, ey)]
                                         + Gy[EIDX(ex, ey)] - Gy[EIDX(ex, ey - 1)]);
    free(Rx); free(Ry); free(Sx); free(Sy); free(Fx); free(Gy);
}

void orc_advect(int Lx, int Ly, double ds, double dt, double cx, double cy,
                int scheme, int limiter, const double* in, double* out)
{
    const int nEx = Lx + 4, nEy = Ly + 4;
    double* fE = malloc(sizeof(double) * (size_t)nEx * nEy);
    for (int ey = 0; ey < nEy; ++ey)
        for (int ex = 0; ex < nEx; ++ex)
            fE[EIDX(ex, ey)] = in[(size_t)wrap(ey - 2, Ly) * Lx + wrap(ex - 2, Lx)];
    if (scheme == 1) ctu1_literal(nEx, nEy, ds, dt, cx, cy, fE, out);
    else ctu2_flux(nEx, nEy, ds, dt, cx, cy, limiter, fE, out);
    free(fE);
}

/* ------------------------------------------------------------------------ */
/* Whole step.                                                               */

/* f_k at lattice node (i, j) including ghost rows; ghost[0..15] bottom,
 * ghost[16..31] top. */
static double f_at(const orc_params* p, const double* f, const double* ghost, int k, int i, int j)
{
    const int Lx = p->Lx, Ly = p->Ly;
    i = wrap(i, Lx);
    if (p->bc_y == 0) j = wrap(j, Ly);
    else if (j < 0) return ghost[k];
    else if (j >= Ly) return ghost[16 + k];
    return f[((size_t)k * Ly + j) * Lx + i];
}

void orc_init(const orc_params* p, const double* rho, const double* ux,
              const double* uy, double* f)
{
    const size_t N = (size_t)p->Lx * p->Ly;
    for (size_t n = 0; n < N; ++n) {
        double fe[16];
        orc_feq(p->T, rho[n], ux[n], uy[n], fe);
        for (int k = 0; k < 16; ++k) f[(size_t)k * N + n] = fe[k];
    }
}

int orc_step_region(const orc_params* p, const double* f_in,
                    int i0, int i1, int j0, int j1, double* out)
{
    if (p->Lx < 1 || p->Ly < 1 || i1 <= i0 || j1 <= j0) return -1;
    if (p->bc_y == 1 && (j0 < 0 || j1 > p->Ly)) return -1;
    double xx[16], xy[16], w[16];
    orc_velocity_set(xx, xy, w);
    const double T = p->T, ds = p->ds, dt = p->dt;

    /* ghost rows of the shear walls: f^eq(rho_w, -+u_w) */
    double ghost[32];
    orc_feq(T, p->rho_wall, -p->u_wall, 0.0, ghost);
    orc_feq(T, p->rho_wall, +p->u_wall, 0.0, ghost + 16);

    const int nx = i1 - i0, ny = j1 - j0;
    const int nEx = nx + 4, nEy = ny + 4;          /* region + 2: stencil reach  */
    const int nGx = nx + 8, nGy = ny + 8;          /* region + 4: + advection    */
    const size_t nE = (size_t)nEx * nEy, nR = (size_t)nx * ny;
    const size_t nG = (size_t)nGx * nGy;

    /* 1. gather f^n on the box extended by four nodes */
    double* fG = malloc(sizeof(double) * 16 * nG);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nGx * (size_t)nGy > 16384)
#endif
    for (int gy = 0; gy < nGy; ++gy)
        for (int gx = 0; gx < nGx; ++gx) {
            const int i = i0 + gx - 4, j = j0 + gy - 4;
            for (int k = 0; k < 16; ++k)
                fG[(size_t)k * nG + (size_t)gy * nGx + gx] = f_at(p, f_in, ghost, k, i, j);
        }

    /* 2. first step of the split: advection, f* = A_k(f^n), on the box
     *    extended by two.  Ghost rows of the walls are boundary values and keep
     *    their state.  Regularization (Eq. ereg) then replaces f* by
     *    f^eq + fhat^neq at every lattice node. */
    double* fE = malloc(sizeof(double) * 16 * nE);
    for (int k = 0; k < 16; ++k) {
        if (p->scheme == 1) ctu1_literal(nGx, nGy, ds, dt, xx[k], xy[k], fG + (size_t)k * nG, fE + (size_t)k * nE);
        else ctu2_flux(nGx, nGy, ds, dt, xx[k], xy[k], p->limiter, fG + (size_t)k * nG, fE + (size_t)k * nE);
    }
    free(fG);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 0; ey < nEy; ++ey)
        for (int ex = 0; ex < nEx; ++ex) {
            const int j = j0 + ey - 2;
            const int is_ghost = (p->bc_y == 1) && (j < 0 || j >= p->Ly);
            double fn[16];
            if (is_ghost) {
                for (int k = 0; k < 16; ++k) fn[k] = ghost[(j < 0 ? 0 : 16) + k];
            } else {
                for (int k = 0; k < 16; ++k) fn[k] = fE[(size_t)k * nE + EIDX(ex, ey)];
                if (p->regularize) orc_regularize_node(T, fn);
            }
            for (int k = 0; k < 16; ++k) fE[(size_t)k * nE + EIDX(ex, ey)] = fn[k];
        }

    /* 2. moments on the extended box */
    double* rho = malloc(sizeof(double) * nE);
    double* ux = malloc(sizeof(double) * nE);
    double* uy = malloc(sizeof(double) * nE);
    double* a2 = malloc(sizeof(double) * 3 * nE);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 0; ey < nEy; ++ey)
        for (int ex = 0; ex < nEx; ++ex) {
            const size_t e = EIDX(ex, ey);
            double fn[16];
            for (int k = 0; k < 16; ++k) fn[k] = fE[(size_t)k * nE + e];
            orc_moments(fn, &rho[e], &ux[e], &uy[e], &a2[3 * e]);
            if (p->a2_eq) {
                a2[3 * e + 0] = rho[e] * (ux[e] * ux[e] + (T - 1.0));
                a2[3 * e + 1] = rho[e] * (ux[e] * uy[e]);
                a2[3 * e + 2] = rho[e] * (uy[e] * uy[e] + (T - 1.0));
            }
        }

    /* 3. Eq. (eder): g = grad(p^i - p^w) / rho + kappa grad(lap rho) */
    double* phi = malloc(sizeof(double) * nE);
    double* lap = calloc(nE, sizeof(double));
    for (size_t e = 0; e < nE; ++e) phi[e] = rho[e] * T - orc_pressure_vdw(T, p->a, p->b, rho[e]);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 1; ey < nEy - 1; ++ey)
        for (int ex = 1; ex < nEx - 1; ++ex) {
#define RH(dx, dy) rho[EIDX(ex + (dx), ey + (dy))]
            const double nn = RH(1, 0) + RH(-1, 0) + RH(0, 1) + RH(0, -1);
            const double dg = RH(1, 1) + RH(-1, 1) + RH(-1, -1) + RH(1, -1);
            lap[EIDX(ex, ey)] = (4.0 * nn + dg - 20.0 * RH(0, 0)) / (6.0 * ds * ds);
#undef RH
        }
    double* gx = malloc(sizeof(double) * nR);
    double* gy = malloc(sizeof(double) * nR);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 2; ey < nEy - 2; ++ey)
        for (int ex = 2; ex < nEx - 2; ++ex) {
            double px = 0.0, py = 0.0, lx = 0.0, ly = 0.0;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    const double wt = w_grad5(dx * dx + dy * dy);
                    px += wt * dx * phi[EIDX(ex + dx, ey + dy)];
                    py += wt * dy * phi[EIDX(ex + dx, ey + dy)];
                }
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const double wt = w_grad3(dx * dx + dy * dy);
                    lx += wt * dx * lap[EIDX(ex + dx, ey + dy)];
                    ly += wt * dy * lap[EIDX(ex + dx, ey + dy)];
                }
            const size_t r = (size_t)(ey - 2) * nx + (ex - 2);
            const double rc = rho[EIDX(ex, ey)];
            gx[r] = (px / ds) / rc + p->kappa * (lx / ds);
            gy[r] = (py / ds) / rc + p->kappa * (ly / ds);
        }

    /* 4. second step of the split: collision and force on the advected state,
     *    f^{n+1} = f* - dt/tau (f* - f^eq(f*)) + dt F_k(f*) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if ((size_t)nEx * (size_t)nEy > 16384)
#endif
    for (int ey = 2; ey < nEy - 2; ++ey)
        for (int ex = 2; ex < nEx - 2; ++ex) {
            const size_t e = EIDX(ex, ey), r = (size_t)(ey - 2) * nx + (ex - 2);
            double feq[16], F[16];
            orc_feq(T, rho[e], ux[e], uy[e], feq);
            orc_force(rho[e], ux[e], uy[e], gx[r], gy[r], &a2[3 * e], F);
            for (int k = 0; k < 16; ++k) {
                const double fk = fE[(size_t)k * nE + e];
                out[(size_t)k * nR + r] = fk - dt / p->tau * (fk - feq[k]) + dt * F[k];
            }
        }

    /* 5. far-field density (Sec. III B): outside the circle of radius
     *    clamp_radius about the lattice centre, f is rescaled by rho_ext / rho */
    if (p->clamp_radius > 0.0) {
        const double cx = 0.5 * (p->Lx - 1), cy = 0.5 * (p->Ly - 1);
        const double r2 = p->clamp_radius * p->clamp_radius;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double dx = (i0 + x) - cx, dy = (j0 + y) - cy;
                if (dx * dx + dy * dy <= r2) continue;
                const size_t r = (size_t)y * nx + x;
                double rho_n = 0.0;
                for (int k = 0; k < 16; ++k) rho_n += out[(size_t)k * nR + r];
                for (int k = 0; k < 16; ++k) out[(size_t)k * nR + r] *= p->clamp_rho / rho_n;
            }
    }

    free(fE); free(rho); free(ux); free(uy); free(a2);
    free(phi); free(lap); free(gx); free(gy);
    return 0;
}

int orc_step(const orc_params* p, const double* f_in, double* f_out)
{
    return orc_step_region(p, f_in, 0, p->Lx, 0, p->Ly, f_out);
}

int orc_run(const orc_params* p, double* f, int64_t nsteps)
{
    const size_t n = (size_t)16 * p->Lx * p->Ly;
    double* tmp = malloc(sizeof(double) * n);
    if (!tmp) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (orc_step(p, f, tmp) != 0) { free(tmp); return -1; }
        memcpy(f, tmp, sizeof(double) * n);
    }
    free(tmp);
    return 0;
}

void orc_field_moments(const orc_params* p, const double* f, double* rho,
                       double* ux, double* uy)
{
    const size_t N = (size_t)p->Lx * p->Ly;
    for (size_t n = 0; n < N; ++n) {
        double fn[16];
        for (int k = 0; k < 16; ++k) fn[k] = f[(size_t)k * N + n];
        orc_moments(fn, &rho[n], &ux[n], &uy[n], NULL);
    }
}

void orc_reduce(const orc_params* p, const double* f, double threshold,
                double stats[11])
{
    double xx[16], xy[16], w[16];
    orc_velocity_set(xx, xy, w);
    const int Lx = p->Lx, Ly = p->Ly;
    const size_t N = (size_t)Lx * Ly;
    for (int s = 0; s < 11; ++s) stats[s] = 0.0;
    const double cxn = 0.5 * (Lx - 1), cyn = 0.5 * (Ly - 1);
    for (int j = 0; j < Ly; ++j)
        for (int i = 0; i < Lx; ++i) {
            const size_t n = (size_t)j * Lx + i;
            double rho = 0.0, jx = 0.0, jy = 0.0;
            int finite = 1;
            for (int k = 0; k < 16; ++k) {
                const double v = f[(size_t)k * N + n];
                if (!isfinite(v)) finite = 0;
                rho += v;
                jx += v * xx[k];
                jy += v * xy[k];
            }
            stats[0] += rho;
            stats[1] += jx;
            stats[2] += jy;
            if (!finite) stats[4] += 1.0;
            if (rho < threshold) {
                const double x = i - cxn, y = j - cyn;
                stats[3] += 1.0;
                stats[5] += x;
                stats[6] += y;
                stats[7] += x * x;
                stats[8] += x * y;
                stats[9] += y * y;
            }
        }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
