/* The CPU oracle under AddressSanitizer and UBSan (test infrastructure).
 * Runs every entry point of the oracle on small and ragged lattices with
 * every option (CTU1/CTU2, limiter on/off, regularization, walls, far-field
 * clamp, both a2 readings), including a 1 x 1 and a 1 x n lattice, and
 * checks that the results are finite.  Exits 0 when all hold. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static int failures = 0;

static void check(int cond, const char* what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static int all_finite(const double* v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* deterministic pseudo-random numbers in [0, 1) */
static unsigned long long state = 88172645463325252ull;
static double uniform(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static void one_case(int Lx, int Ly, int scheme, int limiter, int reg, int walls, int clamp, int a2_eq)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.Lx = Lx;
    p.Ly = Ly;
    p.ds = 1.0;
    p.dt = 0.25;
    p.tau = 0.7;
    p.T = 0.95;
    p.a = 9.0 / 8.0;
    p.b = 1.0 / 3.0;
    p.kappa = 1.0;
    p.scheme = scheme;
    p.limiter = limiter;
    p.regularize = reg;
    p.bc_y = walls;
    p.u_wall = walls ? 0.02 : 0.0;
    p.rho_wall = 1.3;
    p.a2_eq = a2_eq;
    p.clamp_radius = clamp ? 0.3 * (Lx < Ly ? Lx : Ly) : 0.0;
    p.clamp_rho = 1.3;
    const size_t n = (size_t)Lx * Ly;
    double* rho = malloc(n * sizeof *rho);
    double* ux = malloc(n * sizeof *ux);
    double* uy = malloc(n * sizeof *uy);
    double* f = malloc(16 * n * sizeof *f);
    double* g = malloc(16 * n * sizeof *g);
    for (size_t i = 0; i < n; ++i) {
        rho[i] = 1.2 + 0.2 * uniform();
        ux[i] = 0.05 * (uniform() - 0.5);
        uy[i] = 0.05 * (uniform() - 0.5);
    }
    orc_init(&p, rho, ux, uy, f);
    check(all_finite(f, 16 * n), "init");
    check(orc_step(&p, f, g) == 0 && all_finite(g, 16 * n), "step");
    check(orc_run(&p, g, 3) == 0 && all_finite(g, 16 * n), "run");
    /* a region touching both corners */
    {
        const int i0 = Lx > 2 ? 1 : 0, i1 = Lx, j0 = 0, j1 = Ly > 3 ? Ly - 1 : Ly;
        const size_t m = (size_t)(i1 - i0) * (j1 - j0);
        double* out = malloc(16 * m * sizeof *out);
        check(orc_step_region(&p, f, i0, i1, j0, j1, out) == 0 && all_finite(out, 16 * m), "step region");
        free(out);
    }
    orc_field_moments(&p, g, rho, ux, uy);
    check(all_finite(rho, n) && all_finite(ux, n) && all_finite(uy, n), "moments");
    double stats[11];
    orc_reduce(&p, g, 1.25, stats);
    check(all_finite(stats, 10), "reduce");
    /* stencils and pure advection on the density field */
    double* gx = malloc(n * sizeof *gx);
    double* gy = malloc(n * sizeof *gy);
    orc_grad5(Lx, Ly, 1.0, rho, gx, gy);
    check(all_finite(gx, n) && all_finite(gy, n), "grad5");
    orc_grad3(Lx, Ly, 1.0, rho, gx, gy);
    check(all_finite(gx, n) && all_finite(gy, n), "grad3");
    orc_lap3(Lx, Ly, 1.0, rho, gx);
    check(all_finite(gx, n), "lap3");
    orc_advect(Lx, Ly, 1.0, 0.25, 0.7, -1.3, scheme, limiter, rho, gy);
    check(all_finite(gy, n), "advect");
    free(gx);
    free(gy);
    free(rho);
    free(ux);
    free(uy);
    free(f);
    free(g);
}

int main(void)
{
    double xi_x[16], xi_y[16], w[16], feq[16], force[16], a2[3] = {0.01, -0.02, 0.03};
    orc_velocity_set(xi_x, xi_y, w);
    orc_feq(0.9, 1.1, 0.05, -0.02, feq);
    orc_force(1.1, 0.05, -0.02, 0.001, -0.002, a2, force);
    check(all_finite(feq, 16) && all_finite(force, 16), "node functions");
    double r, u, v, a2o[3];
    orc_moments(feq, &r, &u, &v, a2o);
    check(isfinite(r) && isfinite(u) && isfinite(v) && all_finite(a2o, 3), "node moments");
    orc_regularize_node(0.9, feq);
    check(all_finite(feq, 16), "regularize node");
    check(isfinite(orc_pressure_vdw(0.9, 9.0 / 8.0, 1.0 / 3.0, 1.5)), "pressure");
    const int sizes[][2] = {{1, 1}, {1, 7}, {7, 1}, {5, 6}, {13, 9}, {24, 17}};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s)
        for (int scheme = 1; scheme <= 2; ++scheme)
            for (int reg = 0; reg <= 1; ++reg)
                for (int walls = 0; walls <= 1; ++walls)
                    one_case(sizes[s][0], sizes[s][1], scheme, (int)(s & 1) ^ 1, reg, walls, (int)(s % 3 == 2),
                             (int)(s == 4));
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
