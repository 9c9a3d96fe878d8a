/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Plain, slow, FP64 CPU reference of the time step of the third-order
 * isothermal two-dimensional lattice Boltzmann model with 16 off-lattice
 * velocities and corner transport upwind (CTU) advection of
 *   V. Sofonea, T. Biciusca, S. Busuioc, V. E. Ambrus, G. Gonnella, A. Lamura,
 *   "Corner transport upwind lattice Boltzmann model for bubble cavitation",
 *   arXiv:1802.01272 (Phys. Rev. E 97, 023309, 2018).
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
 * load this library.  It shares no code, header, table or helper with the HIP
 * library under paper_1802_01272_amd/.
 *
 * Layout of a distribution field: f[(k * Ly + j) * Lx + i], k = 0..15 in the
 * order of the velocity table (Table "roots"; within each group of four the
 * sign pairs (+,+), (-,+), (-,-), (+,-)), node (i, j) at x = i*ds, y = j*ds.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t Lx, Ly;     /* nodes along x and y                                   */
    double ds, dt;      /* lattice spacing and time step                         */
    double tau;         /* BGK relaxation time                                   */
    double T;           /* temperature                                           */
    double a, b;        /* van der Waals constants, p = rho T/(1-b rho) - a rho^2 */
    double kappa;       /* surface-tension parameter in g                         */
    int32_t scheme;     /* 1 = CTU1 (Eq. ctueq), 2 = CTU2 (flux form, MC limiter)  */
    int32_t regularize; /* 1 = project f onto Hermite order <= 3 each step        */
    int32_t bc_y;       /* 0 = periodic in y, 1 = shear walls (ghost rows)        */
    double u_wall;      /* wall speed u_w: bottom ghost rows -u_w, top +u_w       */
    double rho_wall;    /* density of the ghost rows                              */
    int32_t limiter;    /* CTU2 only: 1 = MC limiter, 0 = limiter identically 0   */
    int32_t a2_eq;      /* 0 = a2 of f itself (literal), 1 = equilibrium a2       */
    double clamp_radius; /* > 0: nodes farther than this from the lattice centre
                            are rescaled to density clamp_rho after the step    */
    double clamp_rho;
} orc_params;

/* Velocity set and weights (Table "roots"). */
void orc_velocity_set(double xi_x[16], double xi_y[16], double w[16]);

/* Equilibrium, Eq. (herfeq). */
void orc_feq(double T, double rho, double ux, double uy, double out[16]);

/* Force term, Eq. (herforce); a2 = {a2_xx, a2_xy, a2_yy}. */
void orc_force(double rho, double ux, double uy, double gx, double gy,
               const double a2[3], double out[16]);

/* Density, velocity and the second Hermite moment a2 = sum_k f_k (xi xi - I). */
void orc_moments(const double f[16], double* rho, double* ux, double* uy,
                 double a2[3]);

/* van der Waals pressure, Eq. (evdw) with general a, b. */
double orc_pressure_vdw(double T, double a, double b, double rho);

/* Regularized replacement of one node: f <- f^eq + fhat^neq, Eq. (ereg). */
void orc_regularize_node(double T, double f[16]);

/* Stencils on a periodic Lx x Ly scalar field (unit spacing ds). */
void orc_grad5(int Lx, int Ly, double ds, const double* phi, double* gx, double* gy);
void orc_grad3(int Lx, int Ly, double ds, const double* phi, double* gx, double* gy);
void orc_lap3(int Lx, int Ly, double ds, const double* phi, double* lap);

/* Pure advection of one periodic scalar field by velocity (cx, cy) over one
 * step: scheme 1 = Eq. (ctueq) literally, 2 = CTU2 flux form (limiter flag). */
void orc_advect(int Lx, int Ly, double ds, double dt, double cx, double cy,
                int scheme, int limiter, const double* in, double* out);

/* f = f^eq(rho, u) at every node (initial state). */
void orc_init(const orc_params* p, const double* rho, const double* ux,
              const double* uy, double* f);

/* One full time step, f_in -> f_out (both 16*Lx*Ly): advection of f_in,
 * then collision and force on the advected state (Sec. II C). Returns 0 or -1. */
int orc_step(const orc_params* p, const double* f_in, double* f_out);

/* Several steps; f is updated in place. Returns 0 or -1. */
int orc_run(const orc_params* p, double* f, int64_t nsteps);

/* One step restricted to nodes (i, j) in [i0,i1) x [j0,j1); out has
 * 16*(i1-i0)*(j1-j0) entries laid out [k][j-j0][i-i0]. */
int orc_step_region(const orc_params* p, const double* f_in,
                    int i0, int i1, int j0, int j1, double* out);

/* Moments at every node (density and velocity u = sum f xi / rho). */
void orc_field_moments(const orc_params* p, const double* f, double* rho,
                       double* ux, double* uy);

/* Diagnostics: sums over the lattice. stats[0..10] =
 * mass, mom_x, mom_y, n_bubble, n_nonfinite, sx, sy, sxx, sxy, syy, (unused)
 * with bubble = {rho < threshold}; positions in node units relative to
 * ((Lx-1)/2, (Ly-1)/2). */
void orc_reduce(const orc_params* p, const double* f, double threshold,
                double stats[11]);

/* Number of OpenMP threads the oracle uses (1 if built without OpenMP). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
