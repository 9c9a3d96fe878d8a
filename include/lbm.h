/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann stepper.
 *
 * The library advances the 16 distribution functions f_k of the third-order
 * isothermal two-dimensional lattice Boltzmann model of
 *   V. Sofonea, T. Biciusca, S. Busuioc, V. E. Ambrus, G. Gonnella, A. Lamura,
 *   "Corner transport upwind lattice Boltzmann model for bubble cavitation",
 *   arXiv:1802.01272 (Phys. Rev. E 97, 023309, 2018)
 * by the two-step explicit split of Sec. II C per time increment: advection
 * first, then collision and force on the advected state,
 *   f*_k = A_k(f^n),   f_k^{n+1} = f*_k - (dt/tau)(f*_k - f_k^eq(f*)) + dt F_k(f*),
 * with the velocity set of Table "roots", the Hermite equilibrium of Eq.
 * (herfeq), the force term of Eq. (herforce) driven by the van der Waals
 * acceleration of Eq. (eder), the optional regularization of Eq. (ereg), and
 * the first- (Eq. ctueq) or second-order (Sec. II C 2) corner transport
 * upwind advection A_k.  Every step of the computation runs in the library's
 * own HIP kernels on the device; the host side only validates, carves the
 * workspace and launches.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Node (i, j), 0 <= i < Lx, 0 <= j < Ly, sits at x = i*ds, y = j*ds.  x is
 *    always periodic; y is periodic or bounded by the shear walls of Sec. III C.
 *  - Velocity k = 0..15 follows Table "roots" (groups of four: |xi| =
 *    (q-, q-), (q+, q-), (q-, q+), (q+, q+) with q-+ = sqrt(3 -+ sqrt 6)); inside
 *    a group the sign pairs are (+,+), (-,+), (-,-), (+,-).
 *  - A distribution field handed across the ABI is FP64, laid out
 *    f[(k * Ly + j) * Lx + i].  Scalar fields are [j * Lx + i].
 *  - Arguments named h_* are host pointers, d_* device pointers.  The caller
 *    owns all buffers, including the device workspace; the library owns only
 *    the small host-side handles it returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls documented "async" only enqueue work on it; calls documented
 *    "sync" wait for it before returning.
 *  - Every call returns an lbm_status; on failure lbm_last_error() gives a
 *    message (thread-local).  No exception crosses the ABI.  A device fault
 *    raised by asynchronous work is reported by the next synchronous call.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument or parameter                          */
    LBM_ECFL = -2,        /* CFL condition of Sec. II C 1 violated               */
    LBM_ENOMEM = -3,      /* workspace smaller than lbm_workspace_bytes()        */
    LBM_EDEVICE = -4,     /* HIP runtime error or device fault                   */
    LBM_ENONFINITE = -5,  /* non-finite distributions found by lbm_reduce        */
    LBM_ESTATE = -6       /* call not valid in the handle's current state        */
} lbm_status;

enum { LBM_FP64 = 0, LBM_FP32_DEV = 1 };     /* storage precision               */
enum { LBM_PERIODIC = 0, LBM_SHEAR_WALLS = 1 }; /* boundary in y                 */
enum { LBM_ROUND_STOCHASTIC = 0, LBM_ROUND_NEAREST = 1 }; /* FP32 storage rounding */
enum { LBM_PAIR = 0 };  /* waves_per_group of lbm_set_launch: see there          */
enum { LBM_BATCH_PER_STEP = 0, LBM_BATCH_PERSISTENT = 1 }; /* lbm_batch_set_mode    */

/* Parameters of one run.  Names follow the paper (Sec. II and III). */
typedef struct {
    int32_t Lx, Ly;       /* lattice nodes along x and y, each >= 1; Lx * Ly
                             (Lx * (Ly + 2) with walls) at most 2^26 (8192 x
                             8192) with FP32 storage, at most 2^26 - 1 with
                             FP64 storage (eight FP64 planes must span fewer
                             than 2^32 bytes)                                  */
    double ds, dt;        /* lattice spacing and time step; CFL of Sec. II C 1:
                             dt * sqrt(3 + sqrt 6) <= ds                       */
    double tau;           /* BGK relaxation time, > 0 (Eq. eBGK)                */
    double T;             /* temperature, > 0 (reference temperature 1)          */
    double a, b;          /* van der Waals constants: p^w = rho T/(1 - b rho)
                             - a rho^2 (Eq. evdw is a = 9/8, b = 1/3; a = b = 0
                             with kappa = 0 is the ideal gas, g = 0)             */
    double kappa;         /* surface-tension parameter of Eq. (eder), >= 0       */
    int32_t scheme;       /* 1 = CTU1, 2 = CTU2 with the MC limiter              */
    int32_t regularize;   /* 0/1: replace the advected f* by f^eq + fhat^neq
                             before the collision, Eq. (ereg)                  */
    int32_t precision;    /* LBM_FP64, or LBM_FP32_DEV: f_k - w_k rho_ref stored
                             and advected in FP32                                */
    double rho_ref;       /* rho_ref of the FP32 deviation storage, > 0          */
    int32_t bc_y;         /* LBM_PERIODIC or LBM_SHEAR_WALLS                     */
    double u_wall;        /* shear walls: ghost rows j = -2,-1 hold
                             f^eq(rho_wall, (-u_wall, 0)), rows Ly, Ly+1 hold
                             f^eq(rho_wall, (+u_wall, 0)) (Sec. III C)           */
    double rho_wall;
    double clamp_radius;  /* > 0: after every step, each node farther than
                             clamp_radius nodes from ((Lx-1)/2, (Ly-1)/2) has
                             its f_k rescaled to density clamp_rho (the fixed
                             far-field density of Sec. III B); <= 0: off      */
    double clamp_rho;     /* density imposed outside the circle, in (0, 1/b) */
    int32_t rounding;     /* LBM_FP32_DEV only: how each new f_k - w_k rho_ref,
                             computed in FP64, is rounded to FP32.
                             LBM_ROUND_STOCHASTIC (0, the default): up or down
                             with probabilities that make the stored value
                             unbiased, so storage errors do not accumulate
                             coherently over many steps; deterministic, from
                             a hash of the run's step count and the node's own
                             values.  LBM_ROUND_NEAREST: to nearest, ties to
                             even.  Ignored for LBM_FP64.                       */
} lbm_params;

/* FP64 diagnostics of one state (Sec. III C).  Bubble = nodes with
 * rho < threshold; positions in node units relative to ((Lx-1)/2, (Ly-1)/2). */
typedef struct {
    double mass, mom_x, mom_y;       /* sum rho, sum rho u (device FP64 sums)  */
    int64_t n_bubble, n_nonfinite;   /* bubble node count N_b; nodes with a
                                        non-finite f_k                          */
    double sx, sy, sxx, sxy, syy;    /* sums of x, y, xx, xy, yy over bubble    */
    /* derived on the host from the sums above: */
    double cx, cy;                   /* bubble centre                           */
    double Txx, Txy, Tyy;            /* gyration tensor, Eq. (gyr)              */
    double a, b;                     /* 2 sqrt(Lambda_max), 2 sqrt(Lambda_min)  */
    double D;                        /* (a - b)/(a + b)                         */
    double theta;                    /* angle of the major axis to x, (-pi/2, pi/2] */
    double A_rel;                    /* N_b / (Lx Ly)                           */
    double R_eq;                     /* ds sqrt(N_b / pi)                       */
} lbm_stats;

typedef struct lbm_run lbm_run;
typedef struct lbm_batch lbm_batch;

/* Library version string (static storage). */
const char* lbm_version(void);

/* Message of the last failed call on this thread (static storage). */
const char* lbm_last_error(void);

/* Host-only check of a parameter set (no device call).  LBM_ECFL when
 * dt * max|xi_k,alpha| > ds, LBM_EINVAL for any other violation. */
lbm_status lbm_validate(const lbm_params* p);

/* Device bytes a run needs (two distribution fields plus reduction and
 * coefficient scratch); 0 if the parameters are invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Start a run in the caller's device workspace d_ws (>= lbm_workspace_bytes,
 * 256-byte aligned) from f = f^eq(rho0, u0) at every node (Eq. herfeq).
 * h_rho0, h_ux0, h_uy0: host arrays of Lx*Ly doubles; rho0 must be finite, > 0
 * and < 1/b.  sync.  On success *out receives a handle (free with
 * lbm_destroy); the workspace must stay allocated while the handle lives. */
lbm_status lbm_init(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream,
                    const double* h_rho0, const double* h_ux0, const double* h_uy0,
                    lbm_run** out);

/* As lbm_init with device arrays d_rho0, d_ux0, d_uy0 (Lx*Ly doubles each,
 * values are not checked).  async. */
lbm_status lbm_init_device(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream,
                           const double* d_rho0, const double* d_ux0, const double* d_uy0,
                           lbm_run** out);

/* Re-open a workspace that holds the state of a run after `step` steps (a
 * checkpoint taken by copying the workspace).  The distribution fields are
 * not touched; the coefficient block and the step counter that seeds the
 * stochastic rounding are rewritten from p and step, so a reopened run
 * continues exactly as the original would.  The parameters must equal those
 * the state was created with. */
lbm_status lbm_attach(const lbm_params* p, void* d_ws, size_t ws_bytes, int64_t step,
                      lbm_run** out);

/* Advance nsteps >= 0 time steps of the split scheme of Sec. II C: each
 * step advects every f_k with CTU1 (Eq. ctueq) or CTU2 (Sec. II C 2, MC
 * limiter), optionally regularizes the advected state (Eq. ereg), then
 * applies the BGK collision toward f^eq (Eq. herfeq) and the force term
 * (Eq. herforce) with g from Eqs. (eder)/(evdw) on the advected density;
 * with shear walls the ghost rows keep f^eq(rho_wall, -+u_wall) (Sec. III C),
 * with clamp_radius > 0 the far field is rescaled (Sec. III B).  Kernels are
 * queued on `stream`; the run must not be stepped from two streams at once.
 * LBM_EINVAL for a null run or nsteps < 0, LBM_ESTATE for a member of a
 * batch (those advance with lbm_batch_step), LBM_EDEVICE on a launch
 * failure.  async. */
lbm_status lbm_step(lbm_run* run, int64_t nsteps, void* stream);

/* Advance nsteps and measure the device time between HIP events recorded
 * on `stream` around the launches; *ms receives the elapsed milliseconds.
 * sync. */
lbm_status lbm_step_timed(lbm_run* run, int64_t nsteps, void* stream, double* ms);

/* Steps taken since lbm_init (or the `step` given to lbm_attach). */
int64_t lbm_step_count(const lbm_run* run);

/* Density rho = sum_k f_k and velocity u = sum_k f_k xi_k / rho (no force
 * shift; the moments of Eq. herfeq) of the current state into host arrays of
 * Lx*Ly doubles, row-major (index j * Lx + i).  LBM_EINVAL for null
 * arguments.  sync. */
lbm_status lbm_moments(lbm_run* run, double* h_rho, double* h_ux, double* h_uy, void* stream);

/* As lbm_moments into device arrays.  async. */
lbm_status lbm_moments_device(lbm_run* run, double* d_rho, double* d_ux, double* d_uy, void* stream);

/* Copy the current state out as FP64 (16*Lx*Ly doubles; in FP32_DEV mode
 * f_k = w_k rho_ref + stored deviation).  sync. */
lbm_status lbm_get_f(lbm_run* run, double* h_f, void* stream);

/* Replace the current state by an FP64 field (16*Lx*Ly doubles; FP32_DEV
 * stores f_k - w_k rho_ref rounded to FP32).  Non-finite values are accepted
 * and reported by lbm_reduce.  sync. */
lbm_status lbm_set_f(lbm_run* run, const double* h_f, void* stream);

/* Device-pointer versions of lbm_get_f / lbm_set_f.  async. */
lbm_status lbm_get_f_device(lbm_run* run, double* d_f, void* stream);
lbm_status lbm_set_f_device(lbm_run* run, const double* d_f, void* stream);

/* FP64 diagnostics of the current state (Sec. III C, Eq. gyr): device sums
 * with wavefront reductions, then the 2x2 eigen-analysis on the host.
 * Returns LBM_ENONFINITE (with *out filled) when n_nonfinite > 0.  sync. */
lbm_status lbm_reduce(lbm_run* run, double rho_threshold, lbm_stats* out, void* stream);

/* The current distribution field of a run, in the library's storage layout:
 * 16 planes of *plane_stride values each, plane k at d_f + k * plane_stride
 * values; within a plane node (i, j) at j * Lx + i, followed with shear walls
 * by the two ghost rows (row Ly: below the lattice, row Ly + 1: above).  FP64
 * values f_k for LBM_FP64 storage, FP32 deviations f_k - w_k rho_ref for
 * LBM_FP32_DEV.  The pointer lies inside the run's workspace and changes with
 * every step (two fields alternate). */
lbm_status lbm_state_device(const lbm_run* run, const void** d_f, int64_t* plane_stride);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): the diagnostics of
 * lbm_reduce for a distribution field d_f the caller holds in the storage
 * layout of lbm_state_device for parameters p (validated as lbm_validate
 * does), without a run handle or a workspace.  It allocates nothing: the
 * partial sums, results and coefficient block live in a fixed device array of
 * the library (about 168 KiB per GPU, 2048 workgroups' partials whatever the
 * lattice size, kept until the process ends); every lattice lbm_validate
 * accepts fits (at most 2^26 nodes per plane), larger ones are rejected with
 * LBM_EINVAL.  All calls on one GPU share that array: calls that overlap in
 * time on one GPU (from several host threads or streams) race and must be
 * serialised by the caller.  Nothing in it needs clearing between calls.
 * Same results, bit for bit, as lbm_reduce on a run holding the same field.
 * sync. */
lbm_status lbm_reduce_field_static(const lbm_params* p, const void* d_f, double rho_threshold, lbm_stats* out,
                                  void* stream);

/* Launch shape: rows of the lattice each strip of 56 columns advances per
 * workgroup (>= 1), and waves_per_group: 1 or 2 wavefronts per workgroup,
 * each marching its own strip (the step kernels keep 32 KiB of LDS per
 * wavefront; 4 is refused), or LBM_PAIR (FP32 storage only): a workgroup of
 * two wavefronts per strip, one advecting and one colliding, which share the
 * advected rows through LDS (each role needs few enough registers for two
 * wavefronts per SIMD).  LBM_EINVAL otherwise, and the previous shape is kept.
 * Defaults come from lbm_autotune or a built-in table (FP32: LBM_PAIR with
 * 32 rows). */
lbm_status lbm_set_launch(lbm_run* run, int32_t rows_per_wave, int32_t waves_per_group);
lbm_status lbm_get_launch(const lbm_run* run, int32_t* rows_per_wave, int32_t* waves_per_group);

/* Time each candidate launch shape for a run with parameters p on a
 * synthetic state held in d_ws (>= lbm_workspace_bytes(p); its contents are
 * overwritten) and return the fastest: rows per chunk from 8 to 512, and
 * waves_per_group 1, 2 or (FP32 storage) LBM_PAIR; 2 + steps_per_trial steps
 * per candidate.  Runs with p's shape created later in the process start
 * with the result.  sync. */
lbm_status lbm_autotune(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream,
                        int32_t steps_per_trial, int32_t* rows_per_wave, int32_t* waves_per_group);

/* Release a run handle (the workspace is the caller's). */
void lbm_destroy(lbm_run* run);

/* ---------------------------------------------------------------------- */
/* Batched runs: n independent runs of arbitrary sizes and parameters that
 * advance together over a shared work list of (run, strip, chunk) items,
 * one grouped launch per time step or one persistent launch for many steps
 * (lbm_batch_set_mode), the launches captured once in a HIP graph and
 * replayed.  All runs must share `precision`, `scheme` and `regularize`. */

size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params* params);

/* h_rho0[r], h_ux0[r], h_uy0[r]: host arrays of Lx_r*Ly_r doubles.  sync. */
lbm_status lbm_batch_init(int32_t n, const lbm_params* params, void* d_ws, size_t ws_bytes,
                          void* stream, const double* const* h_rho0,
                          const double* const* h_ux0, const double* const* h_uy0,
                          lbm_batch** out);

/* Advance every run by nsteps.  graph_steps > 0 captures that many steps in
 * one HIP graph on first use and replays it; 0 launches directly.  async. */
lbm_status lbm_batch_step(lbm_batch* batch, int64_t nsteps, int32_t graph_steps, void* stream);

/* Rows of each run that one work item advances (>= 1) for every run of the
 * batch; rebuilds the work list and drops a captured graph.  FP32 batches
 * run a pair of wavefronts per work item (as LBM_PAIR), FP64 batches one
 * wavefront.  sync. */
lbm_status lbm_batch_set_launch(lbm_batch* batch, int32_t rows_per_wave, void* stream);

/* Time candidate rows-per-item values on the batch itself and keep the
 * fastest: first one value for every run (10 candidates, in each launch
 * mode the batch can use: both for FP32 storage, whose mode is then set to
 * the faster one), then, for each class of runs of one lattice shape and
 * boundary condition (largest total node count first), up to 4 other
 * values for that class alone, kept when they save more than 1%.  The choice for each class is remembered for the
 * process: later lbm_batch_init calls start runs of the same shape,
 * precision, scheme, regularize and boundary from it.  *rows_per_wave
 * receives the common value of the first pass.  The trials advance every
 * run: by (steps_per_trial + 1) steps per candidate, and persistent-launch
 * trials by at least 17 (one launch of 16 or more steps).  sync. */
lbm_status lbm_batch_autotune(lbm_batch* batch, int32_t steps_per_trial, void* stream,
                              int32_t* rows_per_wave);

/* Alternative names of the two batch calls: lbm_init_batch is
 * lbm_batch_init; lbm_step_batch advances every run by nsteps, replaying a
 * captured graph of LBM_BATCH_GRAPH_STEPS steps (lbm_batch_step with that
 * graph_steps).  async. */
enum { LBM_BATCH_GRAPH_STEPS = 20 };
lbm_status lbm_init_batch(int32_t n, const lbm_params* params, void* d_ws, size_t ws_bytes,
                          void* stream, const double* const* h_rho0,
                          const double* const* h_ux0, const double* const* h_uy0,
                          lbm_batch** out);
lbm_status lbm_step_batch(lbm_batch* batch, int64_t nsteps, void* stream);

/* How a batch advances (Sec. III: the paper's runs are independent lattices;
 * batching them is this library's own scheduling).
 * LBM_BATCH_PER_STEP (the default): one grouped launch per time step over
 * the work list.  LBM_BATCH_PERSISTENT (FP32 storage only): one launch runs
 * up to 64 steps of every run; each work item of step s starts as soon as
 * the items around it (within the 4-row / 4-column reach of one step) have
 * finished step s - 1, instead of at a launch boundary, so no run waits for
 * the slowest item of the step.  Field accesses of that launch are
 * device-coherent; results are bit-identical to LBM_BATCH_PER_STEP.  Drops a
 * captured graph.  LBM_EINVAL for an unknown mode or PERSISTENT with FP64
 * storage.  sync. */
lbm_status lbm_batch_set_mode(lbm_batch* batch, int32_t mode, void* stream);
/* The batch's current mode, or -1 for a null batch. */
int32_t lbm_batch_get_mode(const lbm_batch* batch);

/* Bound, in polls, of each dependency wait of the persistent launch (0 =
 * the default, 2^22 polls: several seconds).  A wait that exceeds it sets
 * the batch's error word and lets the launch finish with invalid results, so
 * a launch never hangs; lbm_batch_sync_status reports it.  Drops a captured
 * graph.  sync. */
lbm_status lbm_batch_set_wait_limit(lbm_batch* batch, uint32_t polls, void* stream);

/* Wait for `stream`, then report the batch's error word: LBM_EDEVICE (and
 * the word cleared) if a persistent launch since the last check gave up a
 * dependency wait, in which case the states of every run are invalid;
 * LBM_OK otherwise.  sync. */
lbm_status lbm_batch_sync_status(lbm_batch* batch, void* stream);

/* Borrowed handle of run r (valid while the batch lives) for lbm_moments,
 * lbm_get_f, lbm_set_f and lbm_reduce; lbm_step on it is rejected. */
lbm_run* lbm_batch_run(lbm_batch* batch, int32_t r);

void lbm_batch_destroy(lbm_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
