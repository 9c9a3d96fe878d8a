// lbm_internal.hpp -- definitions shared by the HIP kernels and the host side
// of the library (not part of the public ABI in include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Velocity set of Table "roots": Cartesian components are +-QS or +-QL, the
// roots of He4(x) = x^4 - 6x^2 + 3 (QS = sqrt(3 - sqrt 6), QL = sqrt(3 + sqrt 6)).
// Group g = k / 4 fixes the magnitudes, s = k % 4 the signs
// (+,+), (-,+), (-,-), (+,-).
constexpr double QS = 0.74196378430272585764851359672636;
constexpr double QL = 2.33441421833897723931751226721036;
constexpr double W_SS = 0.20622873928263242075822016977941;  // (5 + 2 sqrt 6)/48
constexpr double W_SL = 0.02083333333333333333333333333333;  // 1/48
constexpr double W_LL = 0.00210459405070091257511316355392;  // (5 - 2 sqrt 6)/48

__host__ __device__ constexpr double group_qx(int g) { return (g == 0 || g == 2) ? QS : QL; }
__host__ __device__ constexpr double group_qy(int g) { return (g < 2) ? QS : QL; }
__host__ __device__ constexpr double group_w(int g) { return g == 0 ? W_SS : (g == 3 ? W_LL : W_SL); }
__host__ __device__ constexpr int sign_x(int k) { return ((k & 3) == 0 || (k & 3) == 3) ? 1 : -1; }
__host__ __device__ constexpr int sign_y(int k) { return ((k & 3) < 2) ? 1 : -1; }
__host__ __device__ constexpr double xi_x(int k) { return sign_x(k) * group_qx(k >> 2); }
__host__ __device__ constexpr double xi_y(int k) { return sign_y(k) * group_qy(k >> 2); }
__host__ __device__ constexpr double weight(int k) { return group_w(k >> 2); }

// Output columns per wavefront: 64 lanes minus a 4-lane halo on each side
// (advection reaches two columns, the force stencils on the advected density
// two more).
constexpr int WAVE = 64;
constexpr int HALO = 4;
constexpr int STRIP = WAVE - 2 * HALO;

// The step kernels hold the advected rows that wait for their collision (a
// ring of four rows of 16 FP64 values per lane, indexed by the row phase) in
// LDS: 32 KiB per wavefront.
constexpr int PENDING_ROWS = 4;
constexpr size_t STEP_LDS_PER_WAVE = (size_t)PENDING_ROWS * 16 * WAVE * sizeof(double);
// a pair of wavefronts per strip (advecting and colliding) shares one such
// ring and a ring of the advected rows' densities
constexpr size_t PAIR_STEP_LDS = STEP_LDS_PER_WAVE + (size_t)PENDING_ROWS * WAVE * sizeof(double);

// ---------------------------------------------------------------------------
// Per-run coefficients, prepared on the host in the storage precision R and
// read by the kernels through uniform (scalar) loads.
template <typename R>
struct StepCoef {
    // advection, in the storage precision R, indexed by the magnitude class m
    // of a velocity component (0: |xi| = QS, 1: |xi| = QL); nu = dt/ds
    R nu_xi[2];    // nu |xi|                            (CTU1 weights)
    // CTU2: the limited corrections are kept unscaled, X' = S^x / k2[mx] and
    // Y' = S^y / k2[my] with k2 = |xi| (1 - nu |xi|); the scales are folded
    // into the blend weights of their differences, indexed [mx][my]:
    R xs1[2][2];   // -nu (1 - nu |xi_y|) k2[mx]   weight of dX at the output row
    R xs2[2][2];   // -nu  nu |xi_y|      k2[mx]   weight of dX at the row upwind in y
    R ys1[2][2];   // -nu (1 - nu |xi_x|) k2[my]   weight of dY at the output column
    R ys2[2][2];   // -nu  nu |xi_x|      k2[my]   weight of dY at the column upwind in x
    R ghost_lo[16], ghost_hi[16];          // stored values of the two wall ghost-row states
    // node-local terms, always FP64
    double rho0;        // rho_ref (deviation storage) or 0
    double T, Tm1;      // T and T - 1
    double a_vdw, b_vdw;
    double kappa_ds;    // kappa / ds
    double inv_ds;      // 1 / ds
    double inv_6ds2;    // 1 / (6 ds^2)
    double dt_tau;      // dt / tau
    double dt;
    double ghost_rho_lo, ghost_rho_hi;  // density of the ghost rows (sum of their f)
    // far-field clamp: nodes with (i - cx)^2 + (j - cy)^2 > r2 are rescaled to
    // density clamp_rho after the step
    double clamp_r2, clamp_cx, clamp_cy, clamp_rho;
    int32_t walls;
    int32_t clamp;
    // FP32 storage rounding: 2^29 - 1 stochastic, 0 to nearest
    uint32_t sr_mask;
};

// magnitude class of the x / y component of velocity k
__host__ __device__ constexpr int mag_x(int k) { return ((k >> 2) == 1 || (k >> 2) == 3) ? 1 : 0; }
__host__ __device__ constexpr int mag_y(int k) { return (k >> 2) >= 2 ? 1 : 0; }

// One run as the step kernels see it.
template <typename R>
struct RunView {
    const R* f_in;
    R* f_out;
    const StepCoef<R>* coef;
    uint32_t* seq;      // step counter pair of the stochastic rounding
    int32_t cur;        // f_in is field cur: the step reads seq[cur]
    int32_t Lx, Ly;
    int32_t rows;       // rows per wavefront
    int32_t nstrips;    // wavefront strips along x
    int64_t plane;      // stride of one distribution plane: Lx * Ly, plus two
                        // ghost rows (Lx * (Ly + 2)) with shear walls
};

// Work item of the batched launch.
struct BatchItem {
    int32_t run, strip, chunk, pad_;
};

template <typename R>
struct BatchRun {
    R* f[2];
    const StepCoef<R>* coef;
    uint32_t* seq;      // the run's step counter pair
    int32_t Lx, Ly;
    int32_t rows, nstrips;
    int64_t plane;
    int32_t walls;      // shear walls (1) or periodic in y (0)
    int32_t item_base;  // index of the run's first work item; its items
                        // follow chunk by chunk, strip by strip
};

// Launch shape of the step kernel.
struct Launch {
    int32_t rows_per_wave;
    int32_t waves_per_group;
};

// Host launchers (lbm_kernels.hip).
template <typename R>
hipError_t launch_step(const RunView<R>& rv, int scheme, int regularize, int walls, int waves_per_group,
                       hipStream_t s);
// wmode: 0 = every item periodic, 1 = every item with walls, 2 = mixed (each
// item takes its run's boundary)
template <typename R>
hipError_t launch_batch_step(const BatchRun<R>* d_runs, const StepCoef<R>* d_coefs,
                             const BatchItem* d_items, int32_t nitems, int32_t cur, int scheme,
                             int regularize, int wmode, int waves_per_group, hipStream_t s);
// Persistent batched launch (FP32 storage only): nsteps steps of every run
// from parity cur0 in one launch of at most max_groups workgroups, after a
// reset of *ticket and done[0..nitems); *err is set (and left set) when a
// dependency wait exceeds wait_limit polls.  The runs' step counters are
// moved on by a second kernel.
template <typename R>
hipError_t launch_batch_persistent(const BatchRun<R>* d_runs, int32_t nruns, const StepCoef<R>* d_coefs,
                                   const BatchItem* d_items, int32_t nitems, int32_t cur0, int32_t nsteps,
                                   int scheme, int regularize, int wmode, uint32_t* ticket, int32_t* done,
                                   uint32_t* err, uint32_t wait_limit, hipStream_t s);

template <typename R>
hipError_t launch_init(R* f, const StepCoef<R>* coef, const double* rho, const double* ux,
                       const double* uy, int64_t n, int64_t plane, hipStream_t s);
template <typename R>
hipError_t launch_fill_ghost(R* f, const StepCoef<R>* coef, int32_t Lx, int32_t Ly, int64_t plane,
                             hipStream_t s);
template <typename R>
hipError_t launch_moments(const R* f, const StepCoef<R>* coef, double* rho, double* ux, double* uy,
                          int64_t n, int64_t plane, hipStream_t s);
template <typename R>
hipError_t launch_get_plane(const R* f, const StepCoef<R>* coef, int k, double* out, int64_t n,
                            int64_t plane, hipStream_t s);
template <typename R>
hipError_t launch_set_plane(R* f, const StepCoef<R>* coef, int k, const double* in, int64_t n,
                            int64_t plane, hipStream_t s);
template <typename R>
hipError_t launch_reduce(const R* f, const StepCoef<R>* coef, int32_t Lx, int32_t Ly, int64_t plane,
                         double threshold, double* partials, int32_t max_blocks, double* result,
                         hipStream_t s);

constexpr int REDUCE_VALUES = 10;
constexpr int REDUCE_MAX_BLOCKS = 2048;

}  // namespace lbm
