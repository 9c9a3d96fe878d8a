// lbm_api.hip -- host side of the C ABI declared in include/lbm.h:
// parameter validation, workspace carving, coefficient tables, launches,
// diagnostics, the launch-shape autotuner and batched runs with HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

thread_local std::string g_error;

lbm_status fail(lbm_status s, const std::string& msg)
{
    g_error = msg;
    return s;
}

lbm_status hip_fail(hipError_t e, const char* what)
{
    return fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool is_finite_d(double v) { return std::isfinite(v); }

// f^eq of Eq. (herfeq) on the host, used for the wall ghost rows.
double feq_host(int k, double T, double rho, double ux, double uy)
{
    const double cx = xi_x(k), cy = xi_y(k);
    const double xu = cx * ux + cy * uy, u2 = ux * ux + uy * uy, x2 = cx * cx + cy * cy;
    return weight(k) * rho
         * (1.0 + xu + 0.5 * (xu * xu - u2 + (T - 1.0) * (x2 - 2.0))
            + xu / 6.0 * (xu * xu - 3.0 * u2 + 3.0 * (T - 1.0) * (x2 - 4.0)));
}

lbm_status validate(const lbm_params* p)
{
    if (!p) return fail(LBM_EINVAL, "null parameters");
    if (p->Lx < 1 || p->Ly < 1) return fail(LBM_EINVAL, "Lx and Ly must be >= 1");
    // one buffer descriptor spans eight distribution planes: at most 2^26
    // nodes per plane (32-bit buffer offsets), and the eight planes must end
    // below the descriptor's 2^32 - 1 byte range (FP64: fewer than 2^26 nodes)
    {
        const int64_t plane = (int64_t)p->Lx * ((int64_t)p->Ly + (p->bc_y == LBM_SHEAR_WALLS ? 2 : 0));
        const int64_t sb = (p->precision == LBM_FP32_DEV) ? 4 : 8;
        if (plane > (int64_t)1 << 26 || 8 * plane * sb > ((int64_t)1 << 32) - 1)
            return fail(LBM_EINVAL, "Lx * Ly (Lx * (Ly + 2) with walls) must not exceed 2^26 nodes with FP32 "
                                    "storage and 2^26 - 1 with FP64 storage");
    }
    const double vals[] = {p->ds, p->dt, p->tau, p->T, p->a, p->b, p->kappa, p->rho_ref, p->u_wall, p->rho_wall,
                           p->clamp_radius, p->clamp_rho};
    for (double v : vals)
        if (!is_finite_d(v)) return fail(LBM_EINVAL, "parameters must be finite");
    if (p->ds <= 0 || p->dt <= 0) return fail(LBM_EINVAL, "ds and dt must be > 0");
    if (p->tau <= 0) return fail(LBM_EINVAL, "tau must be > 0");
    if (p->T <= 0) return fail(LBM_EINVAL, "T must be > 0");
    if (p->a < 0 || p->b < 0 || p->kappa < 0) return fail(LBM_EINVAL, "a, b and kappa must be >= 0");
    if (p->scheme != 1 && p->scheme != 2) return fail(LBM_EINVAL, "scheme must be 1 (CTU1) or 2 (CTU2)");
    if (p->regularize != 0 && p->regularize != 1) return fail(LBM_EINVAL, "regularize must be 0 or 1");
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32_DEV)
        return fail(LBM_EINVAL, "precision must be LBM_FP64 or LBM_FP32_DEV");
    if (p->precision == LBM_FP32_DEV && p->rho_ref <= 0)
        return fail(LBM_EINVAL, "rho_ref must be > 0 for FP32 deviation storage");
    if (p->bc_y != LBM_PERIODIC && p->bc_y != LBM_SHEAR_WALLS) return fail(LBM_EINVAL, "bc_y must be 0 or 1");
    if (p->bc_y == LBM_SHEAR_WALLS) {
        if (p->rho_wall <= 0 || (p->b > 0 && p->b * p->rho_wall >= 1.0))
            return fail(LBM_EINVAL, "rho_wall must lie in (0, 1/b)");
    }
    if (p->clamp_radius > 0) {
        if (p->clamp_rho <= 0 || (p->b > 0 && p->b * p->clamp_rho >= 1.0))
            return fail(LBM_EINVAL, "clamp_rho must lie in (0, 1/b)");
    }
    if (p->rounding != LBM_ROUND_STOCHASTIC && p->rounding != LBM_ROUND_NEAREST)
        return fail(LBM_EINVAL, "rounding must be LBM_ROUND_STOCHASTIC or LBM_ROUND_NEAREST");
    // CFL condition of the CTU schemes: max_k |xi_k,alpha| dt <= ds
    if (QL * p->dt > p->ds * (1.0 + 1e-12))
        return fail(LBM_ECFL, "CFL violated: dt * sqrt(3 + sqrt 6) must not exceed ds");
    return LBM_OK;
}

template <typename R>
void fill_coef(const lbm_params* p, StepCoef<R>& c)
{
    std::memset(&c, 0, sizeof(c));
    const double nu = p->dt / p->ds;
    const double rho0 = (p->precision == LBM_FP32_DEV) ? p->rho_ref : 0.0;
    const double q[2] = {QS, QL};
    for (int mx = 0; mx < 2; ++mx) {
        const double ax = nu * q[mx], k2x = q[mx] * (1 - ax);
        c.nu_xi[mx] = (R)ax;
        for (int my = 0; my < 2; ++my) {
            const double ay = nu * q[my], k2y = q[my] * (1 - ay);
            c.xs1[mx][my] = (R)(-nu * (1 - ay) * k2x);
            c.xs2[mx][my] = (R)(-nu * ay * k2x);
            c.ys1[mx][my] = (R)(-nu * (1 - ax) * k2y);
            c.ys2[mx][my] = (R)(-nu * ax * k2y);
        }
    }
    double rlo = 0, rhi = 0;
    for (int k = 0; k < 16; ++k) {
        const double lo = feq_host(k, p->T, p->rho_wall, -p->u_wall, 0.0);
        const double hi = feq_host(k, p->T, p->rho_wall, +p->u_wall, 0.0);
        rlo += lo;
        rhi += hi;
        c.ghost_lo[k] = (R)(lo - weight(k) * rho0);
        c.ghost_hi[k] = (R)(hi - weight(k) * rho0);
    }
    c.ghost_rho_lo = rlo;
    c.ghost_rho_hi = rhi;
    c.rho0 = rho0;
    c.T = p->T;
    c.Tm1 = p->T - 1.0;
    c.a_vdw = p->a;
    c.b_vdw = p->b;
    c.kappa_ds = p->kappa / p->ds;
    c.inv_ds = 1.0 / p->ds;
    c.inv_6ds2 = 1.0 / (6.0 * p->ds * p->ds);
    c.dt_tau = p->dt / p->tau;
    c.dt = p->dt;
    c.walls = p->bc_y == LBM_SHEAR_WALLS ? 1 : 0;
    c.clamp = p->clamp_radius > 0 ? 1 : 0;
    c.clamp_r2 = p->clamp_radius > 0 ? p->clamp_radius * p->clamp_radius : 0.0;
    c.clamp_cx = 0.5 * (p->Lx - 1);
    c.clamp_cy = 0.5 * (p->Ly - 1);
    c.clamp_rho = p->clamp_rho;
    c.sr_mask = (p->rounding == LBM_ROUND_NEAREST) ? 0u : 0x1FFFFFFFu;
}

size_t storage_bytes(const lbm_params* p) { return p->precision == LBM_FP32_DEV ? 4 : 8; }

// Workspace layout of one run (offsets in bytes, all 256-aligned):
//   [coef (fp32 + fp64 tables)] [reduction partials + result] [field 0] [field 1]
constexpr size_t COEF_BYTES = 8192;
static_assert(sizeof(StepCoef<double>) + sizeof(StepCoef<float>) + 2 * ALIGN <= COEF_BYTES, "coef region");
// the step counter pair of the stochastic rounding sits at the end of the coef region
constexpr size_t SEQ_OFF = COEF_BYTES - 64;
static_assert(sizeof(StepCoef<double>) <= SEQ_OFF && sizeof(StepCoef<float>) <= SEQ_OFF, "seq slot");
constexpr size_t RED_BYTES = (size_t)(REDUCE_MAX_BLOCKS + 1) * REDUCE_VALUES * sizeof(double);

// stride of one distribution plane: the Lx * Ly lattice, then with shear walls
// the two ghost rows (below, above)
int64_t plane_of(const lbm_params* p)
{
    return (int64_t)p->Lx * ((int64_t)p->Ly + (p->bc_y == LBM_SHEAR_WALLS ? 2 : 0));
}

size_t field_bytes(const lbm_params* p) { return align_up((size_t)16 * (size_t)plane_of(p) * storage_bytes(p)); }

size_t run_bytes(const lbm_params* p)
{
    return COEF_BYTES + align_up(RED_BYTES) + 2 * field_bytes(p);
}

// default launch shape: one wavefront per SIMD, so a launch runs in rounds of
// (SIMD count) wavefronts; each wavefront pays about 5 rows of warm-up for
// its march (8 rows at roughly 60% of the cost of a full row).  Pick the rows
// per wavefront that minimise rounds x (rows + 5).
Launch default_launch(const lbm_params* p)
{
    // FP32 storage: a pair of wavefronts per strip, short chunks (measured
    // best at 32-40 rows on 6144^2)
    if (p->precision == LBM_FP32_DEV) return Launch{32, LBM_PAIR};
    static int slots = 0;
    if (slots == 0) {
        int dev = 0, ncu = 0;
        slots = (hipGetDevice(&dev) == hipSuccess
                 && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
                    ? 4 * ncu
                    : 1024;
    }
    const int64_t nstrips = (p->Lx + STRIP - 1) / STRIP;
    int best_rows = 64;
    double best = 1e300;
    for (int rows = 8; rows <= 512; rows += 8) {
        const int64_t nwaves = nstrips * ((p->Ly + rows - 1) / rows);
        const int64_t rounds = (nwaves + slots - 1) / slots;
        const double cost = (double)rounds * (double)(std::min(rows, p->Ly) + 5);
        if (cost < best - 1e-9) {
            best = cost;
            best_rows = rows;
        }
    }
    return Launch{best_rows, 2};
}

// LDS of a step workgroup: the kernels keep the advected rows that wait for
// their collision there (32 KiB per wavefront, or per pair); capped at 64 KiB
// per workgroup.  The pair launch is built for FP32 storage only.
constexpr size_t MAX_STEP_LDS = 65536;
size_t step_lds_bytes(const lbm_params* p, int wpg)
{
    (void)p;
    return wpg == LBM_PAIR ? PAIR_STEP_LDS : (size_t)wpg * STEP_LDS_PER_WAVE;
}
bool launch_fits(const lbm_params* p, int wpg)
{
    if (wpg == LBM_PAIR && p->precision != LBM_FP32_DEV) return false;
    return step_lds_bytes(p, wpg) <= MAX_STEP_LDS;
}

std::mutex g_tune_mutex;
// (Lx, Ly, precision, scheme, regularize, bc_y)
std::map<std::tuple<int, int, int, int, int, int>, Launch> g_tuned;
// rows per work item a batch autotune chose for runs of that shape
std::map<std::tuple<int, int, int, int, int, int>, int> g_batch_tuned;

}  // namespace

struct lbm_run {
    lbm_params p;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    void* coef = nullptr;        // StepCoef<R> for the storage precision
    double* red = nullptr;       // reduction partials; result in the last REDUCE_VALUES slots
    char* field[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t step = 0;
    Launch launch{64, 2};
    lbm_batch* batch = nullptr;  // non-null for a borrowed batch member
};

// polls of one dependency wait of the persistent batched launch before it
// gives up (a poll is a device-scope load and a short sleep, about 1-2 us, so
// the default bounds a wait at several seconds; a correct launch waits at
// most a few work items' time)
constexpr uint32_t DEFAULT_WAIT_LIMIT = 1u << 22;

struct lbm_batch {
    int32_t n = 0;
    int precision = 0, scheme = 2, regularize = 0;
    std::vector<lbm_run> runs;
    void* d_runs = nullptr;   // BatchRun<R>[n]
    void* d_coefs = nullptr;  // StepCoef<R>[n]
    BatchItem* d_items = nullptr;
    int32_t nitems = 0;
    int32_t nitems_periodic = 0;  // items [0, nitems_periodic) belong to periodic runs
    int32_t mode = LBM_BATCH_PER_STEP;
    int32_t* d_done = nullptr;    // persistent launch: one flag per item
    uint32_t* d_sync = nullptr;   // persistent launch: [0] ticket, [1] error
    uint32_t wait_limit = DEFAULT_WAIT_LIMIT;
    int cur = 0;
    int64_t step = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_steps = 0;
    hipStream_t capture_stream = nullptr;
};

namespace {

template <typename R>
StepCoef<R>* coef_of(lbm_run* r) { return static_cast<StepCoef<R>*>(r->coef); }

// (Re)write the two wall ghost rows of field `fld` (no-op without walls).
// Every use of the non-current field as FP64 staging overwrites them.
hipError_t fill_ghosts(lbm_run* r, int fld, hipStream_t s)
{
    if (r->p.bc_y != LBM_SHEAR_WALLS) return hipSuccess;
    const int64_t plane = (int64_t)r->p.Lx * ((int64_t)r->p.Ly + 2);
    return (r->p.precision == LBM_FP32_DEV)
               ? launch_fill_ghost<float>(reinterpret_cast<float*>(r->field[fld]), static_cast<StepCoef<float>*>(r->coef),
                                          r->p.Lx, r->p.Ly, plane, s)
               : launch_fill_ghost<double>(reinterpret_cast<double*>(r->field[fld]), static_cast<StepCoef<double>*>(r->coef),
                                           r->p.Lx, r->p.Ly, plane, s);
}

uint32_t* seq_of(lbm_run* r) { return reinterpret_cast<uint32_t*>(r->ws + SEQ_OFF); }

// coefficients, and the step counter pair set to the run's step (both slots)
template <typename R>
lbm_status upload_coef(lbm_run* r, hipStream_t s)
{
    StepCoef<R> c;
    fill_coef<R>(&r->p, c);
    const uint32_t seq[2] = {(uint32_t)r->step, (uint32_t)r->step};
    HIP_TRY(hipMemcpyAsync(r->coef, &c, sizeof(c), hipMemcpyHostToDevice, s), "upload coefficients");
    HIP_TRY(hipMemcpyAsync(seq_of(r), seq, sizeof(seq), hipMemcpyHostToDevice, s), "upload step counter");
    HIP_TRY(hipStreamSynchronize(s), "upload coefficients");
    return LBM_OK;
}

lbm_status carve(const lbm_params* p, void* d_ws, size_t ws_bytes, lbm_run* r)
{
    if (!d_ws) return fail(LBM_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_ws) % ALIGN) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < run_bytes(p)) return fail(LBM_ENOMEM, "workspace smaller than lbm_workspace_bytes()");
    r->p = *p;
    r->ws = static_cast<char*>(d_ws);
    r->ws_bytes = ws_bytes;
    r->coef = r->ws;
    r->red = reinterpret_cast<double*>(r->ws + COEF_BYTES);
    r->field[0] = r->ws + COEF_BYTES + align_up(RED_BYTES);
    r->field[1] = r->field[0] + field_bytes(p);
    r->cur = 0;
    r->step = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tuned.find({p->Lx, p->Ly, p->precision, p->scheme, p->regularize, p->bc_y});
        r->launch = (it != g_tuned.end()) ? it->second : default_launch(p);
    }
    return LBM_OK;
}

lbm_status upload_coef_any(lbm_run* r, hipStream_t s)
{
    return r->p.precision == LBM_FP32_DEV ? upload_coef<float>(r, s) : upload_coef<double>(r, s);
}

int64_t nodes(const lbm_run* r) { return (int64_t)r->p.Lx * r->p.Ly; }

template <typename R>
RunView<R> view(lbm_run* r)
{
    RunView<R> v;
    v.f_in = reinterpret_cast<const R*>(r->field[r->cur]);
    v.f_out = reinterpret_cast<R*>(r->field[r->cur ^ 1]);
    v.coef = coef_of<R>(r);
    v.seq = seq_of(r);
    v.cur = r->cur;
    v.Lx = r->p.Lx;
    v.Ly = r->p.Ly;
    v.rows = r->launch.rows_per_wave;
    v.nstrips = (r->p.Lx + STRIP - 1) / STRIP;
    v.plane = plane_of(&r->p);
    return v;
}

lbm_status step_once(lbm_run* r, hipStream_t s)
{
    hipError_t e;
    if (r->p.precision == LBM_FP32_DEV)
        e = launch_step<float>(view<float>(r), r->p.scheme, r->p.regularize, r->p.bc_y, r->launch.waves_per_group, s);
    else
        e = launch_step<double>(view<double>(r), r->p.scheme, r->p.regularize, r->p.bc_y, r->launch.waves_per_group, s);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    r->cur ^= 1;
    r->step += 1;
    return LBM_OK;
}

lbm_status init_common(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream, const double* rho,
                       const double* ux, const double* uy, bool host, lbm_run** out)
{
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (!rho || !ux || !uy) return fail(LBM_EINVAL, "null initial fields");
    const int64_t n = (int64_t)p->Lx * p->Ly;
    if (host) {
        for (int64_t i = 0; i < n; ++i) {
            if (!is_finite_d(rho[i]) || !is_finite_d(ux[i]) || !is_finite_d(uy[i]))
                return fail(LBM_EINVAL, "initial fields must be finite");
            if (rho[i] <= 0 || (p->b > 0 && p->b * rho[i] >= 1.0))
                return fail(LBM_EINVAL, "initial density must lie in (0, 1/b)");
        }
    }
    lbm_run* r = new (std::nothrow) lbm_run();
    if (!r) return fail(LBM_EINVAL, "out of host memory");
    st = carve(p, d_ws, ws_bytes, r);
    if (st != LBM_OK) {
        delete r;
        return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = upload_coef_any(r, s);
    if (st != LBM_OK) {
        delete r;
        return st;
    }
    const double *d_rho = rho, *d_ux = ux, *d_uy = uy;
    if (host) {
        // stage the three host arrays in the second field buffer (>= 24 bytes per node)
        double* stage = reinterpret_cast<double*>(r->field[1]);
        hipError_t e = hipMemcpyAsync(stage, rho, n * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(stage + n, ux, n * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(stage + 2 * n, uy, n * sizeof(double), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            delete r;
            return hip_fail(e, "upload initial fields");
        }
        d_rho = stage;
        d_ux = stage + n;
        d_uy = stage + 2 * n;
    }
    const int64_t plane = plane_of(p);
    hipError_t e = (p->precision == LBM_FP32_DEV)
                       ? launch_init<float>(reinterpret_cast<float*>(r->field[0]), coef_of<float>(r), d_rho, d_ux, d_uy, n, plane, s)
                       : launch_init<double>(reinterpret_cast<double*>(r->field[0]), coef_of<double>(r), d_rho, d_ux, d_uy, n, plane, s);
    // ghost rows of both fields (the second after its staging use above)
    for (int fld = 0; fld < 2 && e == hipSuccess; ++fld) e = fill_ghosts(r, fld, s);
    if (e == hipSuccess && host) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete r;
        return hip_fail(e, "init");
    }
    *out = r;
    return LBM_OK;
}

// FP64 staging buffer for one plane / one moment field: the non-current field
lbm_status moments_to(lbm_run* r, double* rho, double* ux, double* uy, hipStream_t s)
{
    const int64_t n = nodes(r);
    hipError_t e = (r->p.precision == LBM_FP32_DEV)
                       ? launch_moments<float>(reinterpret_cast<const float*>(r->field[r->cur]), coef_of<float>(r), rho, ux, uy, n, plane_of(&r->p), s)
                       : launch_moments<double>(reinterpret_cast<const double*>(r->field[r->cur]), coef_of<double>(r), rho, ux, uy, n, plane_of(&r->p), s);
    if (e != hipSuccess) return hip_fail(e, "moments");
    return LBM_OK;
}

lbm_status get_plane(lbm_run* r, int k, double* d_out, hipStream_t s)
{
    const int64_t n = nodes(r);
    hipError_t e = (r->p.precision == LBM_FP32_DEV)
                       ? launch_get_plane<float>(reinterpret_cast<const float*>(r->field[r->cur]), coef_of<float>(r), k, d_out, n, plane_of(&r->p), s)
                       : launch_get_plane<double>(reinterpret_cast<const double*>(r->field[r->cur]), coef_of<double>(r), k, d_out, n, plane_of(&r->p), s);
    if (e != hipSuccess) return hip_fail(e, "get_f");
    return LBM_OK;
}

lbm_status set_plane(lbm_run* r, int k, const double* d_in, hipStream_t s)
{
    const int64_t n = nodes(r);
    hipError_t e = (r->p.precision == LBM_FP32_DEV)
                       ? launch_set_plane<float>(reinterpret_cast<float*>(r->field[r->cur]), coef_of<float>(r), k, d_in, n, plane_of(&r->p), s)
                       : launch_set_plane<double>(reinterpret_cast<double*>(r->field[r->cur]), coef_of<double>(r), k, d_in, n, plane_of(&r->p), s);
    if (e != hipSuccess) return hip_fail(e, "set_f");
    return LBM_OK;
}

void derive_stats(const lbm_params& p, const double* v, lbm_stats* o)
{
    std::memset(o, 0, sizeof(*o));
    o->mass = v[0];
    o->mom_x = v[1];
    o->mom_y = v[2];
    o->n_bubble = (int64_t)std::llround(v[3]);
    o->n_nonfinite = (int64_t)std::llround(v[4]);
    o->sx = v[5];
    o->sy = v[6];
    o->sxx = v[7];
    o->sxy = v[8];
    o->syy = v[9];
    const double N = (double)o->n_bubble;
    o->A_rel = N / ((double)p.Lx * (double)p.Ly);
    o->R_eq = p.ds * std::sqrt(N / M_PI);
    if (o->n_bubble > 0) {
        o->cx = o->sx / N + 0.5 * (p.Lx - 1);
        o->cy = o->sy / N + 0.5 * (p.Ly - 1);
        const double mx = o->sx / N, my = o->sy / N;
        o->Txx = o->sxx / N - mx * mx;
        o->Txy = o->sxy / N - mx * my;
        o->Tyy = o->syy / N - my * my;
        const double h = 0.5 * (o->Txx + o->Tyy);
        const double q = std::sqrt(0.25 * (o->Txx - o->Tyy) * (o->Txx - o->Tyy) + o->Txy * o->Txy);
        const double lmax = h + q, lmin = std::max(h - q, 0.0);
        o->a = 2.0 * std::sqrt(std::max(lmax, 0.0));
        o->b = 2.0 * std::sqrt(lmin);
        o->D = (o->a + o->b) > 0 ? (o->a - o->b) / (o->a + o->b) : 0.0;
        o->theta = 0.5 * std::atan2(2.0 * o->Txy, o->Txx - o->Tyy);
    }
}

}  // namespace

// ============================================================================
// Device scratch of the allocation-free entry point (lbm_reduce_field_static):
// a file-scope array, one copy per GPU, resolved per device with
// hipGetSymbolAddress.  In host code `scratch` names a host-side stand-in,
// never the device memory: only the resolved pointer is passed on.

namespace {
// coefficient block (either precision), then the block partials and the
// REDUCE_VALUES results of the reduction
constexpr size_t SCRATCH_COEF_BYTES = 8192;
static_assert(sizeof(StepCoef<double>) <= SCRATCH_COEF_BYTES && sizeof(StepCoef<float>) <= SCRATCH_COEF_BYTES,
              "scratch coefficient slot");
constexpr size_t SCRATCH_BYTES = SCRATCH_COEF_BYTES + RED_BYTES;
}  // namespace

static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
char* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

// device address of the current device's copy of `scratch` (looked up on
// the first call on that device)
lbm_status scratch_of_current_device(char** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "scratch: current device");
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(LBM_EDEVICE, "scratch: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch: hipGetSymbolAddress");
        if (!ptr) return fail(LBM_EDEVICE, "scratch: null symbol address");
        g_scratch_dev[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}

template <typename R>
lbm_status reduce_field_static(const lbm_params* p, const void* d_f, double threshold, lbm_stats* out,
                               hipStream_t s)
{
    char* scr = nullptr;
    lbm_status st = scratch_of_current_device(&scr);
    if (st != LBM_OK) return st;
    StepCoef<R> c;
    fill_coef<R>(p, c);
    StepCoef<R>* d_coef = reinterpret_cast<StepCoef<R>*>(scr);
    double* partials = reinterpret_cast<double*>(scr + SCRATCH_COEF_BYTES);
    double* result = partials + (size_t)REDUCE_MAX_BLOCKS * REDUCE_VALUES;
    HIP_TRY(hipMemcpyAsync(d_coef, &c, sizeof(c), hipMemcpyHostToDevice, s), "reduce_field_static: coefficients");
    HIP_TRY(launch_reduce<R>(static_cast<const R*>(d_f), d_coef, p->Lx, p->Ly, plane_of(p), threshold, partials,
                             REDUCE_MAX_BLOCKS, result, s),
            "reduce_field_static: launch");
    double v[REDUCE_VALUES];
    HIP_TRY(hipMemcpyAsync(v, result, sizeof(v), hipMemcpyDeviceToHost, s), "reduce_field_static: download");
    HIP_TRY(hipStreamSynchronize(s), "reduce_field_static");
    derive_stats(*p, v, out);
    if (out->n_nonfinite > 0) return fail(LBM_ENONFINITE, "non-finite distribution values in the state");
    return LBM_OK;
}
}  // namespace

// ============================================================================
// C ABI

extern "C" {

const char* lbm_version(void) { return "paper_1802_01272_amd lbm 0.1 (gfx950)"; }

const char* lbm_last_error(void) { return g_error.c_str(); }

lbm_status lbm_validate(const lbm_params* p) { return validate(p); }

size_t lbm_workspace_bytes(const lbm_params* p)
{
    if (validate(p) != LBM_OK) return 0;
    return run_bytes(p);
}

lbm_status lbm_init(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream, const double* h_rho0,
                    const double* h_ux0, const double* h_uy0, lbm_run** out)
{
    return init_common(p, d_ws, ws_bytes, stream, h_rho0, h_ux0, h_uy0, true, out);
}

lbm_status lbm_init_device(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream, const double* d_rho0,
                           const double* d_ux0, const double* d_uy0, lbm_run** out)
{
    return init_common(p, d_ws, ws_bytes, stream, d_rho0, d_ux0, d_uy0, false, out);
}

lbm_status lbm_attach(const lbm_params* p, void* d_ws, size_t ws_bytes, int64_t step, lbm_run** out)
{
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (step < 0) return fail(LBM_EINVAL, "step must be >= 0");
    lbm_run* r = new (std::nothrow) lbm_run();
    if (!r) return fail(LBM_EINVAL, "out of host memory");
    st = carve(p, d_ws, ws_bytes, r);
    if (st == LBM_OK) {
        r->cur = (int)(step & 1);
        r->step = step;
        st = upload_coef_any(r, nullptr);
    }
    if (st != LBM_OK) {
        delete r;
        return st;
    }
    *out = r;
    return LBM_OK;
}

lbm_status lbm_step(lbm_run* run, int64_t nsteps, void* stream)
{
    if (!run) return fail(LBM_EINVAL, "null run");
    if (run->batch) return fail(LBM_ESTATE, "runs of a batch advance with lbm_batch_step");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int64_t i = 0; i < nsteps; ++i) {
        lbm_status st = step_once(run, s);
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

lbm_status lbm_step_timed(lbm_run* run, int64_t nsteps, void* stream, double* ms)
{
    if (!run || !ms) return fail(LBM_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a), "event");
    HIP_TRY(hipEventCreate(&b), "event");
    hipError_t e = hipEventRecord(a, s);
    lbm_status st = (e == hipSuccess) ? lbm_step(run, nsteps, stream) : hip_fail(e, "event record");
    if (st == LBM_OK) {
        e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float f = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
        if (e != hipSuccess) st = hip_fail(e, "event timing");
        *ms = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

int64_t lbm_step_count(const lbm_run* run) { return run ? run->step : -1; }

lbm_status lbm_moments_device(lbm_run* run, double* d_rho, double* d_ux, double* d_uy, void* stream)
{
    if (!run || !d_rho || !d_ux || !d_uy) return fail(LBM_EINVAL, "null argument");
    return moments_to(run, d_rho, d_ux, d_uy, static_cast<hipStream_t>(stream));
}

lbm_status lbm_moments(lbm_run* run, double* h_rho, double* h_ux, double* h_uy, void* stream)
{
    if (!run || !h_rho || !h_ux || !h_uy) return fail(LBM_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = nodes(run);
    // the non-current field buffer holds >= 24 bytes per node
    double* stage = reinterpret_cast<double*>(run->field[run->cur ^ 1]);
    lbm_status st = moments_to(run, stage, stage + n, stage + 2 * n, s);
    if (st != LBM_OK) return st;
    HIP_TRY(hipMemcpyAsync(h_rho, stage, n * sizeof(double), hipMemcpyDeviceToHost, s), "moments download");
    HIP_TRY(hipMemcpyAsync(h_ux, stage + n, n * sizeof(double), hipMemcpyDeviceToHost, s), "moments download");
    HIP_TRY(hipMemcpyAsync(h_uy, stage + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, s), "moments download");
    HIP_TRY(fill_ghosts(run, run->cur ^ 1, s), "moments: ghost rows");
    HIP_TRY(hipStreamSynchronize(s), "moments download");
    return LBM_OK;
}

lbm_status lbm_get_f_device(lbm_run* run, double* d_f, void* stream)
{
    if (!run || !d_f) return fail(LBM_EINVAL, "null argument");
    const int64_t n = nodes(run);
    for (int k = 0; k < 16; ++k) {
        lbm_status st = get_plane(run, k, d_f + k * n, static_cast<hipStream_t>(stream));
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

lbm_status lbm_set_f_device(lbm_run* run, const double* d_f, void* stream)
{
    if (!run || !d_f) return fail(LBM_EINVAL, "null argument");
    const int64_t n = nodes(run);
    for (int k = 0; k < 16; ++k) {
        lbm_status st = set_plane(run, k, d_f + k * n, static_cast<hipStream_t>(stream));
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

lbm_status lbm_get_f(lbm_run* run, double* h_f, void* stream)
{
    if (!run || !h_f) return fail(LBM_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = nodes(run);
    double* stage = reinterpret_cast<double*>(run->field[run->cur ^ 1]);  // one FP64 plane fits
    for (int k = 0; k < 16; ++k) {
        lbm_status st = get_plane(run, k, stage, s);
        if (st != LBM_OK) return st;
        HIP_TRY(hipMemcpyAsync(h_f + k * n, stage, n * sizeof(double), hipMemcpyDeviceToHost, s), "get_f download");
        HIP_TRY(hipStreamSynchronize(s), "get_f download");
    }
    HIP_TRY(fill_ghosts(run, run->cur ^ 1, s), "get_f: ghost rows");
    return LBM_OK;
}

lbm_status lbm_set_f(lbm_run* run, const double* h_f, void* stream)
{
    if (!run || !h_f) return fail(LBM_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = nodes(run);
    double* stage = reinterpret_cast<double*>(run->field[run->cur ^ 1]);
    for (int k = 0; k < 16; ++k) {
        HIP_TRY(hipMemcpyAsync(stage, h_f + k * n, n * sizeof(double), hipMemcpyHostToDevice, s), "set_f upload");
        lbm_status st = set_plane(run, k, stage, s);
        if (st != LBM_OK) return st;
        HIP_TRY(hipStreamSynchronize(s), "set_f upload");
    }
    HIP_TRY(fill_ghosts(run, run->cur ^ 1, s), "set_f: ghost rows");
    return LBM_OK;
}

lbm_status lbm_reduce(lbm_run* run, double rho_threshold, lbm_stats* out, void* stream)
{
    if (!run || !out) return fail(LBM_EINVAL, "null argument");
    if (!is_finite_d(rho_threshold)) return fail(LBM_EINVAL, "threshold must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* result = run->red + (size_t)REDUCE_MAX_BLOCKS * REDUCE_VALUES;
    hipError_t e = (run->p.precision == LBM_FP32_DEV)
                       ? launch_reduce<float>(reinterpret_cast<const float*>(run->field[run->cur]), coef_of<float>(run),
                                              run->p.Lx, run->p.Ly, plane_of(&run->p), rho_threshold, run->red,
                                              REDUCE_MAX_BLOCKS, result, s)
                       : launch_reduce<double>(reinterpret_cast<const double*>(run->field[run->cur]), coef_of<double>(run),
                                               run->p.Lx, run->p.Ly, plane_of(&run->p), rho_threshold, run->red,
                                               REDUCE_MAX_BLOCKS, result, s);
    if (e != hipSuccess) return hip_fail(e, "reduce");
    double v[REDUCE_VALUES];
    HIP_TRY(hipMemcpyAsync(v, result, sizeof(v), hipMemcpyDeviceToHost, s), "reduce download");
    HIP_TRY(hipStreamSynchronize(s), "reduce");
    derive_stats(run->p, v, out);
    if (out->n_nonfinite > 0) return fail(LBM_ENONFINITE, "non-finite distribution values in the state");
    return LBM_OK;
}

lbm_status lbm_reduce_field_static(const lbm_params* p, const void* d_f, double rho_threshold, lbm_stats* out,
                                  void* stream)
{
    if (!p || !d_f || !out) return fail(LBM_EINVAL, "null argument");
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (!is_finite_d(rho_threshold)) return fail(LBM_EINVAL, "threshold must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return p->precision == LBM_FP32_DEV ? reduce_field_static<float>(p, d_f, rho_threshold, out, s)
                                        : reduce_field_static<double>(p, d_f, rho_threshold, out, s);
}

lbm_status lbm_set_launch(lbm_run* run, int32_t rows_per_wave, int32_t waves_per_group)
{
    if (!run) return fail(LBM_EINVAL, "null run");
    if (rows_per_wave < 1) return fail(LBM_EINVAL, "rows_per_wave must be >= 1");
    if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4 && waves_per_group != LBM_PAIR)
        return fail(LBM_EINVAL, "waves_per_group must be 1, 2, 4 or LBM_PAIR");
    if (!launch_fits(&run->p, waves_per_group))
        return fail(LBM_EINVAL, waves_per_group == LBM_PAIR
                                    ? "LBM_PAIR launches need FP32 storage"
                                    : "waves_per_group too large for the LDS of the step kernel (at most 2)");
    run->launch = Launch{rows_per_wave, waves_per_group};
    return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_run* run, int32_t* rows_per_wave, int32_t* waves_per_group)
{
    if (!run || !rows_per_wave || !waves_per_group) return fail(LBM_EINVAL, "null argument");
    *rows_per_wave = run->launch.rows_per_wave;
    *waves_per_group = run->launch.waves_per_group;
    return LBM_OK;
}

lbm_status lbm_autotune(const lbm_params* p, void* d_ws, size_t ws_bytes, void* stream, int32_t steps_per_trial,
                        int32_t* rows_per_wave, int32_t* waves_per_group)
{
    if (!rows_per_wave || !waves_per_group) return fail(LBM_EINVAL, "null argument");
    lbm_status st = validate(p);
    if (st != LBM_OK) return st;
    if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    lbm_run r;
    st = carve(p, d_ws, ws_bytes, &r);
    if (st == LBM_OK) st = upload_coef_any(&r, s);
    if (st != LBM_OK) return st;
    // synthetic state: f^eq of a uniform fluid at the middle of the allowed density range
    {
        const double rho_u = (p->b > 0) ? std::min(1.0, 0.5 / p->b) : 1.0;
        const int64_t n = nodes(&r);
        double* stage = reinterpret_cast<double*>(r.field[1]);
        std::vector<double> h(n, rho_u), z(n, 0.0);
        HIP_TRY(hipMemcpyAsync(stage, h.data(), n * sizeof(double), hipMemcpyHostToDevice, s), "autotune");
        HIP_TRY(hipMemcpyAsync(stage + n, z.data(), n * sizeof(double), hipMemcpyHostToDevice, s), "autotune");
        HIP_TRY(hipMemcpyAsync(stage + 2 * n, z.data(), n * sizeof(double), hipMemcpyHostToDevice, s), "autotune");
        hipError_t e = (p->precision == LBM_FP32_DEV)
                           ? launch_init<float>(reinterpret_cast<float*>(r.field[0]), coef_of<float>(&r), stage, stage + n, stage + 2 * n, n, plane_of(p), s)
                           : launch_init<double>(reinterpret_cast<double*>(r.field[0]), coef_of<double>(&r), stage, stage + n, stage + 2 * n, n, plane_of(p), s);
        for (int fld = 0; fld < 2 && e == hipSuccess; ++fld) e = fill_ghosts(&r, fld, s);
        if (e != hipSuccess) return hip_fail(e, "autotune init");
        HIP_TRY(hipStreamSynchronize(s), "autotune init");
    }
    // fixed candidates plus the default shape's rows and its neighbours
    std::vector<int> rows_c = {8, 16, 24, 32, 40, 48, 64, 96, 128, 192, 256, 384, 512};
    {
        const int d = default_launch(p).rows_per_wave;
        for (int r : {d - 16, d - 8, d, d + 8, d + 16})
            if (r >= 8 && std::find(rows_c.begin(), rows_c.end(), r) == rows_c.end()) rows_c.push_back(r);
    }
    const int wpg_c[] = {1, 2, 4, LBM_PAIR};
    double best = 1e300;
    Launch bl = default_launch(p);
    for (int rows : rows_c) {
        if (rows > 2 * p->Ly && rows != rows_c[0]) continue;
        for (int wpg : wpg_c) {
            if (!launch_fits(p, wpg)) continue;
            r.launch = Launch{rows, wpg};
            for (int w = 0; w < 2; ++w) {
                st = step_once(&r, s);
                if (st != LBM_OK) return st;
            }
            double ms = 0;
            st = lbm_step_timed(&r, steps_per_trial, stream, &ms);
            if (st != LBM_OK) return st;
            if (ms < best) {
                best = ms;
                bl = r.launch;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tuned[{p->Lx, p->Ly, p->precision, p->scheme, p->regularize, p->bc_y}] = bl;
    }
    *rows_per_wave = bl.rows_per_wave;
    *waves_per_group = bl.waves_per_group;
    return LBM_OK;
}

void lbm_destroy(lbm_run* run)
{
    if (run && !run->batch) delete run;
}

lbm_status lbm_state_device(const lbm_run* run, const void** d_f, int64_t* plane_stride)
{
    if (!run || !d_f || !plane_stride) return fail(LBM_EINVAL, "null argument");
    *d_f = run->field[run->cur];
    *plane_stride = plane_of(&run->p);
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// batched runs

}  // extern "C"

// most work items a batch can hold (one row per item)
size_t batch_items_bound(int32_t n, const lbm_params* params)
{
    size_t items = 0;
    for (int i = 0; i < n; ++i) items += (size_t)((params[i].Lx + STRIP - 1) / STRIP) * (size_t)params[i].Ly;
    return items;
}

extern "C" size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params* params)
{
    if (n < 1 || !params) return 0;
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (validate(&params[i]) != LBM_OK) return 0;
        total += run_bytes(&params[i]);
    }
    // tables: runs, coefficient copies, work items, and for the persistent
    // launch one flag per item and the ticket / error words
    const size_t items = batch_items_bound(n, params);
    total += align_up((size_t)n * sizeof(BatchRun<double>)) + align_up((size_t)n * sizeof(StepCoef<double>))
           + align_up(items * sizeof(BatchItem)) + align_up(items * sizeof(int32_t)) + ALIGN;
    return total;
}

namespace {

// forget a captured graph (the work list it baked in has changed)
void drop_graph(lbm_batch* b)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->graph_steps = 0;
    }
}

template <typename R>
lbm_status batch_tables(lbm_batch* b, char* base, hipStream_t s)
{
    std::vector<BatchRun<R>> runs(b->n);
    std::vector<StepCoef<R>> coefs(b->n);
    std::vector<BatchItem> items, wall_items;
    for (int i = 0; i < b->n; ++i) {
        lbm_run& r = b->runs[i];
        BatchRun<R>& br = runs[i];
        br.f[0] = reinterpret_cast<R*>(r.field[0]);
        br.f[1] = reinterpret_cast<R*>(r.field[1]);
        br.coef = nullptr;
        br.seq = seq_of(&r);
        br.Lx = r.p.Lx;
        br.Ly = r.p.Ly;
        br.rows = r.launch.rows_per_wave;
        br.nstrips = (r.p.Lx + STRIP - 1) / STRIP;
        br.plane = plane_of(&r.p);
        br.walls = r.p.bc_y == LBM_SHEAR_WALLS ? 1 : 0;
        fill_coef<R>(&r.p, coefs[i]);
        const int nchunks = (r.p.Ly + br.rows - 1) / br.rows;
        std::vector<BatchItem>& dst = br.walls ? wall_items : items;
        br.item_base = (int32_t)dst.size();  // within its kind; wall runs are offset below
        for (int c = 0; c < nchunks; ++c)
            for (int st = 0; st < br.nstrips; ++st) dst.push_back(BatchItem{i, st, c, 0});
    }
    // periodic items first, then the items of runs with walls
    b->nitems_periodic = (int32_t)items.size();
    for (auto& br : runs)
        if (br.walls) br.item_base += b->nitems_periodic;
    items.insert(items.end(), wall_items.begin(), wall_items.end());
    char* p = base;
    b->d_runs = p;
    p += align_up((size_t)b->n * sizeof(BatchRun<double>));
    b->d_coefs = p;
    p += align_up((size_t)b->n * sizeof(StepCoef<double>));
    b->d_items = reinterpret_cast<BatchItem*>(p);
    b->nitems = (int32_t)items.size();
    {
        std::vector<lbm_params> ps(b->n);
        for (int i = 0; i < b->n; ++i) ps[i] = b->runs[i].p;
        const size_t bound = batch_items_bound(b->n, ps.data());
        if (items.size() > bound) return fail(LBM_EINVAL, "batch work list exceeds its bound");
        p += align_up(bound * sizeof(BatchItem));
        b->d_done = reinterpret_cast<int32_t*>(p);
        p += align_up(bound * sizeof(int32_t));
        b->d_sync = reinterpret_cast<uint32_t*>(p);
    }
    HIP_TRY(hipMemcpyAsync(b->d_runs, runs.data(), runs.size() * sizeof(BatchRun<R>), hipMemcpyHostToDevice, s), "batch tables");
    HIP_TRY(hipMemcpyAsync(b->d_coefs, coefs.data(), coefs.size() * sizeof(StepCoef<R>), hipMemcpyHostToDevice, s), "batch tables");
    HIP_TRY(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s), "batch tables");
    HIP_TRY(hipStreamSynchronize(s), "batch tables");
    return LBM_OK;
}

lbm_status batch_launch(lbm_batch* b, hipStream_t s);

// steps in one persistent launch (the item flags count steps of a launch)
constexpr int32_t PERSIST_MAX_STEPS = 64;

// k steps of every run: k launches of one step, or persistent launches of up
// to PERSIST_MAX_STEPS steps each
lbm_status batch_launch_steps(lbm_batch* b, hipStream_t s, int64_t k)
{
    if (b->mode != LBM_BATCH_PERSISTENT) {
        for (int64_t i = 0; i < k; ++i) {
            lbm_status st = batch_launch(b, s);
            if (st != LBM_OK) return st;
        }
        return LBM_OK;
    }
    const int32_t n_per = b->nitems_periodic, n_wall = b->nitems - b->nitems_periodic;
    const int wmode = n_wall == 0 ? 0 : (n_per == 0 ? 1 : 2);
    while (k > 0) {
        const int32_t m = (int32_t)std::min<int64_t>(k, PERSIST_MAX_STEPS);
        const hipError_t e = launch_batch_persistent<float>(
            static_cast<const BatchRun<float>*>(b->d_runs), b->n, static_cast<const StepCoef<float>*>(b->d_coefs),
            b->d_items, b->nitems, b->cur, m, b->scheme, b->regularize, wmode, b->d_sync, b->d_done, b->d_sync + 1,
            b->wait_limit, s);
        if (e != hipSuccess) return hip_fail(e, "persistent batch launch");
        b->cur ^= (m & 1);
        k -= m;
    }
    return LBM_OK;
}

lbm_status batch_launch(lbm_batch* b, hipStream_t s)
{
    const int32_t n_per = b->nitems_periodic, n_wall = b->nitems - b->nitems_periodic;
    const int wpg = (b->precision == LBM_FP32_DEV) ? LBM_PAIR : 1;
    auto launch = [&](const BatchItem* items, int32_t n, int wmode) -> hipError_t {
        if (b->precision == LBM_FP32_DEV)
            return launch_batch_step<float>(static_cast<const BatchRun<float>*>(b->d_runs),
                                            static_cast<const StepCoef<float>*>(b->d_coefs), items, n, b->cur,
                                            b->scheme, b->regularize, wmode, wpg, s);
        return launch_batch_step<double>(static_cast<const BatchRun<double>*>(b->d_runs),
                                         static_cast<const StepCoef<double>*>(b->d_coefs), items, n, b->cur,
                                         b->scheme, b->regularize, wmode, wpg, s);
    };
    // one launch per step; a batch of one boundary kind uses the kernel built
    // for that kind alone, a mixed batch the kernel that takes each item's
    // (as fast as two launches, one per kind, on the 32-run sweep)
    const hipError_t e = launch(b->d_items, b->nitems, n_wall == 0 ? 0 : (n_per == 0 ? 1 : 2));
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
    b->cur ^= 1;
    return LBM_OK;
}

void batch_advance_members(lbm_batch* b, int64_t nsteps)
{
    b->step += nsteps;
    for (auto& r : b->runs) {
        r.cur = b->cur;
        r.step = b->step;
    }
}

}  // namespace

extern "C" {

lbm_status lbm_batch_init(int32_t n, const lbm_params* params, void* d_ws, size_t ws_bytes, void* stream,
                          const double* const* h_rho0, const double* const* h_ux0, const double* const* h_uy0,
                          lbm_batch** out)
{
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    if (n < 1 || !params || !h_rho0 || !h_ux0 || !h_uy0) return fail(LBM_EINVAL, "bad batch arguments");
    for (int i = 0; i < n; ++i) {
        lbm_status st = validate(&params[i]);
        if (st != LBM_OK) return fail(st, "run " + std::to_string(i) + ": " + g_error);
        if (params[i].precision != params[0].precision || params[i].scheme != params[0].scheme
            || params[i].regularize != params[0].regularize)
            return fail(LBM_EINVAL, "all runs of a batch must share precision, scheme and regularize");
    }
    const size_t need = lbm_batch_workspace_bytes(n, params);
    if (!d_ws) return fail(LBM_EINVAL, "null workspace");
    if (ws_bytes < need) return fail(LBM_ENOMEM, "workspace smaller than lbm_batch_workspace_bytes()");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_EINVAL, "out of host memory");
    b->n = n;
    b->precision = params[0].precision;
    b->scheme = params[0].scheme;
    b->regularize = params[0].regularize;
    b->runs.resize(n);
    char* p = static_cast<char*>(d_ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) {
        lbm_run* r = nullptr;
        lbm_status st = init_common(&params[i], p, run_bytes(&params[i]), stream, h_rho0[i], h_ux0[i], h_uy0[i], true, &r);
        if (st != LBM_OK) {
            delete b;
            return fail(st, "run " + std::to_string(i) + ": " + g_error);
        }
        b->runs[i] = *r;
        delete r;
        b->runs[i].batch = b;
        {
            std::lock_guard<std::mutex> lk(g_tune_mutex);
            const lbm_params& q = params[i];
            auto it = g_batch_tuned.find({q.Lx, q.Ly, q.precision, q.scheme, q.regularize, q.bc_y});
            if (it != g_batch_tuned.end()) b->runs[i].launch.rows_per_wave = it->second;
        }
        p += run_bytes(&params[i]);
    }
    lbm_status st = (b->precision == LBM_FP32_DEV) ? batch_tables<float>(b, p, s) : batch_tables<double>(b, p, s);
    if (st == LBM_OK && hipMemset(b->d_sync, 0, ALIGN) != hipSuccess) st = fail(LBM_EDEVICE, "batch init: sync words");
    if (st != LBM_OK) {
        delete b;
        return st;
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps, int32_t graph_steps, void* stream)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (nsteps < 0 || graph_steps < 0) return fail(LBM_EINVAL, "negative step count");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t done = 0;
    // a captured graph alternates the two field buffers, so it holds an even
    // number of steps and is replayed from an even parity only
    const int32_t gsteps = graph_steps - (graph_steps & 1);
    if (gsteps > 0) {
        if (b->exec && b->graph_steps != gsteps) {
            (void)hipGraphExecDestroy(b->exec);
            (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
        }
        while (nsteps - done >= gsteps) {
            if (b->cur != 0) {
                lbm_status st = batch_launch_steps(b, s, 1);
                if (st != LBM_OK) return st;
                batch_advance_members(b, 1);
                ++done;
                continue;
            }
            if (!b->exec) {
                if (!b->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking), "capture stream");
                HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
                const int saved = b->cur;
                lbm_status st = batch_launch_steps(b, b->capture_stream, gsteps);
                if (st != LBM_OK) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(b->capture_stream, &g);
                    if (g) (void)hipGraphDestroy(g);
                    b->cur = saved;
                    return st;
                }
                b->cur = saved;
                HIP_TRY(hipStreamEndCapture(b->capture_stream, &b->graph), "end capture");
                HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
                b->graph_steps = gsteps;
            }
            HIP_TRY(hipGraphLaunch(b->exec, s), "graph launch");
            // gsteps is even: the parity is unchanged
            batch_advance_members(b, gsteps);
            done += gsteps;
        }
    }
    if (done < nsteps) {
        lbm_status st = batch_launch_steps(b, s, nsteps - done);
        if (st != LBM_OK) return st;
        batch_advance_members(b, nsteps - done);
    }
    return LBM_OK;
}

lbm_status lbm_init_batch(int32_t n, const lbm_params* params, void* d_ws, size_t ws_bytes, void* stream,
                          const double* const* h_rho0, const double* const* h_ux0, const double* const* h_uy0,
                          lbm_batch** out)
{
    return lbm_batch_init(n, params, d_ws, ws_bytes, stream, h_rho0, h_ux0, h_uy0, out);
}

lbm_status lbm_step_batch(lbm_batch* b, int64_t nsteps, void* stream)
{
    return lbm_batch_step(b, nsteps, LBM_BATCH_GRAPH_STEPS, stream);
}

lbm_status lbm_batch_set_mode(lbm_batch* b, int32_t mode, void* stream)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (mode != LBM_BATCH_PER_STEP && mode != LBM_BATCH_PERSISTENT) return fail(LBM_EINVAL, "unknown batch mode");
    if (mode == LBM_BATCH_PERSISTENT && b->precision != LBM_FP32_DEV)
        return fail(LBM_EINVAL, "the persistent batched launch needs FP32 storage");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "batch set mode");
    b->mode = mode;
    drop_graph(b);
    return LBM_OK;
}

int32_t lbm_batch_get_mode(const lbm_batch* b) { return b ? b->mode : -1; }

lbm_status lbm_batch_set_wait_limit(lbm_batch* b, uint32_t polls, void* stream)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "batch wait limit");
    b->wait_limit = polls ? polls : DEFAULT_WAIT_LIMIT;
    drop_graph(b);
    return LBM_OK;
}

lbm_status lbm_batch_sync_status(lbm_batch* b, void* stream)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(s), "batch status");
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, b->d_sync + 1, sizeof(err), hipMemcpyDeviceToHost), "batch status");
    if (err) {
        HIP_TRY(hipMemset(b->d_sync + 1, 0, sizeof(uint32_t)), "batch status");
        return fail(LBM_EDEVICE, "a dependency wait of the persistent batched launch exceeded its bound; "
                                 "the states advanced since the last check are invalid");
    }
    return LBM_OK;
}

lbm_run* lbm_batch_run(lbm_batch* b, int32_t r)
{
    if (!b || r < 0 || r >= b->n) {
        g_error = "batch run index out of range";
        return nullptr;
    }
    return &b->runs[r];
}

lbm_status lbm_batch_set_launch(lbm_batch* b, int32_t rows_per_wave, void* stream)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (rows_per_wave < 1) return fail(LBM_EINVAL, "rows_per_wave must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(s), "batch set launch");
    for (auto& r : b->runs) r.launch.rows_per_wave = rows_per_wave;
    drop_graph(b);
    char* base = static_cast<char*>(b->d_runs);
    return (b->precision == LBM_FP32_DEV) ? batch_tables<float>(b, base, s) : batch_tables<double>(b, base, s);
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t steps_per_trial, void* stream, int32_t* rows_per_wave)
{
    if (!b || !rows_per_wave) return fail(LBM_EINVAL, "null argument");
    if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "batch autotune");
    HIP_TRY(hipEventCreate(&e1), "batch autotune");
    // device time per step of a trial with the batch's current work list and
    // mode (one untimed step first): steps_per_trial steps, or in one
    // persistent launch at least PERSIST_TRIAL_STEPS, since that launch's
    // start and end are shared by all its steps
    constexpr int32_t PERSIST_TRIAL_STEPS = 16;
    auto trial = [&](double* ms_out) -> lbm_status {
        const int32_t k = b->mode == LBM_BATCH_PERSISTENT ? std::max(steps_per_trial, PERSIST_TRIAL_STEPS)
                                                          : steps_per_trial;
        lbm_status st = lbm_batch_step(b, 1, 0, stream);
        if (st != LBM_OK) return st;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(LBM_EDEVICE, "batch autotune event");
        st = lbm_batch_step(b, k, 0, stream);
        if (st != LBM_OK) return st;
        float ms = 0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess
            || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(LBM_EDEVICE, "batch autotune timing");
        *ms_out = ms / k;
        return lbm_batch_sync_status(b, stream);
    };
    // rebuild the work list with the rows now set on each member
    auto retable = [&]() -> lbm_status {
        HIP_TRY(hipStreamSynchronize(s), "batch autotune");
        drop_graph(b);
        char* base = static_cast<char*>(b->d_runs);
        return (b->precision == LBM_FP32_DEV) ? batch_tables<float>(b, base, s) : batch_tables<double>(b, base, s);
    };
    lbm_status st = LBM_OK;
    // 1. one rows value for every run, in each launch mode the batch can use
    // (FP32: one launch per step, or the persistent launch); the fastest
    // pair of mode and rows is kept
    const int rows_c[] = {16, 24, 32, 40, 48, 64, 96, 128, 192, 256};
    double best = 1e300;
    int best_rows = rows_c[0];
    int best_mode = LBM_BATCH_PER_STEP;
    const int modes[2] = {LBM_BATCH_PER_STEP, LBM_BATCH_PERSISTENT};
    const int nmodes = b->precision == LBM_FP32_DEV ? 2 : 1;
    for (int mi = 0; mi < nmodes && st == LBM_OK; ++mi) {
        st = lbm_batch_set_mode(b, modes[mi], stream);
        for (int rows : rows_c) {
            if (st != LBM_OK) break;
            double ms = 0;
            st = lbm_batch_set_launch(b, rows, stream);
            if (st == LBM_OK) st = trial(&ms);
            if (st != LBM_OK) break;
            if (ms < best) {
                best = ms;
                best_rows = rows;
                best_mode = modes[mi];
            }
        }
    }
    if (st == LBM_OK) st = lbm_batch_set_mode(b, best_mode, stream);
    if (st == LBM_OK) st = lbm_batch_set_launch(b, best_rows, stream);
    // 2. then each class of runs (lattice shape and boundary), largest total
    // node count first, tries other rows values with the rest fixed and keeps
    // one that is faster by more than 1%
    std::map<std::tuple<int, int, int>, int64_t> nodes_of;
    for (auto& r : b->runs) nodes_of[{r.p.Lx, r.p.Ly, r.p.bc_y}] += (int64_t)r.p.Lx * r.p.Ly;
    std::vector<std::pair<int64_t, std::tuple<int, int, int>>> classes;
    for (auto& kv : nodes_of) classes.push_back({kv.second, kv.first});
    std::sort(classes.begin(), classes.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    if (st == LBM_OK && classes.size() > 1) st = trial(&best);
    for (size_t c = 0; st == LBM_OK && c < classes.size(); ++c) {
        const auto key = classes[c].second;
        auto set_rows = [&](int rows) {
            for (auto& r : b->runs)
                if (std::make_tuple(r.p.Lx, r.p.Ly, r.p.bc_y) == key) r.launch.rows_per_wave = rows;
        };
        int keep = best_rows;
        for (int rows : {best_rows / 2, (3 * best_rows) / 4, (3 * best_rows) / 2, 2 * best_rows}) {
            if (rows < 8 || rows == best_rows) continue;
            double ms = 0;
            set_rows(rows);
            st = retable();
            if (st == LBM_OK) st = trial(&ms);
            if (st != LBM_OK) break;
            if (ms < 0.99 * best) {
                best = ms;
                keep = rows;
            }
        }
        set_rows(keep);
        if (st == LBM_OK) st = retable();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LBM_OK) return st;
    // batches created later in the process start from these shapes
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        for (auto& r : b->runs)
            g_batch_tuned[{r.p.Lx, r.p.Ly, r.p.precision, r.p.scheme, r.p.regularize, r.p.bc_y}] =
                r.launch.rows_per_wave;
    }
    *rows_per_wave = best_rows;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    delete b;
}

}  // extern "C"
