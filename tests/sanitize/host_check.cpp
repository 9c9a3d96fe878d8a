// Host-side checks of the C ABI under AddressSanitizer and UBSan: every call
// here validates or sizes without touching a GPU (the library is built with
// --offload-host-only for this driver, so it carries no device code).
// Exits 0 when every check holds; prints the first failure otherwise.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "lbm.h"

static int failures = 0;

#define CHECK(cond, what)                                                    \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "FAILED: %s (%s:%d)\n", what, __FILE__, __LINE__); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static lbm_params good(int Lx, int Ly, int precision, int walls)
{
    lbm_params p;
    std::memset(&p, 0, sizeof p);
    p.Lx = Lx;
    p.Ly = Ly;
    p.ds = 1.0;
    p.dt = 0.25;
    p.tau = 0.7;
    p.T = 0.95;
    p.a = 9.0 / 8.0;
    p.b = 1.0 / 3.0;
    p.kappa = 1.0;
    p.scheme = 2;
    p.regularize = 0;
    p.precision = precision;
    p.rho_ref = 1.2;
    p.bc_y = walls ? LBM_SHEAR_WALLS : LBM_PERIODIC;
    p.u_wall = walls ? 0.01 : 0.0;
    p.rho_wall = 1.3;
    p.clamp_radius = 0.0;
    p.clamp_rho = 1.3;
    p.rounding = LBM_ROUND_STOCHASTIC;
    return p;
}

// a rejected parameter set: non-OK status, a message, and no workspace size
static void expect_rejected(const lbm_params& p, const char* what)
{
    const lbm_status st = lbm_validate(&p);
    CHECK(st != LBM_OK, what);
    const char* msg = lbm_last_error();
    CHECK(msg && std::strlen(msg) > 0, "message of a rejected call");
    CHECK(lbm_workspace_bytes(&p) == 0, what);
}

int main()
{
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    CHECK(lbm_version() && std::strlen(lbm_version()) > 0, "version string");

    // valid sets of every kind, and their sizes
    for (int prec : {LBM_FP64, LBM_FP32_DEV})
        for (int walls : {0, 1})
            for (int scheme : {1, 2})
                for (int reg : {0, 1})
                    for (int dims : {0, 1, 2}) {
                        // the largest lattices: 2^26 stored rows x columns
                        // (FP32), one row fewer with FP64; walls store two
                        // ghost rows
                        const int Lx = dims == 0 ? 1 : (dims == 1 ? 37 : 8192);
                        const int Ly = dims == 0 ? 1
                                                 : (dims == 1 ? 23 : 8192 - (walls ? 2 : 0) - (prec == LBM_FP64 ? 1 : 0));
                        lbm_params p = good(Lx, Ly, prec, walls);
                        p.scheme = scheme;
                        p.regularize = reg;
                        CHECK(lbm_validate(&p) == LBM_OK, "valid parameters");
                        const size_t ws = lbm_workspace_bytes(&p);
                        const size_t field = (size_t)16 * Lx * (Ly + (walls ? 2 : 0)) * (prec == LBM_FP64 ? 8 : 4);
                        CHECK(ws >= 2 * field, "workspace holds two fields");
                    }
    {
        lbm_params p = good(64, 64, LBM_FP32_DEV, 0);
        p.clamp_radius = 20.0;
        CHECK(lbm_validate(&p) == LBM_OK, "clamp");
        p.rounding = LBM_ROUND_NEAREST;
        CHECK(lbm_validate(&p) == LBM_OK, "round to nearest");
        p = good(16, 16, LBM_FP64, 0);
        p.a = p.b = p.kappa = 0.0;
        CHECK(lbm_validate(&p) == LBM_OK, "ideal gas");
    }

    // rejected sets
    struct Bad {
        const char* what;
        void (*edit)(lbm_params&);
    };
    const Bad bad[] = {
        {"Lx = 0", [](lbm_params& p) { p.Lx = 0; }},
        {"Ly < 0", [](lbm_params& p) { p.Ly = -5; }},
        {"Lx * Ly overflow", [](lbm_params& p) { p.Lx = 1 << 20; p.Ly = 1 << 20; }},
        {"FP32 beyond 2^26 nodes", [](lbm_params& p) { p.Lx = 8192; p.Ly = 8193; }},
        {"INT32_MAX edge", [](lbm_params& p) { p.Lx = INT32_MAX; p.Ly = 1; }},
        {"ds = 0", [](lbm_params& p) { p.ds = 0.0; }},
        {"dt NaN", [](lbm_params& p) { p.dt = std::numeric_limits<double>::quiet_NaN(); }},
        {"dt beyond CFL", [](lbm_params& p) { p.dt = 0.5; }},
        {"dt < 0", [](lbm_params& p) { p.dt = -0.1; }},
        {"tau = 0", [](lbm_params& p) { p.tau = 0.0; }},
        {"tau inf", [](lbm_params& p) { p.tau = std::numeric_limits<double>::infinity(); }},
        {"T < 0", [](lbm_params& p) { p.T = -1.0; }},
        {"kappa < 0", [](lbm_params& p) { p.kappa = -1e-3; }},
        {"scheme 3", [](lbm_params& p) { p.scheme = 3; }},
        {"regularize 2", [](lbm_params& p) { p.regularize = 2; }},
        {"precision 7", [](lbm_params& p) { p.precision = 7; }},
        {"rho_ref = 0 with FP32", [](lbm_params& p) { p.rho_ref = 0.0; }},
        {"bc_y 5", [](lbm_params& p) { p.bc_y = 5; }},
        {"clamp_rho beyond 1/b", [](lbm_params& p) { p.clamp_radius = 5.0; p.clamp_rho = 3.5; }},
        {"rounding 9", [](lbm_params& p) { p.rounding = 9; }},
    };
    for (const Bad& b : bad) {
        lbm_params p = good(64, 64, LBM_FP32_DEV, 0);
        b.edit(p);
        expect_rejected(p, b.what);
    }
    {
        lbm_params p = good(64, 64, LBM_SHEAR_WALLS, 1);
        p.precision = LBM_FP64;
        p.rho_wall = nan;
        expect_rejected(p, "rho_wall NaN");
        p = good(64, 64, LBM_FP64, 1);
        p.u_wall = inf;
        expect_rejected(p, "u_wall inf");
    }
    CHECK(lbm_validate(nullptr) != LBM_OK, "null parameters");
    CHECK(lbm_workspace_bytes(nullptr) == 0, "null parameters size");

    // batch sizing
    {
        std::vector<lbm_params> ps = {good(256, 256, LBM_FP32_DEV, 0), good(384, 384, LBM_FP32_DEV, 1),
                                      good(37, 5, LBM_FP32_DEV, 0)};
        size_t singles = 0;
        for (auto& p : ps) singles += lbm_workspace_bytes(&p);
        const size_t total = lbm_batch_workspace_bytes((int32_t)ps.size(), ps.data());
        CHECK(total >= singles, "batch workspace covers its runs");
        CHECK(lbm_batch_workspace_bytes(0, ps.data()) == 0, "empty batch");
        CHECK(lbm_batch_workspace_bytes(3, nullptr) == 0, "null batch parameters");
        ps[1].tau = -1.0;
        CHECK(lbm_batch_workspace_bytes((int32_t)ps.size(), ps.data()) == 0, "batch with a bad run");
    }

    // calls that must refuse before any device work
    {
        lbm_params p = good(32, 32, LBM_FP32_DEV, 0);
        lbm_run* run = reinterpret_cast<lbm_run*>(0x1);
        std::vector<double> rho(32 * 32, 1.2), u(32 * 32, 0.0);
        CHECK(lbm_init(&p, nullptr, 1 << 20, nullptr, rho.data(), u.data(), u.data(), &run) != LBM_OK,
              "init without workspace");
        CHECK(run == nullptr, "failed init clears the handle");
        rho[77] = nan;
        CHECK(lbm_init(&p, reinterpret_cast<void*>(256), 1 << 30, nullptr, rho.data(), u.data(), u.data(), &run)
                  != LBM_OK,
              "init with a NaN density");
        CHECK(lbm_init(&p, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr) != LBM_OK, "init without output");
        CHECK(lbm_attach(&p, nullptr, 0, 0, &run) != LBM_OK, "attach without workspace");
        CHECK(lbm_attach(&p, reinterpret_cast<void*>(256), 1 << 30, -1, &run) != LBM_OK, "attach at step -1");
        CHECK(lbm_step(nullptr, 1, nullptr) != LBM_OK, "step of a null run");
        CHECK(lbm_moments(nullptr, nullptr, nullptr, nullptr, nullptr) != LBM_OK, "moments of a null run");
        CHECK(lbm_reduce(nullptr, 1.0, nullptr, nullptr) != LBM_OK, "reduce of a null run");
        lbm_stats stats;
        CHECK(lbm_reduce_field_static(&p, nullptr, 1.0, &stats, nullptr) != LBM_OK, "static reduce of no field");
        CHECK(lbm_reduce_field_static(&p, reinterpret_cast<void*>(256), nan, &stats, nullptr) != LBM_OK,
              "static reduce with a NaN threshold");
        CHECK(lbm_set_launch(nullptr, 32, 1) != LBM_OK, "launch of a null run");
        int32_t r = 0, w = 0;
        CHECK(lbm_get_launch(nullptr, &r, &w) != LBM_OK, "launch query of a null run");
        CHECK(lbm_autotune(&p, nullptr, 0, nullptr, 0, &r, &w) != LBM_OK, "autotune with zero steps");
        lbm_destroy(nullptr);
        const double* h[1] = {rho.data()};
        lbm_batch* batch = reinterpret_cast<lbm_batch*>(0x1);
        CHECK(lbm_batch_init(0, &p, nullptr, 0, nullptr, h, h, h, &batch) != LBM_OK, "empty batch init");
        CHECK(batch == nullptr, "failed batch init clears the handle");
        lbm_params two[2] = {good(32, 32, LBM_FP32_DEV, 0), good(32, 32, LBM_FP64, 0)};
        const double* h2[2] = {rho.data(), rho.data()};
        CHECK(lbm_batch_init(2, two, reinterpret_cast<void*>(256), 1 << 30, nullptr, h2, h2, h2, &batch) != LBM_OK,
              "batch of mixed precisions");
        CHECK(lbm_batch_step(nullptr, 1, 0, nullptr) != LBM_OK, "step of a null batch");
        CHECK(lbm_batch_set_launch(nullptr, 32, nullptr) != LBM_OK, "launch of a null batch");
        CHECK(lbm_batch_autotune(nullptr, 1, nullptr, &r) != LBM_OK, "autotune of a null batch");
        CHECK(lbm_batch_run(nullptr, 0) == nullptr, "member of a null batch");
        CHECK(lbm_batch_set_mode(nullptr, LBM_BATCH_PERSISTENT, nullptr) != LBM_OK, "mode of a null batch");
        CHECK(lbm_batch_get_mode(nullptr) == -1, "mode query of a null batch");
        CHECK(lbm_batch_set_wait_limit(nullptr, 1, nullptr) != LBM_OK, "wait limit of a null batch");
        CHECK(lbm_batch_sync_status(nullptr, nullptr) != LBM_OK, "status of a null batch");
        lbm_batch_destroy(nullptr);
    }

    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
