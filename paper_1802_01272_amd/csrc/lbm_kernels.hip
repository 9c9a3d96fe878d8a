// lbm_kernels.hip -- gfx950 kernels of the CTU lattice Boltzmann stepper.
//
// One time step of the 16-velocity, third-order isothermal lattice Boltzmann
// model of Sofonea et al. (arXiv:1802.01272), split in two explicit steps as
// in Sec. II C: advection first, then collision and force on the advected
// state,
//   f*_k = A_k(f^n),   f_k^{n+1} = f*_k - (dt/tau)(f*_k - f_k^eq) + dt F_k,
// with f^eq of Eq. (herfeq), F_k of Eq. (herforce), the acceleration of
// Eq. (eder) from 25-point stencils on the advected density (Sec. II B),
// optional regularization of f* (Eq. ereg) and CTU1 (Eq. ctueq) or CTU2
// (Sec. II C 2) advection A_k.
//
// Design (MI355X / CDNA4):
//  * A wavefront owns a strip of 64 consecutive columns (56 written, 4 halo
//    columns each side, periodic in x: advection reaches two columns, the
//    force stencils on the advected density two more) and marches up a chunk
//    of rows.  Every x-neighbour access is a DPP wave shift (lane i reads
//    lane i -+ 1); every y-neighbour is a register carried from earlier rows.
//    No barriers: each wavefront is independent.
//  * One pass per step: each loaded row of f^n feeds the advection of the row
//    two behind it; the advected row's density feeds the force stencils, and
//    the row two behind that is collided and stored.  Each value of f is read
//    from HBM once per step (plus the 8-column and 8-row halo) and written
//    once.  The advected rows that wait for their collision stay on chip, in
//    LDS, in FP64.
//  * CTU2 is evaluated in an equivalent rearranged form: the CTU1 bilinear
//    update (Eq. ctueq) plus, per node, the limited corrections X = S^x and
//    Y = S^y (division-free MC limiter) computed once per node and blended
//    with their upwind neighbours.  Up to rounding this equals the paper's
//    flux-difference form with the transverse R^y index read as
//    (i + (1 - s_x)/2, j + (1 - s_y)/2) and the S^y ratio taken in R^y.
//  * Collision and force together are one cubic polynomial in xi with 10
//    per-node coefficients (both f^eq/w_k and F_k/w_k are cubic in xi); it is
//    evaluated for the four sign variants of each velocity group through
//    even/odd parts.
//  * Storage is FP64, or FP32 deviations d_k = f_k - w_k rho_ref (advection
//    is linear and preserves constants, so it acts on d_k directly).  The
//    advective increment A_k(f) - f is formed from upwind differences, so it
//    is exactly zero on a constant field in any precision.  Node-local
//    arithmetic (moments, stencils, collision and force) is FP64 in both
//    storage modes.  With FP32 storage, a rounding that repeats identically
//    from step to step where the flow is nearly steady adds up coherently, so
//    the FP32 path avoids such roundings: the CTU1 part of the increment is
//    summed in FP64 with FP64 weights nu |xi_x| and nu |xi_y| (only the CTU2
//    corrections are FP32), the advected value f + (A f - f) is formed in
//    FP64, and the new deviation is rounded to FP32 stochastically (unbiased,
//    seeded per step).
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "lbm_internal.hpp"

namespace lbm {
namespace {

// ----------------------------------------------------------------------------
// compile-time loop

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// ----------------------------------------------------------------------------
// cross-lane shifts (DPP wave shifts; whole 64-lane wavefront, all lanes active)

constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i reads lane i-1
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i reads lane i+1

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
// value held by the lane of column i-1 / i+1
template <typename R> __device__ __forceinline__ R from_left(R v) { return dpp<DPP_WAVE_SHR1>(v); }
template <typename R> __device__ __forceinline__ R from_right(R v) { return dpp<DPP_WAVE_SHL1>(v); }
// value at column i - s (the upwind neighbour for a velocity of x-sign s)
template <int S, typename R>
__device__ __forceinline__ R upwind_x(R v)
{
    if constexpr (S > 0) return from_left(v);
    else return from_right(v);
}

// Raw buffer access: a field is addressed through two buffer descriptors
// (planes 0-7 and 8-15), a per-lane 32-bit byte offset inside the plane and a
// per-plane scalar byte offset, so no 64-bit address arithmetic runs on the
// vector units.  Requires 8 planes to span less than 4 GiB.
struct FieldRsrc {
    __amdgpu_buffer_rsrc_t half[2];
};
template <typename R>
__device__ __forceinline__ FieldRsrc make_field_rsrc(const R* base, int64_t plane)
{
    FieldRsrc f;
    f.half[0] = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, 0x00020000);
    f.half[1] = __builtin_amdgcn_make_buffer_rsrc((void*)(base + 8 * plane), (short)0, -1, 0x00020000);
    return f;
}
// CPOL: cache policy of the access.  0 = default; CPOL_DEVICE = device
// scope (SC1): loads see stores of other XCDs that have completed, stores
// complete at the device's point of coherence (the persistent batched launch,
// where a workgroup reads what workgroups on other XCDs wrote in the same
// launch).
constexpr int CPOL_DEVICE = 16;
template <int CPOL = 0>
__device__ __forceinline__ void buf_load(float& v, const FieldRsrc& f, int k, uint32_t voff, uint32_t pbytes)
{
    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(f.half[k >> 3], voff, (uint32_t)(k & 7) * pbytes, CPOL));
}
template <int CPOL = 0>
__device__ __forceinline__ void buf_load(double& v, const FieldRsrc& f, int k, uint32_t voff, uint32_t pbytes)
{
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(f.half[k >> 3], voff, (uint32_t)(k & 7) * pbytes, CPOL));
}
template <int CPOL = 0>
__device__ __forceinline__ void buf_store(float v, const FieldRsrc& f, int k, uint32_t voff, uint32_t pbytes)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), f.half[k >> 3], voff, (uint32_t)(k & 7) * pbytes, CPOL);
}
template <int CPOL = 0>
__device__ __forceinline__ void buf_store(double v, const FieldRsrc& f, int k, uint32_t voff, uint32_t pbytes)
{
    using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(f.half[0], 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), f.half[k >> 3], voff, (uint32_t)(k & 7) * pbytes, CPOL);
}

// 1/x for x of order one (densities, 1 - b rho): hardware reciprocal refined
// by two Newton steps, within an ulp or two of the correctly rounded quotient
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

// Storage rounding of an FP64 result to FP32.  With mask = 2^29 - 1 it rounds
// stochastically: a 29-bit offset u is added to the 29 low bits of the FP64
// significand that FP32 drops, and those bits are then cleared, so the
// magnitude rounds up with probability (dropped bits) / 2^29 and the stored
// value is unbiased.  u is the low word of a partner value of the same node
// XOR a per-step seed: for any fixed value, u is uniform over the seeds.  With
// mask = 0 it is the conversion's round-to-nearest-even.
__device__ __forceinline__ float store_round(double x, double partner, uint32_t seed, uint32_t mask)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t u = ((uint32_t)__builtin_bit_cast(uint64_t, partner) ^ seed) & mask;
    const uint64_t t = b + u;
    const uint64_t c = (t & 0xFFFFFFFF00000000ull) | (uint64_t)((uint32_t)t & ~mask);  // mask < 2^32
    return (float)__builtin_bit_cast(double, c);
}

// 32-bit integer hash (the "lowbias32" finaliser of C. Wellons' hash-prospector)
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Seed of this step's stochastic rounding (FP32 storage): the run's step
// counter seq[cur] hashed; the wavefront that owns strip 0 of chunk 0 writes
// seq[cur] + 1 to the other slot, which the next step reads (steps alternate
// cur like the two fields, so captured graphs keep advancing the seed).
template <typename R>
__device__ __forceinline__ uint32_t step_seed(uint32_t* seq, int cur, bool owner)
{
    if constexpr (sizeof(R) != 4) return 0u;
    const uint32_t n = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(seq + cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (owner && (threadIdx.x & (WAVE - 1)) == 0)
        __hip_atomic_store(seq + (cur ^ 1), n + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return mix32(n);
}

// CTU1 part b D2 + a (Dc + b (Du - Dc)) of the advective increment; with
// FOLD (FP64 storage, no walls) f is folded in, and the caller then adds only
// the corrections
template <bool FOLD>
__device__ __forceinline__ float ctu1_part(float, float D2, float Dc, float Du, float a, float b)
{
    return a * (Dc + b * (Du - Dc)) + b * D2;
}
template <bool FOLD>
__device__ __forceinline__ double ctu1_part(double f, double D2, double Dc, double Du, double a, double b)
{
    if constexpr (FOLD) return __builtin_fma(b, D2, f) + a * __builtin_fma(b, Du - Dc, Dc);
    else return a * __builtin_fma(b, Du - Dc, Dc) + b * D2;
}

// minmod(a, b) = median(a, b, 0): 0 when the signs differ, else the smaller one
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// MC-limited correction R Psi_MC(R_up / R) = minmod(2R, 2R_up, (R + R_up)/2)
// (0 for R = 0, no division), returned halved:
// minmod(minmod(R, R_up), (R + R_up)/4).
template <typename R>
__device__ __forceinline__ R mc_half(R r, R ru)
{
    return minmod(minmod(r, ru), R(0.25) * (r + ru));
}

// weights of the fourth-order isotropic 5x5 gradient, by |e|^2: exact to
// fourth order, isotropic fifth-order error, no cos(4 theta) term at seventh
// order; along an axis it is the central difference (2/3, -1/12).  The
// |e|^2 = 4 shell has weight 0.
template <typename R> struct G5W {
    static constexpr R w1 = R(2.0 / 5.0), w2 = R(7.0 / 45.0), w4 = R(0.0),
                       w5 = R(-1.0 / 45.0), w8 = R(1.0 / 720.0);
};

// ----------------------------------------------------------------------------
// The fused step for one wavefront strip.
//
// Rows are processed in order.  At iteration t the newest loaded row is
// r = y0 - 4 + t; row a = r - 2 is advected (it needs f at rows a-2 .. a+2),
// and row o = a - 2 is collided and stored (for t >= 8): its force stencils
// need the advected density of rows o-2 .. o+2.  Per velocity, the ring B
// holds f^n at rows a-1, a, a+1 and the new row a+2; the ring S holds the
// advected rows a-2, a-1 and a until row a-2 is collided.

// ROLE 0: one wavefront does the whole march.  ROLE 1 / ROLE 2: the advecting
// and the colliding wavefront of a pair that shares the LDS ring of advected
// rows (pend) and a ring of their densities (dsl); one barrier per row, the
// collider one row behind the advector.
template <typename R, int SCHEME, bool REG, bool WALLS, int ROLE = 0, int CPOL = 0>
__device__ __forceinline__ void strip_step(const R* __restrict__ fin, R* __restrict__ fout,
                                           const StepCoef<R>* __restrict__ C,
                                           const int Lx, const int Ly, const int64_t plane,
                                           const int strip, const int y0, const int y1,
                                           double* __restrict__ pend, const uint32_t seed,
                                           double* __restrict__ dsl = nullptr)
{
    constexpr bool ADV = ROLE != 2, COL = ROLE != 1;
    using N = double;  // node-local arithmetic (moments, stencils, collision)
    const int lane = threadIdx.x & (WAVE - 1);
    int col = (strip * STRIP - HALO + lane) % Lx;
    if (col < 0) col += Lx;
    const bool out_lane = lane >= HALO && lane < WAVE - HALO && (strip * STRIP + lane - HALO) < Lx;
    // rows y0-4 .. y1+3 are read; the loop runs in groups of four (the ring
    // period), and the few extra rows of the last group are computed, not stored
    const int niter = (y1 - y0) + 8;
    const int niter4 = (niter + 3) & ~3;
    const FieldRsrc src = make_field_rsrc(fin, plane);
    const FieldRsrc dst = make_field_rsrc(fout, plane);
    const uint32_t pbytes = (uint32_t)(plane * (int64_t)sizeof(R));

    // where row r comes from: a lattice row (wrapped periodically), or with
    // walls one of the two ghost rows stored after the lattice rows of each
    // plane (row Ly below the lattice, row Ly + 1 above).  No branch: the
    // row index is selected on the scalar unit.
    auto row_voff = [&](int r) -> uint32_t {
        int rr;
        if constexpr (WALLS) {
            rr = (r < 0) ? Ly : ((r >= Ly) ? Ly + 1 : r);
        } else {
            rr = r % Ly;
            if (rr < 0) rr += Ly;
        }
        return ((uint32_t)rr * (uint32_t)Lx + (uint32_t)col) * (uint32_t)sizeof(R);
    };

    // Rings of four rows per velocity, indexed by phase P (= t mod 4): B[P]
    // holds the new row r, and B[P+1], B[P+2], B[P+3] (mod 4) hold rows a-1,
    // a, a+1.  Roles move by index, never by copying.  Row r+1 is loaded
    // during phase P into B[P+1] once row a-1 has been used.  The advected
    // rows wait for their collision in four LDS slots of this wavefront,
    // indexed the same way (slot P receives row a; slots P+2, P+3 hold rows
    // a-2, a-1; each lane reads back only what it wrote, so no barrier is
    // needed).  They are kept in FP64: with FP32 storage the advected value
    // f + (A f - f) is the exact FP64 sum of two FP32 values, so the
    // collision starts from it unrounded.
    R B[4][16];
    // carries per velocity: the upwind x-difference D1 of the row the CTU1
    // part reuses, and for CTU2 Y' at row a, dX = X'_{i+1} - X'_i at row
    // a-1 (s_y > 0) or a (s_y < 0), and the y-difference that the limiter of
    // row a formed and row a+1 reuses as its D2: R^y at row a+1 (s_y > 0,
    // D2 = -R^y) or R^y at row a+2 (s_y < 0)
    // FP32 storage sums the CTU1 part in FP64, with FP64 weights nu |xi| and
    // an FP64 carry of D1: FP32-rounded weights shift the effective advection
    // speed by a few 1e-8 every step, which moves a growing bubble's interface
    // coherently (after 10^4 steps on a 1024^2 cavitation run, rho and u
    // errors at the interface 3-4x larger).  The CTU2 corrections stay FP32.
    // The regularized CTU2 kernel keeps the FP32 sum with the two FP32
    // weights: the FP64 carries push its advecting wavefront past 256
    // registers (spills to scratch).
    constexpr bool SUM64 = sizeof(R) == 4 && (SCHEME == 1 || !REG);
    using CD = std::conditional_t<SUM64, N, R>;
    CD cD1[16];
    R cY[16], cdX[16], cR2[16];
    // The D2 carry saves 16 subtractions per row but changes the compiler's
    // schedule: at 6144^2 it makes the FP64 CTU2 kernel 2% and the FP32
    // regularized kernel 4.5% faster, the FP64 regularized kernel 3.5% and
    // the FP32 CTU2 kernel 0.3% slower, so only the first two use it.
    constexpr bool CARRY_D2 = SCHEME == 2 && ((sizeof(R) == 8) != REG);
    // per-row stencil rings (same indexing by phase): advected density
    // deviation sums and their x-sums (row a), Laplacian rows and their
    // x-differences and x-sums (row a-1), pending 5x5 gradient sums
    // (rows a-2 .. a+1)
    N dsr[4], hsr[4], Lr[4], dLr[4], sLr[4], ax[4], ay[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) B[i][k] = R(0);
        dsr[i] = hsr[i] = Lr[i] = dLr[i] = sLr[i] = ax[i] = ay[i] = N(0);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        cD1[k] = CD(0);
        cY[k] = cdX[k] = cR2[k] = R(0);
    }
    if constexpr (ADV) {
        const uint32_t voff = row_voff(y0 - 4);
#pragma unroll
        for (int k = 0; k < 16; ++k) buf_load<CPOL>(B[0][k], src, k, voff, pbytes);
    }

    // COLL = false: the first eight rows of the march only fill the rings
    // (advection, density, stencil sums); nothing is collided or stored.
    // WORK = false: the row only loads (its advected row lies below any
    // stencil of the chunk)
    auto body = [&](auto ph, auto coll, const int t, auto work) {
        constexpr bool COLL = decltype(coll)::value;
        constexpr bool WORK = decltype(work)::value;
        constexpr int P = decltype(ph)::value;
        constexpr int iN = P, iM1 = (P + 1) & 3, i0 = (P + 2) & 3, iP1 = (P + 3) & 3;
        R(&cur)[16] = B[iN];
        R(&fm1)[16] = B[iM1];
        R(&f0)[16] = B[i0];
        R(&fp1)[16] = B[iP1];
        N fs[16];                                  // advected row a (written here)
        const int r = y0 - 4 + t;
        const int a = r - 2;
        const int o = a - 2;
        const bool ghost_a = WALLS && (a < 0 || a >= Ly);
        // wall ghost rows are boundary values that keep their state: the
        // increment is multiplied by keep = 0 there (a select would let the
        // compiler branch around each velocity's advection)
        const N keep = ghost_a ? 0.0 : 1.0;
        constexpr bool FOLD = sizeof(R) == 8 && !WALLS;
        // FP32 CTU2: the four corrections accumulate onto the CTU1 part
        constexpr bool ACC = sizeof(R) == 4 && SCHEME == 2;
        // Row a-1 is only needed through D2 = f(a-1) - f(a) of the velocities
        // with s_y > 0 (CTU1; CTU2 carries it): form those, then load row r+1
        // into its slot B[iM1]
        // before any store of this row (loads and stores share one in-order
        // completion counter, so the next row's wait then never waits on
        // this row's stores).
        N ds_r;
        if constexpr (ADV && !WORK) {
            const uint32_t nvoff = row_voff(r + 1);
#pragma unroll
            for (int k = 0; k < 16; ++k) buf_load<CPOL>(fm1[k], src, k, nvoff, pbytes);
            // the D2 carry of the first advecting row (the rows it reads are
            // loaded by the last of these rows)
            if constexpr (CARRY_D2) {
#pragma unroll
                for (int k = 0; k < 16; ++k) cR2[k] = (sign_y(k) > 0) ? fp1[k] - f0[k] : cur[k] - fp1[k];
            }
            if constexpr (ROLE == 1) __syncthreads();
        }
        if constexpr (ADV && WORK) {
        // CTU1: D2 = f(a-1) - f(a) of the velocities with s_y > 0 (CTU2
        // carries it from the previous row's limiter)
        R D2m[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (!CARRY_D2 && sign_y(k) > 0) D2m[k] = fm1[k] - f0[k];
        {
            const uint32_t nvoff = row_voff(r + 1);
#pragma unroll
            for (int k = 0; k < 16; ++k) buf_load<CPOL>(fm1[k], src, k, nvoff, pbytes);
        }

        // --- first step of the split: advection of row a -----------------------
        static_for<0, 16>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            constexpr int SX = sign_x(K), SY = sign_y(K), MX = mag_x(K), MY = mag_y(K);
            const R fj = f0[K];
            // advective increment A_k(f) - f from upwind differences (exact on
            // constants): with D1 = f(i - s_x) - f(i) on row a (Dc) and on the
            // row upwind in y (Du), and D2 = f(a - s_y) - f(a), the CTU1 part
            // is b D2 + a (Dc + b (Du - Dc)), a = nu |xi_x|, b = nu |xi_y|.
            // With only the two weights a and b, D1 enters with weight exactly
            // a where Du = Dc, in any precision (separately rounded FP32
            // weights a - ab, ab and a break that identity, a bias that
            // repeats step after step).  D1 of the row that is reused one row
            // later is carried in cD1.
            const R ax = C->nu_xi[MX], ay = C->nu_xi[MY];
            // FP64 weights nu |xi| (from values the kernel holds anyway; a
            // separate FP64 table in the coefficient block pushed the
            // advecting wavefront past 256 registers)
            const N axd = C->dt * C->inv_ds * (MX ? QL : QS), ayd = C->dt * C->inv_ds * (MY ? QL : QS);
            R inc = 0;    // CTU1 part (FOLD: f + CTU1 part)
            N inc64 = 0;  // SUM64: CTU1 part, plus f without walls
            R corr = 0;   // CTU2 corrections
            if constexpr (SY > 0) {
                const R rx = fj - from_left(fj);          // R^x at row a
                const R rxu = upwind_x<SX>(rx);           // R^x at i - s_x
                const R D1 = (SX > 0) ? -rx : rxu;
                const R D2 = CARRY_D2 ? -cR2[K] : D2m[K];
                if constexpr (SUM64) {
                    const N Dc = (N)D1, Du = cD1[K];
                    inc64 = __builtin_fma(ayd, (N)D2, WALLS ? 0.0 : (N)fj) + axd * __builtin_fma(ayd, Du - Dc, Dc);
                    cD1[K] = Dc;
                } else {
                    const R Dc = D1, Du = cD1[K];
                    inc = ctu1_part<FOLD>(fj, D2, Dc, Du, ax, ay);
                    cD1[K] = Dc;
                }
                if constexpr (SCHEME == 2) {
                    // X' at row a and its x-difference; dX of row a-1 is carried
                    const R X = mc_half(rx, rxu);
                    const R dXj = from_right(X) - X;
                    // Y' at row a+1 (ratio with R^y of row a = -D2); Y' of row a is carried
                    const R Ry1 = fp1[K] - fj;
                    const R Y1 = mc_half(Ry1, -D2);
                    if constexpr (CARRY_D2) cR2[K] = Ry1;
                    const R dY = Y1 - cY[K];
                    if constexpr (ACC) {
                        inc = __builtin_fmaf(C->xs1[MX][MY], dXj, inc);
                        inc = __builtin_fmaf(C->xs2[MX][MY], cdX[K], inc);
                        inc = __builtin_fmaf(C->ys1[MX][MY], dY, inc);
                        inc = __builtin_fmaf(C->ys2[MX][MY], upwind_x<SX>(dY), inc);
                    } else {
                        corr = C->xs1[MX][MY] * dXj + C->xs2[MX][MY] * cdX[K] + C->ys1[MX][MY] * dY
                             + C->ys2[MX][MY] * upwind_x<SX>(dY);
                    }
                    cdX[K] = dXj;
                    cY[K] = Y1;
                }
            } else {
                const R fjp = fp1[K];
                const R rx = fjp - from_left(fjp);        // R^x at row a+1
                const R rxu = upwind_x<SX>(rx);
                const R D1p = (SX > 0) ? -rx : rxu;       // D1 of row a+1
                const R D2 = CARRY_D2 ? cR2[K] : fjp - fj;
                if constexpr (SUM64) {
                    const N Dc = cD1[K], Du = (N)D1p;
                    inc64 = __builtin_fma(ayd, (N)D2, WALLS ? 0.0 : (N)fj) + axd * __builtin_fma(ayd, Du - Dc, Dc);
                    cD1[K] = Du;
                } else {
                    const R Dc = cD1[K], Du = D1p;
                    inc = ctu1_part<FOLD>(fj, D2, Dc, Du, ax, ay);
                    cD1[K] = Du;
                }
                if constexpr (SCHEME == 2) {
                    // X' at row a+1 and its x-difference; dX of row a is carried
                    const R X = mc_half(rx, rxu);
                    const R dXjp = from_right(X) - X;
                    // Y' at row a+1 (ratio with R^y of row a+2); Y' of row a is carried
                    const R Ry2 = cur[K] - fjp;
                    const R Y1 = mc_half(D2, Ry2);
                    if constexpr (CARRY_D2) cR2[K] = Ry2;
                    const R dY = Y1 - cY[K];
                    if constexpr (ACC) {
                        inc = __builtin_fmaf(C->xs1[MX][MY], cdX[K], inc);
                        inc = __builtin_fmaf(C->xs2[MX][MY], dXjp, inc);
                        inc = __builtin_fmaf(C->ys1[MX][MY], dY, inc);
                        inc = __builtin_fmaf(C->ys2[MX][MY], upwind_x<SX>(dY), inc);
                    } else {
                        corr = C->xs1[MX][MY] * cdX[K] + C->xs2[MX][MY] * dXjp + C->ys1[MX][MY] * dY
                             + C->ys2[MX][MY] * upwind_x<SX>(dY);
                    }
                    cdX[K] = dXjp;
                    cY[K] = Y1;
                }
            }
            // f + increment in FP64 (FP32 storage: exact from the two FP32
            // operands)
            if constexpr (SUM64) {
                // CTU2: plus the FP32 corrections accumulated in inc
                N sum = inc64;
                if constexpr (SCHEME == 2) sum += (N)inc;
                if constexpr (WALLS) fs[K] = __builtin_fma(keep, sum, (N)fj);
                else fs[K] = sum;
            } else if constexpr (FOLD) fs[K] = inc + corr;
            else if constexpr (ACC) {
                if constexpr (WALLS) fs[K] = __builtin_fma(keep, (N)inc, (N)fj);
                else fs[K] = (N)fj + (N)inc;
            }
            else if constexpr (WALLS) fs[K] = __builtin_fma(keep, (N)(inc + corr), (N)fj);
            else fs[K] = (N)fj + (N)(inc + corr);
        });

        // --- regularization of the advected row (Eq. ereg): project onto the
        // Hermite space of order <= 3.  Linear in f and exact on w_k rho_ref,
        // so it acts on the stored deviations as they are; a wall ghost state
        // (an equilibrium) is left as it is by the projection.
        if constexpr (REG) {
            {
                N c[4][4];  // c[m][n] = sum_k d_k He_m(xi_x) He_n(xi_y), m + n <= 3
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < 4; ++n) c[m][n] = N(0);
                static_for<0, 4>([&](auto gc) {
                    constexpr int G = decltype(gc)::value;
                    constexpr N qx = group_qx(G), qy = group_qy(G);
                    constexpr N hx[4] = {1.0, qx, qx * qx - 1.0, qx * qx * qx - 3.0 * qx};
                    constexpr N hy[4] = {1.0, qy, qy * qy - 1.0, qy * qy * qy - 3.0 * qy};
                    const N d0 = fs[4 * G], d1 = fs[4 * G + 1], d2 = fs[4 * G + 2], d3 = fs[4 * G + 3];
                    const N see = (d0 + d1) + (d2 + d3);   // even in x, even in y
                    const N soe = (d0 - d1) - (d2 - d3);   // odd in x
                    const N seo = (d0 + d1) - (d2 + d3);   // odd in y
                    const N soo = (d0 - d1) + (d2 - d3);   // odd in both
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int n = 0; n < 4 - m; ++n) {
                            const N s = (m & 1) ? ((n & 1) ? soo : soe) : ((n & 1) ? seo : see);
                            c[m][n] += hx[m] * hy[n] * s;
                        }
                });
                // coefficients of the reconstruction w_k sum c_mn He_m He_n / (m! n!)
                constexpr N fact[4] = {1.0, 1.0, 0.5, 1.0 / 6.0};
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < 4 - m; ++n) c[m][n] *= fact[m] * fact[n];
                static_for<0, 4>([&](auto gc) {
                    constexpr int G = decltype(gc)::value;
                    constexpr N qx = group_qx(G), qy = group_qy(G), w = group_w(G);
                    constexpr N hx[4] = {1.0, qx, qx * qx - 1.0, qx * qx * qx - 3.0 * qx};
                    constexpr N hy[4] = {1.0, qy, qy * qy - 1.0, qy * qy * qy - 3.0 * qy};
                    const N EE = c[0][0] + c[2][0] * hx[2] + c[0][2] * hy[2];
                    const N OE = c[1][0] * hx[1] + c[3][0] * hx[3] + c[1][2] * (hx[1] * hy[2]);
                    const N EO = c[0][1] * hy[1] + c[0][3] * hy[3] + c[2][1] * (hx[2] * hy[1]);
                    const N OO = c[1][1] * (hx[1] * hy[1]);
                    const N Pp = EE + OO, Pm = EE - OO, Sp = OE + EO, Sm = OE - EO;
                    fs[4 * G + 0] = w * (Pp + Sp);   // (+,+)
                    fs[4 * G + 1] = w * (Pm - Sm);   // (-,+)
                    fs[4 * G + 2] = w * (Pp - Sp);   // (-,-)
                    fs[4 * G + 3] = w * (Pm + Sm);   // (+,-)
                });
            }
        }

        // --- advected density of row a and the force stencils (Eq. eder) -----
        ds_r = fs[0];
#pragma unroll
        for (int k = 1; k < 16; ++k) ds_r += fs[k];
#pragma unroll
        for (int k = 0; k < 16; ++k) pend[(iN * 16 + k) * WAVE + lane] = fs[k];
        if constexpr (ROLE == 1) {
            dsl[iN * WAVE + lane] = ds_r;
            __syncthreads();
        }
        }  // ADV
        if constexpr (COL && !WORK) {
            if constexpr (ROLE == 2) __syncthreads();
        }
        if constexpr (COL && WORK) {
        if constexpr (ROLE == 2) {
            __syncthreads();
            ds_r = dsl[iN * WAVE + lane];
        }
        const N rho_r = C->rho0 + ds_r;
        // p^i - p^w = rho T - rho T/(1 - b rho) + a rho^2 = rho^2 (a - b T/(1 - b rho))
        const N phi_r = rho_r * rho_r * (C->a_vdw - C->b_vdw * C->T * recip(1.0 - C->b_vdw * rho_r));

        // 9-point isotropic Laplacian of rho at row a-1 (rho0 drops out)
        const N ds_m1 = dsr[iP1], ds_m2 = dsr[i0];
        const N hs_r = from_left(ds_r) + from_right(ds_r);
        const N L_m1 = (4.0 * (hsr[iP1] + ds_r + ds_m2) + hs_r + hsr[i0] - 20.0 * ds_m1) * C->inv_6ds2;
        const N Lrr = from_right(L_m1), Lll = from_left(L_m1);
        const N dL_m1 = Lrr - Lll, sL_m1 = Lrr + Lll;
        // 9-point isotropic gradient of the Laplacian at row o = a-2
        const N g3x = (1.0 / 3.0) * dLr[iP1] + (1.0 / 12.0) * (dL_m1 + dLr[i0]);
        const N g3y = (1.0 / 3.0) * (L_m1 - Lr[i0]) + (1.0 / 12.0) * (sL_m1 - sLr[i0]);
        dsr[iN] = ds_r;
        hsr[iN] = hs_r;
        Lr[iN] = L_m1;
        dLr[iN] = dL_m1;
        sLr[iN] = sL_m1;

        // fourth-order 5x5 gradient of p^i - p^w: row a adds to rows
        // a-2 .. a+2; ax/ay[(P + d) mod 4] hold the sums of row a-2+d
        N g5x, g5y;
        {
            using W = G5W<N>;
            const N p1 = from_right(phi_r), m1 = from_left(phi_r);
            const N p2 = from_right(p1), m2 = from_left(m1);
            const N dx1 = p1 - m1, dx2 = p2 - m2, s1 = p1 + m1, s2 = p2 + m2;
            static_assert(W::w4 == 0.0, "the |e|^2 = 4 shell is dropped below");
            const N A0 = W::w1 * dx1;
            const N A1 = W::w2 * dx1 + 2.0 * W::w5 * dx2;
            const N A2 = W::w5 * dx1 + 2.0 * W::w8 * dx2;
            const N B1 = W::w1 * phi_r + W::w2 * s1 + W::w5 * s2;
            const N B2 = W::w5 * s1 + W::w8 * s2;
            g5x = ax[iN] + A2;
            g5y = ay[iN] + 2.0 * B2;
            ax[iM1] += A1;
            ay[iM1] += B1;
            ax[i0] += A0;
            ax[iP1] += A1;
            ay[iP1] -= B1;
            ax[iN] = A2;
            ay[iN] = -2.0 * B2;
        }

        if constexpr (COLL) {
            // --- second step of the split: collision and force on row o ------------
            // advected row o = a - 2: LDS ring slot i0
            auto fo = [&](int k) -> N { return pend[(i0 * 16 + k) * WAVE + lane]; };
            // moments of the advected row o: u = sum f xi / rho, a2 = sum f (xi xi - I)
            // (w_k rho_ref drops out of both)
            N jx = 0, jy = 0, axx = 0, axy = 0, ayy = 0;
            static_for<0, 4>([&](auto gc) {
                constexpr int G = decltype(gc)::value;
                constexpr N qx = group_qx(G), qy = group_qy(G);
                const N d0 = fo(4 * G), d1 = fo(4 * G + 1), d2 = fo(4 * G + 2), d3 = fo(4 * G + 3);
                const N see = (d0 + d1) + (d2 + d3);
                const N soe = (d0 - d1) - (d2 - d3);
                const N seo = (d0 + d1) - (d2 + d3);
                const N soo = (d0 - d1) + (d2 - d3);
                jx += qx * soe;
                jy += qy * seo;
                axx += (qx * qx - 1.0) * see;
                ayy += (qy * qy - 1.0) * see;
                axy += (qx * qy) * soo;
            });

            const N ds_j = ds_m2;
            const N rho_j = C->rho0 + ds_j;
            const N inv_rho = recip(rho_j);
            const N gx = g5x * C->inv_ds * inv_rho + C->kappa_ds * g3x;
            const N gy = g5y * C->inv_ds * inv_rho + C->kappa_ds * g3y;
            const N ux = jx * inv_rho, uy = jy * inv_rho;

            // collision + force as dt/tau f^eq_k + dt F_k = w_k sum_mn c_mn xi_x^m xi_y^n;
            // in deviation storage c00 also absorbs -dt/tau rho_ref
            N c00, c10, c01, c20, c02, c11, c30, c21, c12, c03;
            {
                const N dtt = C->dt_tau, dt = C->dt, T1 = C->Tm1;
                const N hu = 0.5 * (ux * ux + uy * uy);
                const N hT = 0.5 * T1;
                const N tr = axx + ayy;
                const N vx = axx * gx + axy * gy, vy = axy * gx + ayy * gy;
                const N gu = gx * ux + gy * uy;
                const N lin = 1.0 - hu - 2.0 * T1;
                c00 = dtt * (ds_j - rho_j * (hu + T1)) - dt * rho_j * gu;
                c10 = dtt * rho_j * ux * lin + dt * (rho_j * gx - 0.5 * gx * tr - vx);
                c01 = dtt * rho_j * uy * lin + dt * (rho_j * gy - 0.5 * gy * tr - vy);
                c20 = dtt * rho_j * (0.5 * ux * ux + hT) + dt * rho_j * gx * ux;
                c02 = dtt * rho_j * (0.5 * uy * uy + hT) + dt * rho_j * gy * uy;
                c11 = dtt * rho_j * ux * uy + dt * rho_j * (gx * uy + gy * ux);
                c30 = dtt * rho_j * ux * (ux * ux * (1.0 / 6.0) + hT) + dt * 0.5 * gx * axx;
                c21 = dtt * rho_j * uy * (0.5 * ux * ux + hT) + dt * (gx * axy + 0.5 * gy * axx);
                c12 = dtt * rho_j * ux * (0.5 * uy * uy + hT) + dt * (0.5 * gx * ayy + gy * axy);
                c03 = dtt * rho_j * uy * (uy * uy * (1.0 / 6.0) + hT) + dt * 0.5 * gy * ayy;
            }

            // far-field clamp (Sec. III B): outside the circle the new state is
            // scaled by s = rho_ext / rho^{n+1}, where rho^{n+1} = rho* because the
            // collision and the force conserve mass.  With A = s (1 - dt/tau),
            // f^{n+1}_k = A f*_k + w_k s P_k, and in deviation storage
            // d^{n+1}_k = A d*_k + w_k (s P_k + (s - 1) rho_ref).
            N s = 1.0;
            if (C->clamp) {
                const N dx = (N)col - C->clamp_cx, dy = (N)o - C->clamp_cy;
                if (dx * dx + dy * dy > C->clamp_r2) s = C->clamp_rho * inv_rho;
            }
            const N A = s * (1.0 - C->dt_tau);
            c00 = s * c00 + (s - 1.0) * C->rho0;
            c10 *= s; c01 *= s; c20 *= s; c02 *= s; c11 *= s;
            c30 *= s; c21 *= s; c12 *= s; c03 *= s;

            const bool store_row = t >= 8 && o < y1;
            const uint32_t soff = ((uint32_t)o * (uint32_t)Lx + (uint32_t)col) * (uint32_t)sizeof(R);

            // f^{n+1}_k = A f*_k + w_k P_k for velocity 4G+s, from the even/odd
            // parts of the polynomial of group G, in FP64 with one rounding to
            // the storage precision (FP32: stochastic, the partner of velocity
            // 4G+s is 4G+(s^1))
            const uint32_t srm = C->sr_mask;
            static_for<0, 4>([&](auto gc) {
                constexpr int G = decltype(gc)::value;
                constexpr N qx = group_qx(G), qy = group_qy(G), wg = group_w(G);
                const N EE = c00 + c20 * (qx * qx) + c02 * (qy * qy);
                const N OE = qx * (c10 + c30 * (qx * qx) + c12 * (qy * qy));
                const N EO = qy * (c01 + c03 * (qy * qy) + c21 * (qx * qx));
                const N OO = (qx * qy) * c11;
                const N Pp = EE + OO, Pm = EE - OO, Sp = OE + EO, Sm = OE - EO;
                const N poly[4] = {wg * (Pp + Sp), wg * (Pm - Sm), wg * (Pp - Sp), wg * (Pm + Sm)};
                N xn[4];
    #pragma unroll
                for (int sv = 0; sv < 4; ++sv) xn[sv] = A * fo(4 * G + sv) + poly[sv];
    #pragma unroll
                for (int sv = 0; sv < 4; ++sv) {
                    const int K = 4 * G + sv;
                    R fnew;
                    if constexpr (sizeof(R) == 4) fnew = store_round(xn[sv], xn[sv ^ 1], seed, srm);
                    else fnew = (R)xn[sv];
                    if (store_row && out_lane) buf_store<CPOL>(fnew, dst, K, soff, pbytes);
                }
            });
        }
        }  // COL
    };

    // scheduling barriers keep the compiler from interleaving consecutive row
    // bodies (which would raise register pressure past the register file)
    using Z = std::integral_constant<bool, false>;
    using O = std::integral_constant<bool, true>;
    // FP32: the eight warm-up rows run a body without the collision; FP64
    // keeps one body for all rows (a second copy of the larger FP64 body
    // costs more in instruction fetch than the collisions it skips).
    constexpr bool PEEL = sizeof(R) == 4;
    int t0 = 0;
    if constexpr (PEEL) {
        t0 = 8;
        // rows t = 0..2 only load: they would advect rows below y0 - 3, which
        // no stencil of the chunk reaches, and row t = 3 forms afresh the
        // carries that row t = 4 needs
        body(std::integral_constant<int, 0>{}, Z{}, 0, Z{});
        body(std::integral_constant<int, 1>{}, Z{}, 1, Z{});
        body(std::integral_constant<int, 2>{}, Z{}, 2, Z{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 3>{}, Z{}, 3, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 0>{}, Z{}, 4, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 1>{}, Z{}, 5, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 2>{}, Z{}, 6, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 3>{}, Z{}, 7, O{});
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int t = t0; t < niter4; t += 4) {
        body(std::integral_constant<int, 0>{}, O{}, t, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 1>{}, O{}, t + 1, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 2>{}, O{}, t + 2, O{});
        __builtin_amdgcn_sched_barrier(0);
        body(std::integral_constant<int, 3>{}, O{}, t + 3, O{});
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Wavefront id -> workgroup order that keeps neighbouring strips on one XCD:
// workgroups are dealt round-robin to the 8 XCDs, so workgroup b runs on XCD
// b % 8; remap so that each XCD gets one contiguous range of logical ids.
__device__ __forceinline__ int xcd_logical_block(int b, int nblocks)
{
    constexpr int NXCD = 8;
    const int q = nblocks / NXCD, rem = nblocks % NXCD;
    const int x = b % NXCD, i = b / NXCD;
    return x * q + (x < rem ? x : rem) + i;
}

// dynamic LDS of a step workgroup: STEP_LDS_PER_WAVE bytes per wavefront
extern __shared__ __attribute__((aligned(16))) char step_lds[];
__device__ __forceinline__ double* wave_lds()
{
    return reinterpret_cast<double*>(step_lds) + (threadIdx.x / WAVE) * (PENDING_ROWS * 16 * WAVE);
}

// One wavefront per SIMD with the full register file (up to 512 registers,
// no spills to memory); the next row is prefetched to cover load latency.
template <typename R> struct WavesPerEU { static constexpr int value = 1; };

template <typename R, int SCHEME, bool REG, bool WALLS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WavesPerEU<R>::value))) void step_kernel(const R* __restrict__ fin, R* __restrict__ fout,
                                                   const StepCoef<R>* __restrict__ coef,
                                                   uint32_t* __restrict__ seq, int cur,
                                                   int Lx, int Ly, int64_t plane, int rows,
                                                   int nstrips, int nwaves)
{
    const int wpg = blockDim.x / WAVE;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    // the wavefront index is the same in all 64 lanes: keep it scalar
    const int wave = __builtin_amdgcn_readfirstlane(lb * wpg + (int)(threadIdx.x / WAVE));
    if (wave >= nwaves) return;  // whole wavefront leaves together
    const int chunk = wave / nstrips, strip = wave - chunk * nstrips;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, Ly);
    const uint32_t seed = step_seed<R>(seq, cur, wave == 0);
    strip_step<R, SCHEME, REG, WALLS>(fin, fout, coef, Lx, Ly, plane, strip, y0, y1, wave_lds(), seed);
}

// A pair of wavefronts per strip (workgroup of 128 lanes): wavefront 0
// advects, wavefront 1 collides and stores.  Each role needs only its own
// registers, so two wavefronts fit one SIMD.
template <typename R, int SCHEME, bool REG, bool WALLS>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void pair_step_kernel(
    const R* __restrict__ fin, R* __restrict__ fout, const StepCoef<R>* __restrict__ coef,
    uint32_t* __restrict__ seq, int cur, int Lx, int Ly, int64_t plane, int rows, int nstrips, int npairs)
{
    const int pair = __builtin_amdgcn_readfirstlane(xcd_logical_block(blockIdx.x, gridDim.x));
    if (pair >= npairs) return;  // the whole workgroup leaves together
    const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int chunk = pair / nstrips, strip = pair - chunk * nstrips;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, Ly);
    double* const pend = reinterpret_cast<double*>(step_lds);  // PAIR_STEP_LDS bytes
    double* const dsl = pend + PENDING_ROWS * 16 * WAVE;
    if (role == 0) {
        strip_step<R, SCHEME, REG, WALLS, 1>(fin, fout, coef, Lx, Ly, plane, strip, y0, y1, pend, 0u, dsl);
    } else {
        const uint32_t seed = step_seed<R>(seq, cur, pair == 0);
        strip_step<R, SCHEME, REG, WALLS, 2>(fin, fout, coef, Lx, Ly, plane, strip, y0, y1, pend, seed, dsl);
    }
}

// Boundary of a batched launch: WMODE 0 (all items periodic) or 1 (all with
// walls) fixes the body at compile time; WMODE 2 covers both kinds in one
// grid, each work item taking the body of its run's boundary on a branch that
// is uniform over the workgroup (the item and its run are scalar).  Every run
// computes exactly what its single-run kernel computes.
template <int WMODE, typename F>
__device__ __forceinline__ void with_walls(int walls, F&& f)
{
    if constexpr (WMODE == 2) {
        if (walls) f(std::integral_constant<bool, true>{});
        else f(std::integral_constant<bool, false>{});
    } else {
        f(std::integral_constant<bool, WMODE == 1>{});
    }
}

template <typename R, int SCHEME, bool REG, int WMODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WavesPerEU<R>::value))) void batch_step_kernel(const BatchRun<R>* __restrict__ runs,
                                                         const StepCoef<R>* __restrict__ coefs,
                                                         const BatchItem* __restrict__ items,
                                                         int nitems, int cur)
{
    const int wpg = blockDim.x / WAVE;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int w = __builtin_amdgcn_readfirstlane(lb * wpg + (int)(threadIdx.x / WAVE));
    if (w >= nitems) return;
    const BatchItem it = items[w];
    const BatchRun<R> run = runs[it.run];
    const int y0 = it.chunk * run.rows;
    const int y1 = min(y0 + run.rows, run.Ly);
    R* const fa = run.f[0];
    R* const fb = run.f[1];
    const uint32_t seed = step_seed<R>(run.seq, cur, it.strip == 0 && it.chunk == 0);
    with_walls<WMODE>(run.walls, [&](auto wl) {
        strip_step<R, SCHEME, REG, decltype(wl)::value>(cur ? fb : fa, cur ? fa : fb, coefs + it.run, run.Lx, run.Ly,
                                                        run.plane, it.strip, y0, y1, wave_lds(), seed);
    });
}

// The batched launch with a pair of wavefronts per work item (FP32 storage).
template <typename R, int SCHEME, bool REG, int WMODE>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void batch_pair_step_kernel(
    const BatchRun<R>* __restrict__ runs, const StepCoef<R>* __restrict__ coefs, const BatchItem* __restrict__ items,
    int nitems, int cur)
{
    const int w = __builtin_amdgcn_readfirstlane(xcd_logical_block(blockIdx.x, gridDim.x));
    if (w >= nitems) return;  // the whole workgroup leaves together
    const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const BatchItem it = items[w];
    const BatchRun<R> run = runs[it.run];
    const int y0 = it.chunk * run.rows;
    const int y1 = min(y0 + run.rows, run.Ly);
    R* const fa = run.f[0];
    R* const fb = run.f[1];
    double* const pend = reinterpret_cast<double*>(step_lds);  // PAIR_STEP_LDS bytes
    double* const dsl = pend + PENDING_ROWS * 16 * WAVE;
    with_walls<WMODE>(run.walls, [&](auto wl) {
        constexpr bool WL = decltype(wl)::value;
        if (role == 0) {
            strip_step<R, SCHEME, REG, WL, 1>(cur ? fb : fa, cur ? fa : fb, coefs + it.run, run.Lx, run.Ly,
                                              run.plane, it.strip, y0, y1, pend, 0u, dsl);
        } else {
            const uint32_t seed = step_seed<R>(run.seq, cur, it.strip == 0 && it.chunk == 0);
            strip_step<R, SCHEME, REG, WL, 2>(cur ? fb : fa, cur ? fa : fb, coefs + it.run, run.Lx, run.Ly,
                                              run.plane, it.strip, y0, y1, pend, seed, dsl);
        }
    });
}

// ----------------------------------------------------------------------------
// Persistent batched launch (FP32 storage, a pair of wavefronts per work
// item): one launch advances every run of the batch by nsteps, with no
// launch boundary between steps.  Workgroups take tickets t = s * nitems + i
// in order from one counter (item i of step s).  Before item i of step s
// reads its input, its advecting wavefront waits until every item whose
// output rows and columns overlap the item's input (its run's items within
// 4 rows and 4 columns, periodic wrap included) has finished step s - 1:
// that covers the reads of step s (the neighbours' outputs of step s - 1)
// and the writes of step s (the buffer that the neighbours read in step
// s - 1; the neighbourhood is symmetric).  A ticket only waits for smaller
// tickets, which running workgroups hold, so the launch always drains.
// Field accesses are device-coherent (CPOL_DEVICE), and the colliding
// wavefront publishes done[i] = s + 1 only after its stores have completed.
// Every wait is bounded: past wait_limit polls the launch sets *err, stops
// waiting and finishes (its results are then invalid).  The step counters
// of the stochastic rounding are read, not written; batch_seq_kernel moves
// them on after the launch.

// first index and count of the blocks of `per` (the last one ragged) of
// 0..L-1 that cover positions lo..hi, wrapped periodically or clipped
__device__ __forceinline__ void block_span(int lo, int hi, int L, int per, int nblk, bool wrap, int& first,
                                           int& count)
{
    if (!wrap) {
        lo = max(lo, 0);
        hi = min(hi, L - 1);
        first = lo / per;
        count = hi / per - first + 1;
        return;
    }
    if (hi - lo + 1 >= L) {
        first = 0;
        count = nblk;
        return;
    }
    lo = ((lo % L) + L) % L;
    hi = ((hi % L) + L) % L;
    first = lo / per;
    const int last = hi / per;
    // a range that wraps past L - 1 runs from block `first` to the end and
    // on from block 0 to `last`
    count = lo > hi ? min(last + nblk - first + 1, nblk) : last - first + 1;
}

__device__ __forceinline__ bool wait_done(const int32_t* done, int j, int s, uint32_t limit, uint32_t* err)
{
    uint32_t polls = 0;
    while (__hip_atomic_load(done + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < s) {
        if (++polls > limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

template <typename R, int SCHEME, bool REG, int WMODE>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void batch_persistent_kernel(
    const BatchRun<R>* __restrict__ runs, const StepCoef<R>* __restrict__ coefs, const BatchItem* __restrict__ items,
    int nitems, int cur0, int nsteps, uint32_t* __restrict__ ticket, int32_t* __restrict__ done,
    uint32_t* __restrict__ err, uint32_t wait_limit)
{
    __shared__ uint32_t tick;
    const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t total = (uint32_t)nitems * (uint32_t)nsteps;
    double* const pend = reinterpret_cast<double*>(step_lds);  // PAIR_STEP_LDS bytes
    double* const dsl = pend + PENDING_ROWS * 16 * WAVE;
    for (;;) {
        if (threadIdx.x == 0) tick = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(tick);
        __syncthreads();  // tick is read by both wavefronts before it is written again
        if (t >= total) break;
        const int s = (int)(t / (uint32_t)nitems);
        const int i = (int)(t - (uint32_t)s * (uint32_t)nitems);
        const BatchItem it = items[i];
        const BatchRun<R> run = runs[it.run];
        const int y0 = it.chunk * run.rows;
        const int y1 = min(y0 + run.rows, run.Ly);
        const int cur = (cur0 + s) & 1;
        R* const fa = run.f[0];
        R* const fb = run.f[1];
        if (role == 0 && s > 0 && lane == 0) {
            const int x0 = it.strip * STRIP;
            const int x1 = min(x0 + STRIP, run.Lx);
            const int nchunks = (run.Ly + run.rows - 1) / run.rows;
            int cf, cn, sf, sn;
            block_span(y0 - 4, y1 + 3, run.Ly, run.rows, nchunks, run.walls == 0, cf, cn);
            block_span(x0 - HALO, x1 - 1 + HALO, run.Lx, STRIP, run.nstrips, true, sf, sn);
            bool ok = true;
            for (int a = 0; a < cn && ok; ++a) {
                const int c = (cf + a) % nchunks;
                for (int b = 0; b < sn && ok; ++b)
                    ok = wait_done(done, run.item_base + c * run.nstrips + (sf + b) % run.nstrips, s, wait_limit, err);
            }
        }
        // the field loads below are not moved above the wait
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        with_walls<WMODE>(run.walls, [&](auto wl) {
            constexpr bool WL = decltype(wl)::value;
            if (role == 0) {
                strip_step<R, SCHEME, REG, WL, 1, CPOL_DEVICE>(cur ? fb : fa, cur ? fa : fb, coefs + it.run, run.Lx,
                                                               run.Ly, run.plane, it.strip, y0, y1, pend, 0u, dsl);
            } else {
                const uint32_t n0 = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(run.seq + cur0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                const uint32_t seed = mix32(n0 + (uint32_t)s);
                strip_step<R, SCHEME, REG, WL, 2, CPOL_DEVICE>(cur ? fb : fa, cur ? fa : fb, coefs + it.run, run.Lx,
                                                               run.Ly, run.plane, it.strip, y0, y1, pend, seed, dsl);
            }
        });
        if (role == 1) {
            // this wavefront's stores have completed before the item is published
            __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (lane == 0) __hip_atomic_store(done + i, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Clear the persistent launch's ticket counter and item flags.
__global__ void batch_reset_kernel(uint32_t* __restrict__ ticket, int32_t* __restrict__ done, int nitems)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nitems) done[i] = 0;
    if (i == 0) *ticket = 0u;
}

// After a persistent launch of nsteps steps from parity cur0: leave each
// run's step counter pair as nsteps launches of one step would
// (seq[(cur0 + nsteps) & 1] = n0 + nsteps, the other slot one less).
template <typename R>
__global__ void batch_seq_kernel(const BatchRun<R>* __restrict__ runs, int nruns, int cur0, int nsteps)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    uint32_t* seq = runs[r].seq;
    const uint32_t n0 = seq[cur0];
    seq[(cur0 + nsteps) & 1] = n0 + (uint32_t)nsteps;
    seq[(cur0 + nsteps + 1) & 1] = n0 + (uint32_t)nsteps - 1u;
}

// ----------------------------------------------------------------------------
// auxiliary kernels (all in FP64 arithmetic)

__device__ __forceinline__ double feq_k(int k, double T, double rho, double ux, double uy)
{
    // Eq. (herfeq)
    const double cx = xi_x(k), cy = xi_y(k);
    const double xu = cx * ux + cy * uy, u2 = ux * ux + uy * uy, x2 = cx * cx + cy * cy;
    return weight(k) * rho
         * (1.0 + xu + 0.5 * (xu * xu - u2 + (T - 1.0) * (x2 - 2.0))
            + xu * (1.0 / 6.0) * (xu * xu - 3.0 * u2 + 3.0 * (T - 1.0) * (x2 - 4.0)));
}

template <typename R>
__global__ void init_kernel(R* __restrict__ f, const StepCoef<R>* __restrict__ C, const double* __restrict__ rho,
                            const double* __restrict__ ux, const double* __restrict__ uy, int64_t n,
                            int64_t plane)
{
    const double T = (double)C->T;
    const double rho0 = (double)C->rho0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double r = rho[i], vx = ux[i], vy = uy[i];
#pragma unroll
        for (int k = 0; k < 16; ++k) f[k * plane + i] = (R)(feq_k(k, T, r, vx, vy) - weight(k) * rho0);
    }
}

template <typename R>
__global__ void moments_kernel(const R* __restrict__ f, const StepCoef<R>* __restrict__ C, double* __restrict__ rho,
                               double* __restrict__ ux, double* __restrict__ uy, int64_t n, int64_t plane)
{
    const double rho0 = (double)C->rho0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double v = (double)f[k * plane + i] + weight(k) * rho0;
            r += v;
            jx += v * xi_x(k);
            jy += v * xi_y(k);
        }
        rho[i] = r;
        ux[i] = jx / r;
        uy[i] = jy / r;
    }
}

template <typename R>
__global__ void get_plane_kernel(const R* __restrict__ f, const StepCoef<R>* __restrict__ C, int k,
                                 double* __restrict__ out, int64_t n, int64_t plane)
{
    const double off = weight(k) * (double)C->rho0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)f[k * plane + i] + off;
}

template <typename R>
__global__ void set_plane_kernel(R* __restrict__ f, const StepCoef<R>* __restrict__ C, int k,
                                 const double* __restrict__ in, int64_t n, int64_t plane)
{
    const double off = weight(k) * (double)C->rho0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        f[k * plane + i] = (R)(in[i] - off);
}

// Wall ghost rows, stored after the Ly lattice rows of every plane: row Ly
// holds the state below the lattice, row Ly + 1 the state above it.
template <typename R>
__global__ void fill_ghost_kernel(R* __restrict__ f, const StepCoef<R>* __restrict__ C, int Lx, int Ly,
                                  int64_t plane)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * (int64_t)Lx;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool low = i < Lx;
#pragma unroll
        for (int k = 0; k < 16; ++k) f[k * plane + (int64_t)Ly * Lx + i] = low ? C->ghost_lo[k] : C->ghost_hi[k];
    }
}

// FP64 sums over the lattice: mass, momentum, bubble count, non-finite count
// and the first and second position moments of the bubble (rho < threshold).
template <typename R>
__global__ __launch_bounds__(256) void reduce_kernel(const R* __restrict__ f, const StepCoef<R>* __restrict__ C,
                                                     int Lx, int Ly, int64_t plane, double threshold,
                                                     double* __restrict__ partials)
{
    const int64_t n = (int64_t)Lx * Ly;
    const double rho0 = (double)C->rho0;
    const double cxn = 0.5 * (Lx - 1), cyn = 0.5 * (Ly - 1);
    double acc[REDUCE_VALUES];
#pragma unroll
    for (int v = 0; v < REDUCE_VALUES; ++v) acc[v] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        bool finite = true;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double v = (double)f[k * plane + i] + weight(k) * rho0;
            finite = finite && isfinite(v);
            r += v;
            jx += v * xi_x(k);
            jy += v * xi_y(k);
        }
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        if (!finite) acc[4] += 1.0;
        if (r < threshold) {
            const int64_t jj = i / Lx;
            const double x = (double)(i - jj * Lx) - cxn, y = (double)jj - cyn;
            acc[3] += 1.0;
            acc[5] += x;
            acc[6] += y;
            acc[7] += x * x;
            acc[8] += x * y;
            acc[9] += y * y;
        }
    }
    // wavefront reduction, then across the workgroup's wavefronts in LDS
    __shared__ double lds[256 / WAVE][REDUCE_VALUES];
#pragma unroll
    for (int v = 0; v < REDUCE_VALUES; ++v) {
        double s = acc[v];
#pragma unroll
        for (int off = WAVE / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
        acc[v] = s;
    }
    const int wv = threadIdx.x / WAVE, ln = threadIdx.x & (WAVE - 1);
    if (ln == 0) {
#pragma unroll
        for (int v = 0; v < REDUCE_VALUES; ++v) lds[wv][v] = acc[v];
    }
    __syncthreads();
    if (threadIdx.x < REDUCE_VALUES) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s += lds[w][threadIdx.x];
        partials[blockIdx.x * REDUCE_VALUES + threadIdx.x] = s;
    }
}

// Sum of the block partials in a fixed order (deterministic).
__global__ __launch_bounds__(64) void reduce_final_kernel(const double* __restrict__ partials, int nblocks,
                                                          double* __restrict__ out)
{
    const int v = threadIdx.x;
    if (v < REDUCE_VALUES) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[b * REDUCE_VALUES + v];
        out[v] = s;
    }
}

int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers

template <typename R>
hipError_t launch_step(const RunView<R>& rv, int scheme, int regularize, int walls, int wpg, hipStream_t s)
{
    // wpg = LBM_PAIR: one workgroup of two wavefronts per strip and chunk
    // (FP32 storage only: the pair kernels are instantiated for FP32 alone);
    // else wpg independent wavefronts per workgroup
    const bool pair = wpg == LBM_PAIR;
    const int nchunks = (rv.Ly + rv.rows - 1) / rv.rows;
    const int nwaves = rv.nstrips * nchunks;  // pairs with LBM_PAIR
#define LBM_DISPATCH(LAUNCH)                       \
    if (scheme == 1) {                             \
        if (regularize) {                          \
            if (walls) LAUNCH(1, true, true);      \
            else LAUNCH(1, true, false);           \
        } else {                                   \
            if (walls) LAUNCH(1, false, true);     \
            else LAUNCH(1, false, false);          \
        }                                          \
    } else {                                       \
        if (regularize) {                          \
            if (walls) LAUNCH(2, true, true);      \
            else LAUNCH(2, true, false);           \
        } else {                                   \
            if (walls) LAUNCH(2, false, true);     \
            else LAUNCH(2, false, false);          \
        }                                          \
    }
    if constexpr (sizeof(R) == 4) {
        if (pair) {
#define LBM_PAIR_LAUNCH(SC, RG, WL)                                                                         \
    hipLaunchKernelGGL((pair_step_kernel<R, SC, RG, WL>), dim3(nwaves), dim3(2 * WAVE), PAIR_STEP_LDS, s, \
                       rv.f_in, rv.f_out, rv.coef, rv.seq, rv.cur, rv.Lx, rv.Ly, rv.plane, rv.rows,      \
                       rv.nstrips, nwaves)
            LBM_DISPATCH(LBM_PAIR_LAUNCH)
#undef LBM_PAIR_LAUNCH
            return hipGetLastError();
        }
    }
    if (pair) return hipErrorInvalidValue;
    const int nblocks = (nwaves + wpg - 1) / wpg;
    const dim3 grid(nblocks), block(WAVE * wpg);
    const size_t lds = wpg * STEP_LDS_PER_WAVE;
#define LBM_SINGLE_LAUNCH(SC, RG, WL)                                                                          \
    hipLaunchKernelGGL((step_kernel<R, SC, RG, WL>), grid, block, lds, s, rv.f_in, rv.f_out, rv.coef, rv.seq, \
                       rv.cur, rv.Lx, rv.Ly, rv.plane, rv.rows, rv.nstrips, nwaves)
    LBM_DISPATCH(LBM_SINGLE_LAUNCH)
#undef LBM_SINGLE_LAUNCH
#undef LBM_DISPATCH
    return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_step(const BatchRun<R>* d_runs, const StepCoef<R>* d_coefs, const BatchItem* d_items,
                             int32_t nitems, int32_t cur, int scheme, int regularize, int wmode, int wpg,
                             hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (wmode < 0 || wmode > 2) return hipErrorInvalidValue;
    const bool pair = wpg == LBM_PAIR;
#define LBM_DISPATCH(LAUNCH)                                         \
    if (scheme == 1) {                                               \
        if (regularize) {                                            \
            if (wmode == 0) LAUNCH(1, true, 0);                      \
            else if (wmode == 1) LAUNCH(1, true, 1);                 \
            else LAUNCH(1, true, 2);                                 \
        } else {                                                     \
            if (wmode == 0) LAUNCH(1, false, 0);                     \
            else if (wmode == 1) LAUNCH(1, false, 1);                \
            else LAUNCH(1, false, 2);                                \
        }                                                            \
    } else {                                                         \
        if (regularize) {                                            \
            if (wmode == 0) LAUNCH(2, true, 0);                      \
            else if (wmode == 1) LAUNCH(2, true, 1);                 \
            else LAUNCH(2, true, 2);                                 \
        } else {                                                     \
            if (wmode == 0) LAUNCH(2, false, 0);                     \
            else if (wmode == 1) LAUNCH(2, false, 1);                \
            else LAUNCH(2, false, 2);                                \
        }                                                            \
    }
    if constexpr (sizeof(R) == 4) {
        if (pair) {
#define LBM_PAIR_LAUNCH(SC, RG, WM)                                                                          \
    hipLaunchKernelGGL((batch_pair_step_kernel<R, SC, RG, WM>), dim3(nitems), dim3(2 * WAVE), PAIR_STEP_LDS, s, \
                       d_runs, d_coefs, d_items, nitems, cur)
            LBM_DISPATCH(LBM_PAIR_LAUNCH)
#undef LBM_PAIR_LAUNCH
            return hipGetLastError();
        }
    }
    if (pair) return hipErrorInvalidValue;
    const int nblocks = (nitems + wpg - 1) / wpg;
    const dim3 grid(nblocks), block(WAVE * wpg);
    const size_t lds = wpg * STEP_LDS_PER_WAVE;
#define LBM_SINGLE_LAUNCH(SC, RG, WM) \
    hipLaunchKernelGGL((batch_step_kernel<R, SC, RG, WM>), grid, block, lds, s, d_runs, d_coefs, d_items, nitems, cur)
    LBM_DISPATCH(LBM_SINGLE_LAUNCH)
#undef LBM_SINGLE_LAUNCH
#undef LBM_DISPATCH
    return hipGetLastError();
}

// workgroups of one persistent kernel that the device holds at once
template <typename K>
int resident_groups(K kernel, int block, size_t lds)
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess) return 0;
    return per_cu * cus;
}

template <typename R>
hipError_t launch_batch_persistent(const BatchRun<R>* d_runs, int32_t nruns, const StepCoef<R>* d_coefs,
                                   const BatchItem* d_items, int32_t nitems, int32_t cur0, int32_t nsteps,
                                   int scheme, int regularize, int wmode, uint32_t* ticket, int32_t* done,
                                   uint32_t* err, uint32_t wait_limit, hipStream_t s)
{
    if constexpr (sizeof(R) != 4) {
        return hipErrorInvalidValue;
    } else {
        if (nitems <= 0 || nsteps <= 0) return hipSuccess;
        if (wmode < 0 || wmode > 2 || (int64_t)nitems * nsteps >= (int64_t)1 << 31) return hipErrorInvalidValue;
        hipLaunchKernelGGL(batch_reset_kernel, dim3(grid_for(nitems, 256)), dim3(256), 0, s, ticket, done, nitems);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t total = (int64_t)nitems * nsteps;
#define LBM_PERSIST_LAUNCH(SC, RG, WM)                                                                    \
    {                                                                                                     \
        auto* k = batch_persistent_kernel<R, SC, RG, WM>;                                                 \
        const int cap = resident_groups(k, 2 * WAVE, PAIR_STEP_LDS);                                      \
        if (cap <= 0) return hipErrorInvalidConfiguration;                                                \
        const int grid = (int)std::min<int64_t>(cap, total);                                              \
        hipLaunchKernelGGL(k, dim3(grid), dim3(2 * WAVE), PAIR_STEP_LDS, s, d_runs, d_coefs, d_items, nitems, \
                           cur0, nsteps, ticket, done, err, wait_limit);                                  \
    }
        if (scheme == 1) {
            if (regularize) {
                if (wmode == 0) LBM_PERSIST_LAUNCH(1, true, 0)
                else if (wmode == 1) LBM_PERSIST_LAUNCH(1, true, 1)
                else LBM_PERSIST_LAUNCH(1, true, 2)
            } else {
                if (wmode == 0) LBM_PERSIST_LAUNCH(1, false, 0)
                else if (wmode == 1) LBM_PERSIST_LAUNCH(1, false, 1)
                else LBM_PERSIST_LAUNCH(1, false, 2)
            }
        } else {
            if (regularize) {
                if (wmode == 0) LBM_PERSIST_LAUNCH(2, true, 0)
                else if (wmode == 1) LBM_PERSIST_LAUNCH(2, true, 1)
                else LBM_PERSIST_LAUNCH(2, true, 2)
            } else {
                if (wmode == 0) LBM_PERSIST_LAUNCH(2, false, 0)
                else if (wmode == 1) LBM_PERSIST_LAUNCH(2, false, 1)
                else LBM_PERSIST_LAUNCH(2, false, 2)
            }
        }
#undef LBM_PERSIST_LAUNCH
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((batch_seq_kernel<R>), dim3(grid_for(nruns, 64)), dim3(64), 0, s, d_runs, nruns, cur0,
                           nsteps);
        return hipGetLastError();
    }
}

template <typename R>
hipError_t launch_init(R* f, const StepCoef<R>* coef, const double* rho, const double* ux, const double* uy,
                       int64_t n, int64_t plane, hipStream_t s)
{
    hipLaunchKernelGGL((init_kernel<R>), dim3(grid_for(n, 256)), dim3(256), 0, s, f, coef, rho, ux, uy, n, plane);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fill_ghost(R* f, const StepCoef<R>* coef, int32_t Lx, int32_t Ly, int64_t plane, hipStream_t s)
{
    hipLaunchKernelGGL((fill_ghost_kernel<R>), dim3(grid_for(2 * (int64_t)Lx, 256)), dim3(256), 0, s, f, coef, Lx, Ly,
                       plane);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_moments(const R* f, const StepCoef<R>* coef, double* rho, double* ux, double* uy, int64_t n,
                          int64_t plane, hipStream_t s)
{
    hipLaunchKernelGGL((moments_kernel<R>), dim3(grid_for(n, 256)), dim3(256), 0, s, f, coef, rho, ux, uy, n, plane);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_get_plane(const R* f, const StepCoef<R>* coef, int k, double* out, int64_t n, int64_t plane,
                            hipStream_t s)
{
    hipLaunchKernelGGL((get_plane_kernel<R>), dim3(grid_for(n, 256)), dim3(256), 0, s, f, coef, k, out, n, plane);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_set_plane(R* f, const StepCoef<R>* coef, int k, const double* in, int64_t n, int64_t plane,
                            hipStream_t s)
{
    hipLaunchKernelGGL((set_plane_kernel<R>), dim3(grid_for(n, 256)), dim3(256), 0, s, f, coef, k, in, n, plane);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_reduce(const R* f, const StepCoef<R>* coef, int32_t Lx, int32_t Ly, int64_t plane,
                         double threshold, double* partials, int32_t max_blocks, double* result, hipStream_t s)
{
    int nb = grid_for((int64_t)Lx * Ly, 256);
    if (nb > max_blocks) nb = max_blocks;
    hipLaunchKernelGGL((reduce_kernel<R>), dim3(nb), dim3(256), 0, s, f, coef, Lx, Ly, plane, threshold, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(64), 0, s, partials, nb, result);
    return hipGetLastError();
}

#define LBM_INSTANTIATE(R)                                                                                   \
    template hipError_t launch_step<R>(const RunView<R>&, int, int, int, int, hipStream_t);                  \
    template hipError_t launch_batch_step<R>(const BatchRun<R>*, const StepCoef<R>*, const BatchItem*,       \
                                             int32_t, int32_t, int, int, int, int, hipStream_t);             \
    template hipError_t launch_init<R>(R*, const StepCoef<R>*, const double*, const double*, const double*, \
                                       int64_t, int64_t, hipStream_t);                                       \
    template hipError_t launch_fill_ghost<R>(R*, const StepCoef<R>*, int32_t, int32_t, int64_t, hipStream_t); \
    template hipError_t launch_moments<R>(const R*, const StepCoef<R>*, double*, double*, double*, int64_t, \
                                          int64_t, hipStream_t);                                             \
    template hipError_t launch_get_plane<R>(const R*, const StepCoef<R>*, int, double*, int64_t, int64_t,    \
                                            hipStream_t);                                                    \
    template hipError_t launch_set_plane<R>(R*, const StepCoef<R>*, int, const double*, int64_t, int64_t,    \
                                            hipStream_t);                                                    \
    template hipError_t launch_reduce<R>(const R*, const StepCoef<R>*, int32_t, int32_t, int64_t, double,    \
                                         double*, int32_t, double*, hipStream_t);                            \
    template hipError_t launch_batch_persistent<R>(const BatchRun<R>*, int32_t, const StepCoef<R>*,          \
                                                   const BatchItem*, int32_t, int32_t, int32_t, int, int, int, \
                                                   uint32_t*, int32_t*, uint32_t*, uint32_t, hipStream_t);
LBM_INSTANTIATE(float)
LBM_INSTANTIATE(double)
#undef LBM_INSTANTIATE

}  // namespace lbm
