// copy_probe.hip -- memory-side ceilings for the step kernels' access shape.
//
// Measurement only (not part of the stepper): plain copies of a 16-plane FP32
// distribution field that move the same bytes as one time step, in the same
// pattern as the step kernels or in simpler ones, so that the step's achieved
// bandwidth can be set against what its access shape allows on the part.
//
//  * strip copy: one 64-lane wavefront per strip of OUTW columns, marching a
//    chunk of rows; each lane loads its column of all 16 planes for every row
//    of the chunk plus HALO_Y rows above and below, and stores the 16 values
//    of its column for the chunk's own rows when it is one of the strip's
//    OUTW output lanes.  OUTW = 56 with 4 halo columns on each side is the
//    step's shape (strips start every 224 bytes, inside cache lines); OUTW =
//    64 without halo columns gives strips aligned to 256 bytes.  The next row
//    is loaded before the current one is stored, as in the step.  Optional
//    dynamic LDS per workgroup limits how many wavefronts a CU holds.
//  * flat copy: a grid-stride copy of the whole field in 16-byte vectors.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    constexpr int NXCD = 8;
    const int q = nblocks / NXCD, rem = nblocks % NXCD;
    const int x = b % NXCD, i = b / NXCD;
    return x * q + (x < rem ? x : rem) + i;
}

extern __shared__ char probe_lds[];

template <int OUTW, int HX>
__global__ __launch_bounds__(64) void strip_copy_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                        int Lx, int Ly, int rows, int hy, int nstrips, int nwaves,
                                                        int touch_lds)
{
    const int wave = xcd_remap(blockIdx.x, gridDim.x);
    if (wave >= nwaves) return;
    if (touch_lds) probe_lds[threadIdx.x] = 0;  // keeps the LDS allocation live
    const int lane = threadIdx.x;
    const int chunk = wave / nstrips, strip = wave - chunk * nstrips;
    int col = (strip * OUTW - HX + lane) % Lx;
    if (col < 0) col += Lx;
    const bool out_lane = lane >= HX && lane < HX + OUTW && strip * OUTW + lane - HX < Lx;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, Ly);
    const int64_t plane = (int64_t)Lx * Ly;
    auto row_of = [&](int r) {
        int rr = r % Ly;
        return rr < 0 ? rr + Ly : rr;
    };
    float v[16], n[16];
    {
        const int64_t off = (int64_t)row_of(y0 - hy) * Lx + col;
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = src[k * plane + off];
    }
    for (int r = y0 - hy; r < y1 + hy; ++r) {
        if (r + 1 < y1 + hy) {
            const int64_t off = (int64_t)row_of(r + 1) * Lx + col;
#pragma unroll
            for (int k = 0; k < 16; ++k) n[k] = src[k * plane + off];
        }
        if (r >= y0 && r < y1 && out_lane) {
            const int64_t off = (int64_t)r * Lx + col;
#pragma unroll
            for (int k = 0; k < 16; ++k) dst[k * plane + off] = v[k];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = n[k];
    }
}

// The same strip march on a strip-blocked field: columns in blocks of 56,
// layout f[block][row][k][56], so the 16 values of a strip's row are one
// contiguous 3584-byte span; lanes 0-3 and 60-63 read their halo columns from
// the neighbouring blocks (periodic over nblocks * 56 columns).
__global__ __launch_bounds__(64) void blocked_copy_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                         int nblocks, int Ly, int rows, int hy, int nwaves,
                                                         int touch_lds)
{
    const int wave = xcd_remap(blockIdx.x, gridDim.x);
    if (wave >= nwaves) return;
    if (touch_lds) probe_lds[threadIdx.x] = 0;
    const int lane = threadIdx.x;
    const int Lx = nblocks * 56;
    const int chunk = wave / nblocks, strip = wave - chunk * nblocks;
    int col = (strip * 56 - 4 + lane) % Lx;
    if (col < 0) col += Lx;
    const int blk = col / 56, pos = col - blk * 56;
    const bool out_lane = lane >= 4 && lane < 60;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, Ly);
    const int64_t row_stride = 16 * 56;
    const int64_t lane_base = (int64_t)blk * Ly * row_stride + pos;
    const int64_t out_base = (int64_t)strip * Ly * row_stride + (lane - 4);
    auto row_of = [&](int r) {
        int rr = r % Ly;
        return rr < 0 ? rr + Ly : rr;
    };
    float v[16], n[16];
    {
        const int64_t off = lane_base + (int64_t)row_of(y0 - hy) * row_stride;
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = src[off + k * 56];
    }
    for (int r = y0 - hy; r < y1 + hy; ++r) {
        if (r + 1 < y1 + hy) {
            const int64_t off = lane_base + (int64_t)row_of(r + 1) * row_stride;
#pragma unroll
            for (int k = 0; k < 16; ++k) n[k] = src[off + k * 56];
        }
        if (r >= y0 && r < y1 && out_lane) {
            const int64_t off = out_base + (int64_t)r * row_stride;
#pragma unroll
            for (int k = 0; k < 16; ++k) dst[off + k * 56] = v[k];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = n[k];
    }
}

__global__ __launch_bounds__(256) void flat_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                        int64_t n4)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

// Strip copy of a 16-plane FP32 field of Lx x Ly nodes (periodic rows and
// columns): outw = 56 (4 halo columns each side) or 64 (none), halo_y rows
// above and below each chunk of `rows` rows, lds_bytes of dynamic LDS per
// workgroup (0 = none).  Returns a hipError_t code (0 = launched).
int probe_strip_copy(const float* d_src, float* d_dst, int Lx, int Ly, int outw, int rows, int halo_y,
                     int lds_bytes, void* stream)
{
    if (!d_src || !d_dst || Lx < 64 || Ly < 1 || rows < 1 || halo_y < 0 || halo_y > Ly || lds_bytes < 0
        || lds_bytes > 65536 || (outw != 56 && outw != 64))
        return (int)hipErrorInvalidValue;
    const int nstrips = (Lx + outw - 1) / outw;
    const int nchunks = (Ly + rows - 1) / rows;
    const int nwaves = nstrips * nchunks;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (outw == 56)
        hipLaunchKernelGGL((strip_copy_kernel<56, 4>), dim3(nwaves), dim3(64), lds_bytes, s, d_src, d_dst, Lx, Ly,
                           rows, halo_y, nstrips, nwaves, lds_bytes > 0 ? 1 : 0);
    else
        hipLaunchKernelGGL((strip_copy_kernel<64, 0>), dim3(nwaves), dim3(64), lds_bytes, s, d_src, d_dst, Lx, Ly,
                           rows, halo_y, nstrips, nwaves, lds_bytes > 0 ? 1 : 0);
    return (int)hipGetLastError();
}

// Strip copy of a strip-blocked 16-plane FP32 field of nblocks * 56 x Ly
// nodes (layout f[block][row][k][56]), same march and options as
// probe_strip_copy with 56 output columns.
int probe_blocked_copy(const float* d_src, float* d_dst, int nblocks, int Ly, int rows, int halo_y, int lds_bytes,
                       void* stream)
{
    if (!d_src || !d_dst || nblocks < 2 || Ly < 1 || rows < 1 || halo_y < 0 || halo_y > Ly || lds_bytes < 0
        || lds_bytes > 65536)
        return (int)hipErrorInvalidValue;
    const int nchunks = (Ly + rows - 1) / rows;
    const int nwaves = nblocks * nchunks;
    hipLaunchKernelGGL(blocked_copy_kernel, dim3(nwaves), dim3(64), lds_bytes, static_cast<hipStream_t>(stream),
                       d_src, d_dst, nblocks, Ly, rows, halo_y, nwaves, lds_bytes > 0 ? 1 : 0);
    return (int)hipGetLastError();
}

// Grid-stride copy of n_floats (a multiple of 4) in 16-byte vectors.
int probe_flat_copy(const float* d_src, float* d_dst, int64_t n_floats, void* stream)
{
    if (!d_src || !d_dst || n_floats < 4 || (n_floats & 3)) return (int)hipErrorInvalidValue;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(flat_copy_kernel, dim3(4096), dim3(256), 0, s, reinterpret_cast<const float4*>(d_src),
                       reinterpret_cast<float4*>(d_dst), n_floats / 4);
    return (int)hipGetLastError();
}

}  // extern "C"
