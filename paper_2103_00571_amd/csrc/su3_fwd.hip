// su3_fwd.hip -- forward SU(3) link multiply c[s][j] = a[s][j] * b[j] on
// gfx950 (SU3_Bench core kernel: arXiv 2103.00571, Background / SU3_Bench).
//
// The product is HBM-bound (0.75 flop per byte in FP64), so the kernels are
// built around the memory stream, not the arithmetic:
//
//  * Each thread owns a fixed "unit" position inside a site: the unit is the
//    smallest run of output rows whose input and output bytes are whole,
//    16-byte aligned multiples of 16 B (FP64: 1 row = 48 B in / 48 B out;
//    FP32: 2 rows; BF16: 4 rows; reconstruct-12: 2 links = 96 B in / 144 B
//    out). A wavefront therefore streams one contiguous span of memory with
//    global_load/store_dwordx4, and every fetched cache line is used whole.
//  * The grid is persistent (a multiple of 3 workgroups, a few per CU) and
//    grid-strides over units. Because the step is a multiple of the number
//    of units per site, a thread meets the same link index j on every
//    iteration, so the b[j] entries it needs are loaded into registers once
//    (the paper's "local transposed copy of B" on Xeon becomes registers).
//  * Two units per iteration are loaded before either is stored, to keep
//    more bytes in flight per wave.
//  * Loads and stores of a and c are nontemporal (streamed once).
//  * 64-bit offsets throughout (a FP64 L=48 lattice is 3.06e9 bytes).
#include "su3_internal.hpp"

#ifndef SU3_UNROLL
#define SU3_UNROLL 2
#endif

namespace su3 {

// ---------------------------------------------------------------- FP64 AoS
// unit = one output row (j, k) of one site: 3 complex doubles in and out.
struct RowF64 {
    d2 x[3];
};

__device__ __forceinline__ void row_f64(const d2 *__restrict__ src, RowF64 &r)
{
#pragma unroll
    for (int m = 0; m < 3; ++m)
        r.x[m] = ld_stream(src + m);
}

__device__ __forceinline__ void row_f64_out(const RowF64 &r, const double (&br)[9], const double (&bi)[9],
                                            d2 *__restrict__ dst)
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m)
            cmac(re, im, r.x[m].x, r.x[m].y, br[3 * m + l], bi[3 * m + l]);
        d2 o = {re, im};
        st_stream(dst + l, o);
    }
}

__global__ __launch_bounds__(kBlock) void fwd_aos_f64(const d2 *__restrict__ a, const double *__restrict__ b,
                                                      d2 *__restrict__ c, int64_t rows)
{
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    const int j = (int)((first % 12) / 3);
    double br[9], bi[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        br[q] = b[2 * (9 * j + q)];
        bi[q] = b[2 * (9 * j + q) + 1];
    }
    int64_t r = first;
#if SU3_UNROLL >= 2
    for (; r + step < rows; r += 2 * step) {
        RowF64 u0, u1;
        row_f64(a + 3 * r, u0);
        row_f64(a + 3 * (r + step), u1);
        row_f64_out(u0, br, bi, c + 3 * r);
        row_f64_out(u1, br, bi, c + 3 * (r + step));
    }
#endif
    for (; r < rows; r += step) {
        RowF64 u0;
        row_f64(a + 3 * r, u0);
        row_f64_out(u0, br, bi, c + 3 * r);
    }
}

// ---------------------------------------------------------------- FP32 AoS
// unit = two consecutive output rows q0 = 2w, q0 + 1 of a site (w = 0..5),
// 6 complex floats = 48 B = 3 x 16 B in and out. The rows may belong to two
// different links (q / 3), so two b matrices are kept.
struct BF32 {
    float r[9], i[9];
};

__device__ __forceinline__ void load_b_f32(const float *__restrict__ b, int j, BF32 &m)
{
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        m.r[q] = b[2 * (9 * j + q)];
        m.i[q] = b[2 * (9 * j + q) + 1];
    }
}

// one output row from three complex inputs (interleaved re/im in x[0..5])
__device__ __forceinline__ void row_f32(const float *x, const BF32 &m, float *o)
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        float re = 0.0f, im = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            cmac(re, im, x[2 * k], x[2 * k + 1], m.r[3 * k + l], m.i[3 * k + l]);
        o[2 * l] = re;
        o[2 * l + 1] = im;
    }
}

__device__ __forceinline__ void unit_f32(f4 *__restrict__ dst, const f4 (&v)[3], const BF32 &m0, const BF32 &m1)
{
    float x[12], o[12];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        x[4 * t] = v[t].x;
        x[4 * t + 1] = v[t].y;
        x[4 * t + 2] = v[t].z;
        x[4 * t + 3] = v[t].w;
    }
    row_f32(x, m0, o);
    row_f32(x + 6, m1, o + 6);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        f4 w = {o[4 * t], o[4 * t + 1], o[4 * t + 2], o[4 * t + 3]};
        st_stream(dst + t, w);
    }
}

__global__ __launch_bounds__(kBlock) void fwd_aos_f32(const f4 *__restrict__ a, const float *__restrict__ b,
                                                      f4 *__restrict__ c, int64_t units)
{
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    const int w = (int)(first % 6);
    BF32 m0, m1;
    load_b_f32(b, (2 * w) / 3, m0);
    load_b_f32(b, (2 * w + 1) / 3, m1);
    int64_t u = first;
#if SU3_UNROLL >= 2
    for (; u + step < units; u += 2 * step) {
        f4 v0[3], v1[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            v0[t] = ld_stream(a + 3 * u + t);
            v1[t] = ld_stream(a + 3 * (u + step) + t);
        }
        unit_f32(c + 3 * u, v0, m0, m1);
        unit_f32(c + 3 * (u + step), v1, m0, m1);
    }
#endif
    for (; u < units; u += step) {
        f4 v0[3];
#pragma unroll
        for (int t = 0; t < 3; ++t)
            v0[t] = ld_stream(a + 3 * u + t);
        unit_f32(c + 3 * u, v0, m0, m1);
    }
}

// ---------------------------------------------------------------- BF16 AoS
// unit = four consecutive output rows q = 4w .. 4w+3 (w = 0..2), 12 complex
// bf16 = 48 B in and out. Row i uses b[(4w + i) / 3]; each row keeps its own
// copy of the b entries it needs (selected once, outside the loop).
__device__ __forceinline__ void unit_bf16(u4 *__restrict__ dst, const u4 (&v)[3], const BF32 (&m)[4])
{
    float x[24], o[24];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const uint32_t wv[4] = {v[t].x, v[t].y, v[t].z, v[t].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            x[8 * t + 2 * h] = bf16_lo(wv[h]);
            x[8 * t + 2 * h + 1] = bf16_hi(wv[h]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        row_f32(x + 6 * i, m[i], o + 6 * i);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        u4 w = {pack_bf16x2(o[8 * t], o[8 * t + 1]), pack_bf16x2(o[8 * t + 2], o[8 * t + 3]),
                pack_bf16x2(o[8 * t + 4], o[8 * t + 5]), pack_bf16x2(o[8 * t + 6], o[8 * t + 7])};
        st_stream(dst + t, w);
    }
}

__global__ __launch_bounds__(kBlock) void fwd_aos_bf16(const u4 *__restrict__ a, const float *__restrict__ b,
                                                       u4 *__restrict__ c, int64_t units)
{
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    const int w = (int)(first % 3);
    BF32 m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        load_b_f32(b, (4 * w + i) / 3, m[i]);
    int64_t u = first;
#if SU3_UNROLL >= 2
    for (; u + step < units; u += 2 * step) {
        u4 v0[3], v1[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            v0[t] = ld_stream(a + 3 * u + t);
            v1[t] = ld_stream(a + 3 * (u + step) + t);
        }
        unit_bf16(c + 3 * u, v0, m);
        unit_bf16(c + 3 * (u + step), v1, m);
    }
#endif
    for (; u < units; u += step) {
        u4 v0[3];
#pragma unroll
        for (int t = 0; t < 3; ++t)
            v0[t] = ld_stream(a + 3 * u + t);
        unit_bf16(c + 3 * u, v0, m);
    }
}

// ----------------------------------------------------- reconstruct-12 AoS
// unit = two links 2w, 2w+1 (w = 0, 1) of a site: rows 0-1 of each link in
// FP32 (2 x 48 B = 6 x 16 B in), full 3x3 FP32 products out (2 x 72 B =
// 9 x 16 B). Row 2 of each a link is rebuilt as conj(row0 x row1).
__device__ __forceinline__ void recon_row2_f32(const float *r0, const float *r1, float *r2)
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int p = (l + 1) % 3, q = (l + 2) % 3;
        // (r0 x r1)_l = r0_p r1_q - r0_q r1_p, then conjugate
        float xr = r0[2 * p] * r1[2 * q];
        xr = __builtin_fmaf(-r0[2 * p + 1], r1[2 * q + 1], xr);
        xr = __builtin_fmaf(-r0[2 * q], r1[2 * p], xr);
        xr = __builtin_fmaf(r0[2 * q + 1], r1[2 * p + 1], xr);
        float xi = r0[2 * p] * r1[2 * q + 1];
        xi = __builtin_fmaf(r0[2 * p + 1], r1[2 * q], xi);
        xi = __builtin_fmaf(-r0[2 * q], r1[2 * p + 1], xi);
        xi = __builtin_fmaf(-r0[2 * q + 1], r1[2 * p], xi);
        r2[2 * l] = xr;
        r2[2 * l + 1] = -xi;
    }
}

__device__ __forceinline__ void unit_r12(f4 *__restrict__ dst, const f4 (&v)[6], const BF32 &m0, const BF32 &m1)
{
    float x[2][18], o[36];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            x[h][4 * t] = v[3 * h + t].x;
            x[h][4 * t + 1] = v[3 * h + t].y;
            x[h][4 * t + 2] = v[3 * h + t].z;
            x[h][4 * t + 3] = v[3 * h + t].w;
        }
        recon_row2_f32(x[h], x[h] + 6, x[h] + 12);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        row_f32(x[0] + 6 * k, m0, o + 6 * k);
        row_f32(x[1] + 6 * k, m1, o + 18 + 6 * k);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        f4 w = {o[4 * t], o[4 * t + 1], o[4 * t + 2], o[4 * t + 3]};
        st_stream(dst + t, w);
    }
}

__global__ __launch_bounds__(kBlock) void fwd_aos_r12(const f4 *__restrict__ a, const float *__restrict__ b,
                                                      f4 *__restrict__ c, int64_t units)
{
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    const int w = (int)(first % 2);
    BF32 m0, m1;
    load_b_f32(b, 2 * w, m0);
    load_b_f32(b, 2 * w + 1, m1);
    int64_t u = first;
#if SU3_UNROLL >= 2
    for (; u + step < units; u += 2 * step) {
        f4 v0[6], v1[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            v0[t] = ld_stream(a + 6 * u + t);
            v1[t] = ld_stream(a + 6 * (u + step) + t);
        }
        unit_r12(c + 9 * u, v0, m0, m1);
        unit_r12(c + 9 * (u + step), v1, m0, m1);
    }
#endif
    for (; u < units; u += step) {
        f4 v0[6];
#pragma unroll
        for (int t = 0; t < 6; ++t)
            v0[t] = ld_stream(a + 6 * u + t);
        unit_r12(c + 9 * u, v0, m0, m1);
    }
}

// ---------------------------------------------------------------- SoA
// Thread per (site, link): blockIdx.y is the link j, so b[j] is uniform over
// the workgroup and lives in scalar registers; each of the 9 plane loads and
// stores of a wavefront is one contiguous 1 KiB (FP64) or 512 B (FP32) run.
template <typename V, typename S>
__global__ __launch_bounds__(kBlock) void fwd_soa(const V *__restrict__ a, const S *__restrict__ b,
                                                  V *__restrict__ c, int64_t n)
{
    const int j = blockIdx.y;
    S br[9], bi[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        br[q] = b[2 * (9 * j + q)];
        bi[q] = b[2 * (9 * j + q) + 1];
    }
    const V *__restrict__ ap = a + (int64_t)(9 * j) * n;
    V *__restrict__ cp = c + (int64_t)(9 * j) * n;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += step) {
        V x[9];
#pragma unroll
        for (int q = 0; q < 9; ++q)
            x[q] = ld_stream(ap + q * n + s);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                S re = 0, im = 0;
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    cmac(re, im, x[3 * k + m].x, x[3 * k + m].y, br[3 * m + l], bi[3 * m + l]);
                V o = {re, im};
                st_stream(cp + (3 * k + l) * n + s, o);
            }
    }
}

// ---------------------------------------------------------------- launchers
// Workgroups of a forward kernel that fit on one CU at once (registers and
// LDS permitting), from the runtime's occupancy calculator; cached per device.
static int occupancy(const void *kernel, std::atomic<int> (&cache)[kMaxDevices])
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return -1;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0)
        return n;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kBlock, 0) != hipSuccess || n <= 0)
        return -1;
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

int fwd_resident_blocks(int precision)
{
    static std::atomic<int> c64[kMaxDevices], c32[kMaxDevices], c16[kMaxDevices], c12[kMaxDevices];
    switch (precision) {
    case 0: return occupancy(reinterpret_cast<const void *>(fwd_aos_f64), c64);
    case 1: return occupancy(reinterpret_cast<const void *>(fwd_aos_f32), c32);
    case 2: return occupancy(reinterpret_cast<const void *>(fwd_aos_bf16), c16);
    default: return occupancy(reinterpret_cast<const void *>(fwd_aos_r12), c12);
    }
}

int soa_resident_blocks(int elem_bytes)
{
    static std::atomic<int> c64[kMaxDevices], c32[kMaxDevices];
    if (elem_bytes == 16)
        return occupancy(reinterpret_cast<const void *>(fwd_soa<d2, double>), c64);
    return occupancy(reinterpret_cast<const void *>(fwd_soa<f2, float>), c32);
}

hipError_t launch_fwd_aos_f64(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos_f64, dim3((unsigned)grid), dim3(kBlock), s, (const d2 *)a, (const double *)b, (d2 *)c,
                    sites * 12);
}

hipError_t launch_fwd_aos_f32(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos_f32, dim3((unsigned)grid), dim3(kBlock), s, (const f4 *)a, (const float *)b, (f4 *)c,
                    sites * 6);
}

hipError_t launch_fwd_aos_bf16(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos_bf16, dim3((unsigned)grid), dim3(kBlock), s, (const u4 *)a, (const float *)b, (u4 *)c,
                    sites * 3);
}

hipError_t launch_fwd_aos_r12(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos_r12, dim3((unsigned)grid), dim3(kBlock), s, (const f4 *)a, (const float *)b, (f4 *)c,
                    sites * 2);
}

hipError_t launch_fwd_soa(const void *a, const void *b, void *c, int64_t sites, int elem_bytes, int64_t grid,
                          hipStream_t s)
{
    if (elem_bytes == 16)
        return launch_k(fwd_soa<d2, double>, dim3((unsigned)grid, 4), dim3(kBlock), s, (const d2 *)a,
                        (const double *)b, (d2 *)c, sites);
    return launch_k(fwd_soa<f2, float>, dim3((unsigned)grid, 4), dim3(kBlock), s, (const f2 *)a, (const float *)b,
                    (f2 *)c, sites);
}

} // namespace su3
