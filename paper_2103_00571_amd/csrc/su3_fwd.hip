// su3_fwd.hip -- forward SU(3) link multiply c[s][j] = a[s][j] * b[j] on
// gfx950 (SU3_Bench core kernel: arXiv 2103.00571, Background / SU3_Bench).
//
// The product is HBM-bound (0.75 flop per byte in FP64), so the kernels are
// built around the memory stream, not the arithmetic:
//
//  * Site-major (AoS) forms: each thread owns a fixed "unit" position inside
//    a site -- the smallest run of output rows whose input and output bytes
//    are whole 16-byte chunks (FP64: 1 row, 48 B in / 48 B out; FP32: 2 rows;
//    BF16: 4 rows; reconstruct-12: 2 links, 96 B in / 144 B out). Global
//    memory is moved in whole-wavefront 1 KiB runs and transposed to one unit
//    per lane through LDS (see fwd_aos).
//  * The grid is persistent (every workgroup resident, a multiple of 3) and
//    grid-strides over tiles. The stride is a whole number of sites, so a
//    thread meets the same link index j on every tile and keeps the b[j]
//    entries it needs in registers, loaded once (on Xeon the paper keeps a
//    local transposed copy of B; here the copy is registers).
//  * a and c are streamed with nontemporal 16-byte loads and stores.
//  * 64-bit offsets throughout (a FP64 L=48 lattice is 3.06e9 bytes).
#include "su3_internal.hpp"

#ifndef SU3_UNROLL
#define SU3_UNROLL 2
#endif

namespace su3 {

// ------------------------------------------------------------ AoS forms
// Each form describes one "unit" (kIn 16-byte chunks in, kOut chunks out,
// kUnitsPerSite units per site), the b coefficients a thread at unit
// position `pos` of a site needs, and the arithmetic of one unit.

// three complex inputs x[0..5] (interleaved) times a 3x3 link -> one row
template <typename S>
__device__ __forceinline__ void row_times(const S *x, const S (&mr)[9], const S (&mi)[9], S *o)
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        S re = 0, im = 0;
#pragma unroll
        for (int m = 0; m < 3; ++m)
            cmac(re, im, x[2 * m], x[2 * m + 1], mr[3 * m + l], mi[3 * m + l]);
        o[2 * l] = re;
        o[2 * l + 1] = im;
    }
}

template <typename S>
struct Link {
    S r[9], i[9];
};

template <typename S>
__device__ __forceinline__ void load_link(const S *__restrict__ b, int j, Link<S> &m)
{
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        m.r[q] = b[2 * (9 * j + q)];
        m.i[q] = b[2 * (9 * j + q) + 1];
    }
}

template <int N, typename S>
__device__ __forceinline__ void unpack_chunks(const u4 (&v)[N], S *x)
{
    constexpr int P = 16 / sizeof(S);
#pragma unroll
    for (int t = 0; t < N; ++t) {
        typedef S SV __attribute__((ext_vector_type(P)));
        const SV w = __builtin_bit_cast(SV, v[t]);
#pragma unroll
        for (int h = 0; h < P; ++h)
            x[P * t + h] = w[h];
    }
}

template <int N, typename S>
__device__ __forceinline__ void pack_chunks(const S *x, u4 (&v)[N])
{
    constexpr int P = 16 / sizeof(S);
#pragma unroll
    for (int t = 0; t < N; ++t) {
        typedef S SV __attribute__((ext_vector_type(P)));
        SV w;
#pragma unroll
        for (int h = 0; h < P; ++h)
            w[h] = x[P * t + h];
        v[t] = __builtin_bit_cast(u4, w);
    }
}

// FP64: unit = output row k of link j (pos = 3j + k); 48 B in, 48 B out.
struct FormF64 {
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 12;
    typedef double B;
    typedef Link<double> Coef;
    __device__ static void load(const B *b, int pos, Coef &m) { load_link(b, pos / 3, m); }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &m, u4 (&o)[kOut])
    {
        double x[6], y[6];
        unpack_chunks<3>(v, x);
        row_times(x, m.r, m.i, y);
        pack_chunks<3>(y, o);
    }
};

// FP32: unit = rows 2w and 2w+1 of a site (w = 0..5), which may belong to two
// links; 48 B in, 48 B out.
struct FormF32 {
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 6;
    typedef float B;
    struct Coef {
        Link<float> m[2];
    };
    __device__ static void load(const B *b, int pos, Coef &c)
    {
        load_link(b, (2 * pos) / 3, c.m[0]);
        load_link(b, (2 * pos + 1) / 3, c.m[1]);
    }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &c, u4 (&o)[kOut])
    {
        float x[12], y[12];
        unpack_chunks<3>(v, x);
        row_times(x, c.m[0].r, c.m[0].i, y);
        row_times(x + 6, c.m[1].r, c.m[1].i, y + 6);
        pack_chunks<3>(y, o);
    }
};

// BF16 storage, FP32 arithmetic: unit = rows 4w .. 4w+3 (w = 0..2); row i
// uses link (4w + i) / 3; 48 B in, 48 B out, rounded to nearest even.
struct FormBF16 {
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 3;
    typedef float B;
    struct Coef {
        Link<float> m[4];
    };
    __device__ static void load(const B *b, int pos, Coef &c)
    {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            load_link(b, (4 * pos + i) / 3, c.m[i]);
    }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &c, u4 (&o)[kOut])
    {
        uint32_t w[12];
        unpack_chunks<3>(v, w);
        float x[24], y[24];
#pragma unroll
        for (int h = 0; h < 12; ++h) {
            x[2 * h] = bf16_lo(w[h]);
            x[2 * h + 1] = bf16_hi(w[h]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            row_times(x + 6 * i, c.m[i].r, c.m[i].i, y + 6 * i);
#pragma unroll
        for (int h = 0; h < 12; ++h)
            w[h] = pack_bf16x2(y[2 * h], y[2 * h + 1]);
        pack_chunks<3>(w, o);
    }
};

// Third row of a link in SU(3) from its first two: conj(row0 x row1), FP32.
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

// Reconstruct-12: unit = links 2w, 2w+1 (w = 0, 1); rows 0-1 of each in FP32
// (96 B in), the full FP32 products out (144 B).
struct FormR12 {
    static constexpr int kIn = 6, kOut = 9, kUnitsPerSite = 2;
    typedef float B;
    struct Coef {
        Link<float> m[2];
    };
    __device__ static void load(const B *b, int pos, Coef &c)
    {
        load_link(b, 2 * pos, c.m[0]);
        load_link(b, 2 * pos + 1, c.m[1]);
    }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &c, u4 (&o)[kOut])
    {
        float x[24], y[36];
        unpack_chunks<6>(v, x);   // link h: rows 0-1 at x[12h .. 12h+11]
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float a[18];
#pragma unroll
            for (int q = 0; q < 12; ++q)
                a[q] = x[12 * h + q];
            recon_row2_f32(a, a + 6, a + 12);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                row_times(a + 6 * k, c.m[h].r, c.m[h].i, y + 18 * h + 6 * k);
        }
        pack_chunks<9>(y, o);
    }
};

// Order LDS traffic between the lanes of one wavefront (LDS operations of a
// wavefront execute in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Site-major forward for form F. A wavefront works on tiles of 64
// consecutive units: its global loads and stores are whole 1 KiB runs (lane l
// moves chunk i*64 + l of the tile), and a private LDS slice transposes
// between that order and one unit per lane (lane l reads chunks
// l*kIn .. l*kIn+kIn-1). No workgroup barrier is needed: each wavefront only
// touches its own slice. kUnroll tiles are loaded before the first is
// processed, to keep more bytes in flight.
//
// The tile stride (all wavefronts x 64 units) is a multiple of kUnitsPerSite
// because the grid is a multiple of 3 workgroups of 256 threads, so lane l of
// a wavefront sees the same unit position -- and the same b links -- on every
// tile: its b coefficients are loaded once into registers.
template <class F, int kUnroll>
__global__ __launch_bounds__(kBlock) void fwd_aos(const u4 *__restrict__ a, const typename F::B *__restrict__ b,
                                                  u4 *__restrict__ c, int64_t units)
{
    constexpr int kWaves = kBlock / 64;
    constexpr int kSlots = 64 * (F::kIn > F::kOut ? F::kIn : F::kOut);
    __shared__ u4 stage[kWaves][kSlots];
    const int lane = threadIdx.x & 63;
    u4 *my = stage[threadIdx.x >> 6];
    const int64_t wave0 = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    typename F::Coef coef;
    F::load(b, (int)((wave0 * 64 + lane) % F::kUnitsPerSite), coef);
    const int64_t nin = units * F::kIn, nout = units * F::kOut;

    for (int64_t t0 = wave0; t0 * 64 < units; t0 += kUnroll * nwaves) {
        // all kUnroll tiles whole: no per-chunk bounds checks (wave-uniform)
        const bool whole = (t0 + (kUnroll - 1) * nwaves + 1) * 64 <= units;
        u4 v[kUnroll][F::kIn];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t base = (t0 + u * nwaves) * 64 * F::kIn + lane;
#pragma unroll
            for (int i = 0; i < F::kIn; ++i) {
                const int64_t g = base + 64 * i;
                v[u][i] = (whole || g < nin) ? ld_stream(a + g) : u4{0, 0, 0, 0};
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t t = t0 + u * nwaves;
            if (t * 64 >= units)
                break;
#pragma unroll
            for (int i = 0; i < F::kIn; ++i)
                my[64 * i + lane] = v[u][i];
            wave_sync();
            u4 x[F::kIn], o[F::kOut];
#pragma unroll
            for (int i = 0; i < F::kIn; ++i)
                x[i] = my[F::kIn * lane + i];
            F::apply(x, coef, o);
            wave_sync();
#pragma unroll
            for (int i = 0; i < F::kOut; ++i)
                my[F::kOut * lane + i] = o[i];
            wave_sync();
            const int64_t base = t * 64 * F::kOut + lane;
#pragma unroll
            for (int i = 0; i < F::kOut; ++i) {
                const int64_t g = base + 64 * i;
                if (whole || g < nout)
                    st_stream(c + g, my[64 * i + lane]);
            }
            wave_sync();
        }
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
    case 0: return occupancy(reinterpret_cast<const void *>(fwd_aos<FormF64, SU3_UNROLL>), c64);
    case 1: return occupancy(reinterpret_cast<const void *>(fwd_aos<FormF32, SU3_UNROLL>), c32);
    case 2: return occupancy(reinterpret_cast<const void *>(fwd_aos<FormBF16, SU3_UNROLL>), c16);
    default: return occupancy(reinterpret_cast<const void *>(fwd_aos<FormR12, SU3_UNROLL>), c12);
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
    return launch_k(fwd_aos<FormF64, SU3_UNROLL>, dim3((unsigned)grid), dim3(kBlock), s, (const u4 *)a,
                    (const double *)b, (u4 *)c, sites * FormF64::kUnitsPerSite);
}

hipError_t launch_fwd_aos_f32(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos<FormF32, SU3_UNROLL>, dim3((unsigned)grid), dim3(kBlock), s, (const u4 *)a,
                    (const float *)b, (u4 *)c, sites * FormF32::kUnitsPerSite);
}

hipError_t launch_fwd_aos_bf16(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos<FormBF16, SU3_UNROLL>, dim3((unsigned)grid), dim3(kBlock), s, (const u4 *)a,
                    (const float *)b, (u4 *)c, sites * FormBF16::kUnitsPerSite);
}

hipError_t launch_fwd_aos_r12(const void *a, const void *b, void *c, int64_t sites, int64_t grid, hipStream_t s)
{
    return launch_k(fwd_aos<FormR12, SU3_UNROLL>, dim3((unsigned)grid), dim3(kBlock), s, (const u4 *)a,
                    (const float *)b, (u4 *)c, sites * FormR12::kUnitsPerSite);
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
