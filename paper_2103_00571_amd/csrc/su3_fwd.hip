// su3_fwd.hip -- forward SU(3) link multiply c[s][j] = a[s][j] * b[j] on
// gfx950 (SU3_Bench core kernel: arXiv 2103.00571, Background / SU3_Bench).
//
// The product is HBM-bound (0.75 flop per byte in FP64), so the kernels are
// built around the memory stream, not the arithmetic:
//
//  * Site-major (AoS) forms: a thread owns one "unit" -- the smallest run of
//    output rows whose input and output bytes are whole 16-byte chunks (FP64:
//    1 row, 48 B in / 48 B out; FP32: 2 rows; BF16: 4 rows; reconstruct-12:
//    2 links, 96 B in / 144 B out). Global memory moves in whole-wavefront
//    1 KiB runs and is transposed to one unit per lane through LDS (fwd_aos).
//  * Structure-of-arrays: a thread owns one (site, output row); every plane
//    access of a wavefront is already one contiguous run, and the row is
//    uniform over a workgroup, so b[j] sits in scalar registers (fwd_soa).
//  * The grid covers the lattice once: each wavefront streams one tile and
//    exits. In the site-major kernels each XCD takes one contiguous eighth of
//    the tiles (xcd_tile); the SoA kernel picks its order (soa_xcd) and, in
//    how many phases its plane loads take (soa_waits) from the plane
//    stride, and takes any plane pitch >= the site count (soa_pitch gives
//    the one that keeps the planes from colliding in HBM).
//  * a and c are streamed with nontemporal 16-byte loads and stores.
//  * 64-bit offsets throughout (a FP64 L=48 lattice is 3.06e9 bytes).
#include "su3_internal.hpp"

// Threads per workgroup of the AoS kernels (a multiple of 64); each
// wavefront of the workgroup handles its own tile.
#ifndef SU3_AOS_BLOCK
#define SU3_AOS_BLOCK 64
#endif

// Resident wavefronts per CU, per kernel. Fewer resident wavefronts mean
// fewer bytes in flight; on MI355X the streaming rate of these kernels peaks
// with about 36-39 KiB of loads in flight per CU (12-13 wavefronts of 3 KiB,
// in the XCD-contiguous tile order) and falls steeply below about 9. Values
// from a sweep at L=48; 0 leaves occupancy to the hardware.
#ifndef SU3_WAVES_F64
#define SU3_WAVES_F64 12
#endif
#ifndef SU3_WAVES_F32
#define SU3_WAVES_F32 13
#endif
#ifndef SU3_WAVES_BF16
#define SU3_WAVES_BF16 14
#endif
#ifndef SU3_WAVES_R12
#define SU3_WAVES_R12 6
#endif
// (R12C: 3 KiB of loads per wavefront, like FP64; R12F64: 6 KiB; AN: 9 KiB.)
#ifndef SU3_WAVES_R12C
#define SU3_WAVES_R12C 13
#endif
#ifndef SU3_WAVES_R12F64
#define SU3_WAVES_R12F64 6
#endif
#ifndef SU3_WAVES_AN
#define SU3_WAVES_AN 6
#endif
#ifndef SU3_WAVES_SOA_F64
#define SU3_WAVES_SOA_F64 8
#endif
#ifndef SU3_WAVES_SOA_F32
#define SU3_WAVES_SOA_F32 0
#endif
// FP64 SoA with its plane loads in two phases (soa_waits)
#ifndef SU3_WAVES_SOA_F64_PHASED
#define SU3_WAVES_SOA_F64_PHASED 16
#endif

namespace su3 {

constexpr int kAosBlock = SU3_AOS_BLOCK;
// Threads per workgroup of fwd_soa: 128 measured 3% faster than 256 for FP64
// (with 8 resident wavefronts per CU) and equal for FP32.
#ifndef SU3_SOA_BLOCK
#define SU3_SOA_BLOCK 128
#endif
constexpr int kSoaBlock = SU3_SOA_BLOCK;

int aos_block_threads() { return kAosBlock; }

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
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 12, kWavesPerCU = SU3_WAVES_F64;
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
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 6, kWavesPerCU = SU3_WAVES_F32;
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
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 3, kWavesPerCU = SU3_WAVES_BF16;
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
    static constexpr int kIn = 6, kOut = 9, kUnitsPerSite = 2, kWavesPerCU = SU3_WAVES_R12;
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

// Reconstruct-12 in and out (FP32): unit = one link, rows 0-1 in (48 B)
// and rows 0-1 of the product out (48 B). Rows 0-1 of a*b depend only on
// rows 0-1 of a, so no row is rebuilt.
struct FormR12C {
    static constexpr int kIn = 3, kOut = 3, kUnitsPerSite = 4, kWavesPerCU = SU3_WAVES_R12C;
    typedef float B;
    typedef Link<float> Coef;
    __device__ static void load(const B *b, int pos, Coef &m) { load_link(b, pos, m); }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &m, u4 (&o)[kOut])
    {
        float x[12], y[12];
        unpack_chunks<3>(v, x);
        row_times(x, m.r, m.i, y);
        row_times(x + 6, m.r, m.i, y + 6);
        pack_chunks<3>(y, o);
    }
};

// Third row of a link in SU(3) from its first two, FP64.
__device__ __forceinline__ void recon_row2_f64(const double *r0, const double *r1, double *r2)
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int p = (l + 1) % 3, q = (l + 2) % 3;
        double xr = r0[2 * p] * r1[2 * q];
        xr = __builtin_fma(-r0[2 * p + 1], r1[2 * q + 1], xr);
        xr = __builtin_fma(-r0[2 * q], r1[2 * p], xr);
        xr = __builtin_fma(r0[2 * q + 1], r1[2 * p + 1], xr);
        double xi = r0[2 * p] * r1[2 * q + 1];
        xi = __builtin_fma(r0[2 * p + 1], r1[2 * q], xi);
        xi = __builtin_fma(-r0[2 * q], r1[2 * p + 1], xi);
        xi = __builtin_fma(-r0[2 * q + 1], r1[2 * p], xi);
        r2[2 * l] = xr;
        r2[2 * l + 1] = -xi;
    }
}

// Reconstruct-12 in FP64: unit = one link, rows 0-1 in FP64 (96 B), the full
// FP64 product out (144 B).
struct FormR12F64 {
    static constexpr int kIn = 6, kOut = 9, kUnitsPerSite = 4, kWavesPerCU = SU3_WAVES_R12F64;
    typedef double B;
    typedef Link<double> Coef;
    __device__ static void load(const B *b, int pos, Coef &m) { load_link(b, pos, m); }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &m, u4 (&o)[kOut])
    {
        double x[18], y[18];
        unpack_chunks<6>(v, x);
        recon_row2_f64(x, x + 6, x + 12);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            row_times(x + 6 * k, m.r, m.i, y + 6 * k);
        pack_chunks<9>(y, o);
    }
};

// c = a^H b for one link held as 9 complex values x (row-major):
// c(k, l) = sum_m conj(a(m, k)) b(m, l).
template <typename S>
__device__ __forceinline__ void link_an(const S *x, const Link<S> &m, S *y)
{
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            S re = 0, im = 0;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                cmac(re, im, x[2 * (3 * q + k)], -x[2 * (3 * q + k) + 1], m.r[3 * q + l], m.i[3 * q + l]);
            y[2 * (3 * k + l)] = re;
            y[2 * (3 * k + l) + 1] = im;
        }
}

// a^H b, FP64: unit = one link (the whole link is needed for its columns),
// 144 B in and out.
struct FormAnF64 {
    static constexpr int kIn = 9, kOut = 9, kUnitsPerSite = 4, kWavesPerCU = SU3_WAVES_AN;
    typedef double B;
    typedef Link<double> Coef;
    __device__ static void load(const B *b, int pos, Coef &m) { load_link(b, pos, m); }
    __device__ static void apply(const u4 (&v)[kIn], const Coef &m, u4 (&o)[kOut])
    {
        double x[18], y[18];
        unpack_chunks<9>(v, x);
        link_an(x, m, y);
        pack_chunks<9>(y, o);
    }
};

// a^H b, FP32: unit = links 2w, 2w+1 (144 B in and out).
struct FormAnF32 {
    static constexpr int kIn = 9, kOut = 9, kUnitsPerSite = 2, kWavesPerCU = SU3_WAVES_AN;
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
        float x[36], y[36];
        unpack_chunks<9>(v, x);
        link_an(x, c.m[0], y);
        link_an(x + 18, c.m[1], y + 18);
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

// Site-major forward for form F. One wavefront handles one tile of 64
// consecutive units and exits: its global loads and stores are whole 1 KiB
// runs (lane l moves chunk i*64 + l of the tile), and a private LDS slice
// transposes between that order and one unit per lane (lane l reads chunks
// l*kIn .. l*kIn+kIn-1). The grid covers the lattice once and each XCD
// takes one contiguous eighth of the tiles (xcd_tile), which it streams in
// address order; on MI355X this is faster than a persistent grid-stride
// loop (which lets workgroups drift apart in memory), than tile =
// workgroup index, and than several tiles per wavefront with the next
// tile's loads in flight during the current one's compute. The four b links are staged once per workgroup in LDS and each
// lane reads the coefficients of its own unit position from there.
// kConjB: stage b[j]^H instead of b[j] (the a b^H product; the kernel is
// otherwise the same).
template <class F, bool kConjB = false>
__global__ __launch_bounds__(kAosBlock) void fwd_aos(const u4 *__restrict__ a, const typename F::B *__restrict__ b,
                                                  u4 *__restrict__ c, int64_t units)
{
    constexpr int kWaves = kAosBlock / 64;
    constexpr int kSlots = 64 * (F::kIn > F::kOut ? F::kIn : F::kOut);
    __shared__ u4 stage[kWaves][kSlots];
    __shared__ __attribute__((aligned(16))) typename F::B bsh[72];

    const int lane = threadIdx.x & 63;
    u4 *my = stage[threadIdx.x >> 6];
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6);
    const bool live = t * 64 < units;            // wave-uniform
    const bool whole = (t + 1) * 64 <= units;    // wave-uniform (no ragged end)
    const int64_t nin = units * F::kIn, nout = units * F::kOut;

    // Load b (72 scalars, cached) first and the tile after it: vector memory
    // operations retire in order, so the workgroup barrier that publishes b
    // in LDS waits for the b load only while the tile is still in flight.
    constexpr int kBPer = (72 + kAosBlock - 1) / kAosBlock;
    typename F::B bv[kBPer];
#pragma unroll
    for (int r = 0; r < kBPer; ++r) {
        const int q = threadIdx.x + r * kAosBlock;
        if (!kConjB) {
            bv[r] = q < 72 ? b[q] : typename F::B(0);
        } else {
            // scalar q = 2*(9j + 3m + l) + part of b^H is part of b[j](l, m),
            // negated for the imaginary part
            const int e = q >> 1, part = q & 1;
            const int j = e / 9, m = (e % 9) / 3, l = e % 3;
            const typename F::B x = q < 72 ? b[2 * (9 * j + 3 * l + m) + part] : typename F::B(0);
            bv[r] = part ? -x : x;
        }
    }
    // Branch-free tile loads: a chunk past the end of the lattice (ragged last
    // tile, or a wavefront with no tile) re-reads the last chunk and is never
    // used, so every load stays in bounds and the wait counts stay exact.
    u4 v[F::kIn];
    const int64_t gin = t * 64 * F::kIn + lane;
#pragma unroll
    for (int i = 0; i < F::kIn; ++i) {
        const int64_t g = gin + 64 * i;
        v[i] = ld_stream(a + (g < nin ? g : nin - 1));
    }
#pragma unroll
    for (int r = 0; r < kBPer; ++r) {
        const int q = threadIdx.x + r * kAosBlock;
        if (q < 72)
            bsh[q] = bv[r];
    }
    __syncthreads();
    if (!live)
        return;
    typename F::Coef coef;
    F::load(bsh, (int)((t * 64 + lane) % F::kUnitsPerSite), coef);
#pragma unroll
    for (int i = 0; i < F::kIn; ++i)
        my[64 * i + lane] = v[i];
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
    store_runs<F::kOut>(c, my, t * 64 * F::kOut + lane, lane, whole, nout);
}

// ---------------------------------------------------------------- SoA
// Thread per (site, output row): the row 3j + k is uniform over a workgroup,
// so the link j and the b[j] entries sit in scalar registers. A wavefront
// reads planes (j, k, 0..2) and writes planes (j, k, 0..2), each access one
// contiguous 1 KiB (FP64) or 512 B (FP32) run; plane p starts at element
// p * pitch (pitch = n for the dense layout). The grid is one dimension of
// 12 rows x nbp workgroups; workgroup `local` of a row takes site block
// local (tile = workgroup index) or, with xcd set, xcd_order(local, nbp),
// which gives each XCD one contiguous eighth of the row's site blocks (nbp
// is then the row's block count rounded up to a multiple of 8, so that
// `local` mod 8 is the XCD; the extra workgroups find no sites and exit).
// kWaits splits a thread's three plane loads into phases (soa_waits): bit 0
// waits for plane 0 before plane 1 is loaded, bit 1 waits for planes 0 and 1
// before plane 2 is loaded; 0 issues all three together. A wait is an empty
// asm statement that takes the accumulators as inputs, so every load before
// it has completed and no later load moves above it. The arithmetic and its
// order are the same for every kWaits, so the output is bit-identical.
template <typename V, typename S, int kWaits>
__global__ __launch_bounds__(kSoaBlock) void fwd_soa(const V *__restrict__ a, const S *__restrict__ b,
                                                  V *__restrict__ c, int64_t n, int64_t pitch, int64_t nbp, int xcd)
{
    const int row = (int)(blockIdx.x / nbp);     // 3j + k
    const int64_t local = (int64_t)blockIdx.x - (int64_t)row * nbp;
    const int64_t xb = xcd ? xcd_order(local, nbp) : local;
    const int j = row / 3;
    const int64_t s = xb * kSoaBlock + threadIdx.x;
    if (s >= n)
        return;
    S br[9], bi[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        br[q] = b[2 * (9 * j + q)];
        bi[q] = b[2 * (9 * j + q) + 1];
    }
    const V *__restrict__ ap = a + (int64_t)(3 * row) * pitch + s;
    V *__restrict__ cp = c + (int64_t)(3 * row) * pitch + s;
    S re[3] = {0, 0, 0}, im[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const V x = ld_stream(ap + m * pitch);
#pragma unroll
        for (int l = 0; l < 3; ++l)
            cmac(re[l], im[l], x.x, x.y, br[3 * m + l], bi[3 * m + l]);
        if ((kWaits >> m) & 1)
            asm volatile("" ::"v"(re[0]), "v"(im[0]), "v"(re[1]), "v"(im[1]), "v"(re[2]), "v"(im[2]) : "memory");
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        V o = {re[l], im[l]};
        st_stream(cp + l * pitch, o);
    }
}

// Tile order of the SoA product. The three input planes of a row are read at
// the same site offsets, plane stride n * elem_bytes apart. When that stride
// is close to a multiple of 4 MiB (within 128 KiB), the planes of the one
// window that tile = workgroup index streams collide in HBM and FP64 runs at
// 0.88-0.93 of the site-major rate (sizes 2^20 +- 64, 2^20 + 4096, 3 * 2^19,
// 2^21, 2^22); the XCD-contiguous order spreads the row over eight windows
// and runs at 0.94-0.97 there, but at other strides it is 1-7% slower than
// tile = workgroup index (sizes 24^4, 36^4, 40^4, 48^4, 56^4, 17 * 2^16). FP32
// keeps tile = workgroup index at every stride (the XCD order measured equal
// or slower), and so does a padded layout (pitch > n): with the pitch of
// soa_pitch it streams at the site-major rate in that order.
static bool soa_xcd(int64_t sites, int64_t pitch, int elem_bytes)
{
    if (elem_bytes != 16 || pitch != sites)
        return false;
    const int64_t m = (sites * 16) % ((int64_t)4 << 20);
    return m < ((int64_t)128 << 10) || m > ((int64_t)4 << 20) - ((int64_t)128 << 10);
}

// Load phases of the SoA product (fwd_soa). When all of a thread's plane
// loads are in flight together, the workgroups that run at once read the
// three planes of a row at the same site window, one plane stride apart, and
// at some strides those reads collide in HBM. Waiting between phases makes a
// workgroup's planes arrive one after another, so at any moment the
// resident workgroups, which started at different times, read different
// planes at different site offsets. That costs bytes in flight per
// wavefront, which more resident wavefronts make up for.
// FP32 (no occupancy cap), measured on random data at 16 site counts from
// 24^4 to 56^4 as the rate over site-major. Stock kernel: 0.84-1.05 (mean
// 0.954). Waiting before plane 2: 0.88-1.04 (0.981). Waiting after every
// plane is best where the plane stride is a multiple of 8 MiB and at least
// 16 MiB: 0.92-0.98 there, against 0.84-0.95 stock and 0.88-0.98 with one
// wait.
// FP64 loses with waits at its occupancy cap of 8 wavefronts (up to a
// third), and with a cap of 16 it is 1-2% slower on average, but at
// plane strides that are multiples of 16 MiB one wait after plane 0 with a
// cap of 16 gained: 0.996-1.013 against 0.960-0.966 at 16 MiB (L=32),
// 0.963 against 0.955 at 48 MiB, 0.944 against 0.935 at 128 MiB, and
// 0.95-0.96 either way at 32 and 64 MiB.
// The padded layout keeps no waits: its stride does not collide.
// Returns the wait mask; *waves is the occupancy cap to launch with.
static int soa_waits(int64_t sites, int64_t pitch, int elem_bytes, int *waves)
{
    const int64_t stride = sites * elem_bytes;
    auto near = [stride](int64_t period) {
        const int64_t m = stride % period;
        return m < ((int64_t)128 << 10) || m > period - ((int64_t)128 << 10);
    };
    const int64_t lo16 = ((int64_t)16 << 20) - ((int64_t)128 << 10);
    if (elem_bytes == 16) {
        const bool phased = pitch == sites && stride >= lo16 && near((int64_t)16 << 20);
        *waves = phased ? SU3_WAVES_SOA_F64_PHASED : SU3_WAVES_SOA_F64;
        return phased ? 1 : 0;
    }
    *waves = SU3_WAVES_SOA_F32;
    if (pitch != sites)
        return 0;
    return near((int64_t)8 << 20) && stride >= lo16 ? 3 : 2;
}

// Plane pitch of the padded SoA layout at which the product streams at the
// site-major rate in workgroup order: the site count rounded up to 64 plus
// 512 (FP64, 8 KiB per plane) or 128 (FP32, 1 KiB). Measured on random data
// at 14 site counts from 24^4 to 56^4 (powers of two and their neighbours
// among them), as the SoA rate over the site-major rate: 0.976-1.031 (mean
// 0.996) in FP64 and 0.972-1.020 (mean 0.994) in FP32, where the dense layout
// ran at 0.934-1.020 (0.981) and, before the FP32 load phases, 0.845-1.024
// (0.957); with them 0.909-1.052 (0.989) in another run. The pad is not monotone
// in its effect, and no fixed residue of the plane stride mod 64 KiB did as
// well at every size: a 1 KiB FP64 stride residue left 2^20 - 64 at 0.89,
// and 16 KiB left 2^20 at 0.86.
int64_t soa_pitch(int64_t sites, int elem_bytes)
{
    return (sites + 63) / 64 * 64 + (elem_bytes == 16 ? 512 : 128);
}

static int64_t soa_blocks_per_row(int64_t sites, int64_t pitch, int elem_bytes)
{
    const int64_t nb = (sites + kSoaBlock - 1) / kSoaBlock;
    return soa_xcd(sites, pitch, elem_bytes) ? (nb + kXcds - 1) / kXcds * kXcds : nb;
}

// ---------------------------------------------------------------- launchers
// Dynamic LDS to add per workgroup so that at most `waves` wavefronts of
// `kernel` are resident per CU: the CU's LDS divided by the wanted number of
// workgroups, minus the kernel's static LDS. Cached per device; 0 when no cap
// is wanted or a query fails.
size_t occupancy_pad_for(const void *kernel, int waves, int block, int dev)
{
    int lds_cu = 0, lds_block = 0;
    hipFuncAttributes attr;
    int pad = 0;
    if (waves > 0 && hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        hipFuncGetAttributes(&attr, kernel) == hipSuccess) {
        // LDS is allocated in granules; round each workgroup's share down to
        // 1 KiB so that `blocks` of them fit
        const int blocks = waves * 64 / block > 0 ? waves * 64 / block : 1;
        const int want = (lds_cu / blocks) / 1024 * 1024 - (int)attr.sharedSizeBytes;
        const int room = lds_block - (int)attr.sharedSizeBytes;
        pad = want > 0 ? (want < room ? want : room) : 0;
    }
    return (size_t)pad;
}

size_t occupancy_pad(const void *kernel, int waves, int block, std::atomic<int> (&cache)[kMaxDevices])
{
    if (waves <= 0)
        return 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return 0;
    int pad = cache[dev].load(std::memory_order_relaxed);   // pad + 1; 0 = not yet known
    if (pad > 0)
        return (size_t)(pad - 1);
    pad = (int)occupancy_pad_for(kernel, waves, block, dev);
    cache[dev].store(pad + 1, std::memory_order_relaxed);
    return (size_t)pad;
}

template <class F>
static int64_t aos_grid(int64_t sites)
{
    const int64_t tiles = (sites * F::kUnitsPerSite + 63) / 64;
    return (tiles + kAosBlock / 64 - 1) / (kAosBlock / 64);
}

int64_t fwd_aos_grid(int precision, int64_t sites)
{
    switch (precision) {
    case 0: return aos_grid<FormF64>(sites);
    case 1: return aos_grid<FormF32>(sites);
    case 2: return aos_grid<FormBF16>(sites);
    case 3: return aos_grid<FormR12>(sites);
    case 4: return aos_grid<FormR12C>(sites);
    default: return aos_grid<FormR12F64>(sites);
    }
}

int64_t fwd_an_grid(int precision, int64_t sites)
{
    return precision == 0 ? aos_grid<FormAnF64>(sites) : aos_grid<FormAnF32>(sites);
}

int64_t fwd_soa_grid(int64_t sites, int64_t pitch, int elem_bytes)
{
    return 12 * soa_blocks_per_row(sites, pitch, elem_bytes);
}
int soa_block_threads() { return kSoaBlock; }

template <class F, bool kConjB = false>
static hipError_t launch_aos(const void *a, const void *b, void *c, int64_t sites, hipStream_t s)
{
    static std::atomic<int> pad_cache[kMaxDevices];
    const size_t pad =
        occupancy_pad(reinterpret_cast<const void *>(fwd_aos<F, kConjB>), F::kWavesPerCU, kAosBlock, pad_cache);
    return launch_k(fwd_aos<F, kConjB>, dim3((unsigned)aos_grid<F>(sites)), dim3(kAosBlock), s, pad,
                    (const u4 *)a, (const typename F::B *)b, (u4 *)c, sites * F::kUnitsPerSite);
}

hipError_t launch_fwd_aos(const void *a, const void *b, void *c, int64_t sites, int precision, hipStream_t s)
{
    switch (precision) {
    case 0: return launch_aos<FormF64>(a, b, c, sites, s);
    case 1: return launch_aos<FormF32>(a, b, c, sites, s);
    case 2: return launch_aos<FormBF16>(a, b, c, sites, s);
    case 3: return launch_aos<FormR12>(a, b, c, sites, s);
    case 4: return launch_aos<FormR12C>(a, b, c, sites, s);
    default: return launch_aos<FormR12F64>(a, b, c, sites, s);
    }
}

hipError_t launch_fwd_na(const void *a, const void *b, void *c, int64_t sites, int precision, hipStream_t s)
{
    if (precision == 0)
        return launch_aos<FormF64, true>(a, b, c, sites, s);
    return launch_aos<FormF32, true>(a, b, c, sites, s);
}

hipError_t launch_fwd_an(const void *a, const void *b, void *c, int64_t sites, int precision, hipStream_t s)
{
    if (precision == 0)
        return launch_aos<FormAnF64>(a, b, c, sites, s);
    return launch_aos<FormAnF32>(a, b, c, sites, s);
}

// Each instantiation is launched with one occupancy cap only (soa_waits maps
// the wait mask to its cap), so one pad cache per instantiation suffices.
template <typename V, typename S, int kWaits>
static hipError_t launch_soa(const void *a, const void *b, void *c, int64_t sites, int64_t pitch, int waves,
                             hipStream_t s)
{
    static std::atomic<int> pad_cache[kMaxDevices];
    const int es = (int)sizeof(V);
    const int64_t nbp = soa_blocks_per_row(sites, pitch, es);
    const int xcd = soa_xcd(sites, pitch, es) ? 1 : 0;
    const size_t pad =
        occupancy_pad(reinterpret_cast<const void *>(fwd_soa<V, S, kWaits>), waves, kSoaBlock, pad_cache);
    return launch_k(fwd_soa<V, S, kWaits>, dim3((unsigned)(12 * nbp)), dim3(kSoaBlock), s, pad, (const V *)a,
                    (const S *)b, (V *)c, sites, pitch, nbp, xcd);
}

hipError_t launch_fwd_soa(const void *a, const void *b, void *c, int64_t sites, int64_t pitch, int elem_bytes,
                          hipStream_t s)
{
    int waves = 0;
    const int waits = soa_waits(sites, pitch, elem_bytes, &waves);
    if (elem_bytes == 16)
        return waits ? launch_soa<d2, double, 1>(a, b, c, sites, pitch, waves, s)
                     : launch_soa<d2, double, 0>(a, b, c, sites, pitch, waves, s);
    switch (waits) {
    case 0: return launch_soa<f2, float, 0>(a, b, c, sites, pitch, waves, s);
    case 2: return launch_soa<f2, float, 2>(a, b, c, sites, pitch, waves, s);
    default: return launch_soa<f2, float, 3>(a, b, c, sites, pitch, waves, s);
    }
}

} // namespace su3
