// su3_layout.hip -- data movement around the link multiply on gfx950:
// AoS <-> SoA transposes, FP64 <-> storage-form conversion (pack/unpack),
// and the plain streaming copy used as the bandwidth reference.
#include "su3_internal.hpp"

#include <type_traits>

// Resident wavefronts per CU for the reconstruct-12 unpack (9 KiB of stores
// and 3 or 6 KiB of loads per wavefront).
#ifndef SU3_WAVES_UNPACK_R12
#define SU3_WAVES_UNPACK_R12 7
#endif
// ... and for the reconstruct-12 pack (9 KiB of loads per wavefront).
#ifndef SU3_WAVES_PACK_R12
#define SU3_WAVES_PACK_R12 6
#endif

namespace su3 {

// The elementwise setup kernels (FP32 and BF16 pack and unpack, transposes)
// loop over their items with a grid stride, on a grid of up to kOnePass
// workgroups: one pass for any lattice that fits in memory, which streams
// faster than fewer workgroups looping.
constexpr int64_t kOnePass = (int64_t)1 << 24;

typedef uint32_t u2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------ AoS <-> SoA
// One workgroup moves a tile of 64 sites at a time through LDS: the site-
// major side is read or written as one contiguous run of 64*36 elements, the
// plane side as 36 contiguous runs of 64 elements. The LDS row has one
// element of padding so that the column walk does not hit one bank.
// A whole tile is moved with every load of a thread issued before the first
// LDS write (9 elements per thread), nontemporal loads and stores, and, in
// FP64, the XCD-contiguous tile order (each XCD one contiguous eighth of the
// tiles; a one-pass grid). Against element-at-a-time loops with plain
// accesses in tile = workgroup index order (random data, AoS -> SoA / SoA ->
// AoS, TB/s): FP64 L=48 5.30 / 5.75 against 5.31 / 5.62, L=32 5.65 / 5.85
// against 5.16 / 5.47; FP32 (workgroup order: the XCD order was 0-6% slower
// there) L=48 5.64 / 5.96 against 5.33 / 5.54, L=32 6.06 / 5.80 against
// 5.04 / 5.15. 128- and 64-thread workgroups, 32-site tiles and loads in
// three phases were within 2% either way or slower. The last, ragged tile
// moves element by element.
constexpr int kTileSites = 64;

template <typename V, bool kToSoa, bool kXcd>
__global__ __launch_bounds__(kBlock) void transpose_aos_soa(const V *__restrict__ src, V *__restrict__ dst,
                                                            int64_t n, int64_t pitch)
{
    __shared__ V tile[36][kTileSites + 1];
    constexpr int kPer = 36 * kTileSites / kBlock;
    static_assert(kPer * kBlock == 36 * kTileSites, "a tile splits evenly over the workgroup");
    const int64_t tiles = (n + kTileSites - 1) / kTileSites;
    // the XCD order needs the one-pass grid (one workgroup per tile)
    int64_t t = blockIdx.x;
    if (kXcd && (int64_t)gridDim.x >= tiles)
        t = xcd_order(blockIdx.x, gridDim.x);
    for (; t < tiles; t += gridDim.x) {
        const int64_t s0 = t * kTileSites;
        const int ns = (int)((n - s0) < kTileSites ? (n - s0) : kTileSites);
        if (ns == kTileSites) {
            V v[kPer];
            if (kToSoa) {
#pragma unroll
                for (int i = 0; i < kPer; ++i)
                    v[i] = ld_stream(src + s0 * 36 + threadIdx.x + i * kBlock);
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = threadIdx.x + i * kBlock;
                    tile[e % 36][e / 36] = v[i];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = threadIdx.x + i * kBlock;
                    v[i] = tile[e / kTileSites][e % kTileSites];
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = threadIdx.x + i * kBlock;
                    st_stream(dst + (int64_t)(e / kTileSites) * pitch + s0 + e % kTileSites, v[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = threadIdx.x + i * kBlock;
                    v[i] = ld_stream(src + (int64_t)(e / kTileSites) * pitch + s0 + e % kTileSites);
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = threadIdx.x + i * kBlock;
                    tile[e / kTileSites][e % kTileSites] = v[i];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const int e = threadIdx.x + i * kBlock;
                    v[i] = tile[e % 36][e / 36];
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i)
                    st_stream(dst + s0 * 36 + threadIdx.x + i * kBlock, v[i]);
            }
        } else if (kToSoa) {
            for (int e = threadIdx.x; e < ns * 36; e += kBlock)
                tile[e % 36][e / 36] = src[s0 * 36 + e];
            __syncthreads();
            for (int e = threadIdx.x; e < 36 * kTileSites; e += kBlock) {
                const int p = e / kTileSites, sl = e % kTileSites;
                if (sl < ns)
                    dst[(int64_t)p * pitch + s0 + sl] = tile[p][sl];
            }
        } else {
            for (int e = threadIdx.x; e < 36 * kTileSites; e += kBlock) {
                const int p = e / kTileSites, sl = e % kTileSites;
                if (sl < ns)
                    tile[p][sl] = src[(int64_t)p * pitch + s0 + sl];
            }
            __syncthreads();
            for (int e = threadIdx.x; e < ns * 36; e += kBlock)
                dst[s0 * 36 + e] = tile[e % 36][e / 36];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ pack
// FP64 complex -> FP32 complex, round to nearest even (v_cvt_f32_f64).
template <int B>
__global__ __launch_bounds__(B) void pack_f32(const d2 *__restrict__ src, f2 *__restrict__ dst, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * B + threadIdx.x; e < n; e += (int64_t)gridDim.x * B) {
        const d2 v = src[e];
        f2 o = {(float)v.x, (float)v.y};
        dst[e] = o;
    }
}

// FP64 complex -> BF16 (re, im), through FP32, each step to nearest even.
template <int B>
__global__ __launch_bounds__(B) void pack_bf16(const d2 *__restrict__ src, uint32_t *__restrict__ dst,
                                                    int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * B + threadIdx.x; e < n; e += (int64_t)gridDim.x * B) {
        const d2 v = src[e];
        dst[e] = pack_bf16x2((float)v.x, (float)v.y);
    }
}

// FP64 links -> rows 0 and 1 in FP32 (V = f2, round to nearest even) or FP64
// (V = d2), the reconstruct-12 storage. One wavefront per tile of 64 links:
// whole-wavefront 1 KiB runs of the tile's links (9 chunks each) in, the
// rows 0-1 of each (3 or 6 chunks) out, through a private LDS slice.
template <typename V>
__global__ __launch_bounds__(64) void pack_r12(const u4 *__restrict__ src, u4 *__restrict__ dst, int64_t links)
{
    constexpr int kOut = sizeof(V) == 8 ? 3 : 6;   // output chunks per link
    __shared__ u4 stage[64 * 9];
    const int lane = threadIdx.x;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t nin = links * 9, nout = links * kOut;
    const bool whole = (t + 1) * 64 <= links;
    u4 v[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int64_t g = t * 64 * 9 + 64 * i + lane;
        v[i] = ld_stream(src + (g < nin ? g : nin - 1));   // in bounds; unused past the end
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        stage[64 * i + lane] = v[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    typedef typename std::conditional<sizeof(V) == 8, float, double>::type E;   // element of V
    V o[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const d2 w = __builtin_bit_cast(d2, stage[9 * lane + q]);
        o[q] = V{(E)w.x, (E)w.y};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    V *out = reinterpret_cast<V *>(stage) + 6 * lane;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        out[q] = o[q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < kOut; ++i) {
        const int64_t g = t * 64 * kOut + 64 * i + lane;
        if (whole || g < nout)
            st_stream(dst + g, stage[64 * i + lane]);
    }
}

// ------------------------------------------------------------ unpack
template <int B>
__global__ __launch_bounds__(B) void unpack_f32(const f2 *__restrict__ src, d2 *__restrict__ dst, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * B + threadIdx.x; e < n; e += (int64_t)gridDim.x * B) {
        const f2 v = src[e];
        d2 o = {(double)v.x, (double)v.y};
        dst[e] = o;
    }
}

// BF16 -> FP64, exact; two complex numbers per thread (one 8-byte load, two
// 16-byte stores). n2 = number of pairs (36 complex per site, so no odd one).
template <int B>
__global__ __launch_bounds__(B) void unpack_bf16(const u2 *__restrict__ src, d2 *__restrict__ dst, int64_t n2)
{
    for (int64_t e = (int64_t)blockIdx.x * B + threadIdx.x; e < n2; e += (int64_t)gridDim.x * B) {
        const u2 w = src[e];
        const d2 o0 = {(double)bf16_lo(w.x), (double)bf16_hi(w.x)};
        const d2 o1 = {(double)bf16_lo(w.y), (double)bf16_hi(w.y)};
        dst[2 * e] = o0;
        dst[2 * e + 1] = o1;
    }
}

// Rows 0-1 (FP32 or FP64) -> full FP64 link; row 2 = conj(row0 x row1) evaluated in
// FP64 without contraction, each product and difference rounded on its own,
// in the order (r0_p r1_q) - (r0_q r1_p) with each complex product formed as
// (re*re - im*im, re*im + im*re). The result is then a fixed function of the
// stored rows, independent of compiler contraction choices.
// One wavefront per tile of 64 links, the streaming pattern of the product
// kernels: the tile's rows 0-1 (3 chunks per link in FP32, 6 in FP64) and its
// full FP64 links (9 chunks each) move in whole-wavefront 1 KiB runs, and a
// private LDS slice turns them into one link per lane. Row 2 is rebuilt in
// FP64 with contraction off, in the oracle's operation order, so the result
// is bit-exact.
template <typename V>
__global__ __launch_bounds__(64) void unpack_r12(const u4 *__restrict__ src, u4 *__restrict__ dst, int64_t links)
{
#pragma clang fp contract(off)
    constexpr int kIn = sizeof(V) == 8 ? 3 : 6;   // input chunks per link
    __shared__ u4 stage[64 * 9];
    const int lane = threadIdx.x;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t nin = links * kIn, nout = links * 9;
    const bool whole = (t + 1) * 64 <= links;
    u4 v[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) {
        const int64_t g = t * 64 * kIn + 64 * i + lane;
        v[i] = ld_stream(src + (g < nin ? g : nin - 1));   // in bounds; unused past the end
    }
#pragma unroll
    for (int i = 0; i < kIn; ++i)
        stage[64 * i + lane] = v[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double r[12];
    const V *in = reinterpret_cast<const V *>(stage) + 6 * lane;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const V w = in[q];
        r[2 * q] = (double)w.x;
        r[2 * q + 1] = (double)w.y;
    }
    d2 o[9];
#pragma unroll
    for (int q = 0; q < 6; ++q)
        o[q] = d2{r[2 * q], r[2 * q + 1]};
    const double *r0 = r, *r1 = r + 6;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int p = (l + 1) % 3, q = (l + 2) % 3;
        const double pr = r0[2 * p] * r1[2 * q] - r0[2 * p + 1] * r1[2 * q + 1];
        const double pi = r0[2 * p] * r1[2 * q + 1] + r0[2 * p + 1] * r1[2 * q];
        const double qr = r0[2 * q] * r1[2 * p] - r0[2 * q + 1] * r1[2 * p + 1];
        const double qi = r0[2 * q] * r1[2 * p + 1] + r0[2 * q + 1] * r1[2 * p];
        o[6 + l] = d2{pr - qr, -(pi - qi)};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < 9; ++q)
        stage[9 * lane + q] = __builtin_bit_cast(u4, o[q]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int64_t g = t * 64 * 9 + 64 * i + lane;
        if (whole || g < nout)
            st_stream(dst + g, stage[64 * i + lane]);
    }
}

// ------------------------------------------------------------ stream copy
// dst[i] = src[i] over 16-byte elements, one element per thread, with
// nontemporal loads and stores; the grid covers the buffer once, so the
// dispatcher streams it in address order. Workgroups of one wavefront.
constexpr int kCopyBlock = 64;

__global__ __launch_bounds__(kCopyBlock) void stream_copy(const u4 *__restrict__ src, u4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kCopyBlock + threadIdx.x;
    if (i < n)
        st_stream(dst + i, ld_stream(src + i));
}

// Access-shape probe: wavefront w (the workgroup index, or with order 1 its
// XCD-contiguous tile, xcd_order) reads chunks w*64*RA + 64 i + lane of a
// (i < RA) and likewise of b, and writes chunks w*64*W + 64 i + lane of c,
// the same whole-wavefront 1 KiB runs and per-lane chunk counts as the
// kernels it stands beside, with no arithmetic beyond folding the loads
// into the stored values (so that no load is dead).
template <int RA, int RB, int W>
__global__ __launch_bounds__(64) void stream_shape(const u4 *__restrict__ a, const u4 *__restrict__ b,
                                                   u4 *__restrict__ c, int order)
{
    const int64_t w = order ? xcd_order(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int lane = threadIdx.x;
    u4 va[RA], vb[RB > 0 ? RB : 1];
#pragma unroll
    for (int i = 0; i < RA; ++i)
        va[i] = ld_stream(a + w * 64 * RA + 64 * i + lane);
#pragma unroll
    for (int i = 0; i < RB; ++i)
        vb[i] = ld_stream(b + w * 64 * RB + 64 * i + lane);
    u4 x = va[0];
#pragma unroll
    for (int i = 1; i < RA; ++i)
        x ^= va[i];
#pragma unroll
    for (int i = 0; i < RB; ++i)
        x ^= vb[i];
#pragma unroll
    for (int i = 0; i < W; ++i) {
        u4 o = x;
        o.x += (uint32_t)i;
        st_stream(c + w * 64 * W + 64 * i + lane, o);
    }
}

// ------------------------------------------------------------ launchers
static unsigned grid_for(int64_t items, int64_t per_block, int64_t cap = kOnePass)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g > cap)
        g = cap;
    if (g < 1)
        g = 1;
    return (unsigned)g;
}

hipError_t launch_aos_soa(const void *src, void *dst, int64_t sites, int64_t pitch, int elem_bytes, bool to_soa,
                          hipStream_t s)
{
    const unsigned g = grid_for(sites, kTileSites);
    if (elem_bytes == 16) {
        if (to_soa)
            return launch_k(transpose_aos_soa<d2, true, true>, dim3(g), dim3(kBlock), s, 0, (const d2 *)src, (d2 *)dst,
                            sites, pitch);
        return launch_k(transpose_aos_soa<d2, false, true>, dim3(g), dim3(kBlock), s, 0, (const d2 *)src, (d2 *)dst,
                        sites, pitch);
    }
    if (to_soa)
        return launch_k(transpose_aos_soa<f2, true, false>, dim3(g), dim3(kBlock), s, 0, (const f2 *)src, (f2 *)dst,
                        sites, pitch);
    return launch_k(transpose_aos_soa<f2, false, false>, dim3(g), dim3(kBlock), s, 0, (const f2 *)src, (f2 *)dst,
                    sites, pitch);
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s)
{
    const int64_t n = bytes / 16;
    return launch_k(stream_copy, dim3((unsigned)((n + kCopyBlock - 1) / kCopyBlock)), dim3(kCopyBlock), s, 0,
                    (const u4 *)src, (u4 *)dst, n);
}

bool stream_shape_supported(int in_a, int in_b, int out)
{
    return (in_a == 1 && in_b == 0 && out == 1) || (in_a == 3 && in_b == 0 && out == 3) ||
           (in_a == 3 && in_b == 3 && out == 3) || (in_a == 6 && in_b == 0 && out == 9) ||
           (in_a == 9 && in_b == 0 && out == 9);
}

template <int RA, int RB, int W>
static hipError_t launch_shape_k(const void *a, const void *b, void *c, int64_t tiles, int waves, int order,
                                 hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return hipErrorInvalidDevice;
    const size_t pad = occupancy_pad_for(reinterpret_cast<const void *>(stream_shape<RA, RB, W>), waves, 64, dev);
    return launch_k(stream_shape<RA, RB, W>, dim3((unsigned)tiles), dim3(64), s, pad, (const u4 *)a, (const u4 *)b,
                    (u4 *)c, order);
}

hipError_t launch_stream_shape(const void *a, const void *b, void *c, int64_t tiles, int in_a, int in_b, int out,
                               int waves_per_cu, int tile_order, hipStream_t s)
{
    if (in_a == 1 && in_b == 0 && out == 1)
        return launch_shape_k<1, 0, 1>(a, b, c, tiles, waves_per_cu, tile_order, s);
    if (in_a == 3 && in_b == 0 && out == 3)
        return launch_shape_k<3, 0, 3>(a, b, c, tiles, waves_per_cu, tile_order, s);
    if (in_a == 3 && in_b == 3 && out == 3)
        return launch_shape_k<3, 3, 3>(a, b, c, tiles, waves_per_cu, tile_order, s);
    if (in_a == 6 && in_b == 0 && out == 9)
        return launch_shape_k<6, 0, 9>(a, b, c, tiles, waves_per_cu, tile_order, s);
    if (in_a == 9 && in_b == 0 && out == 9)
        return launch_shape_k<9, 0, 9>(a, b, c, tiles, waves_per_cu, tile_order, s);
    return hipErrorInvalidValue;
}

template <typename V>
static hipError_t launch_pack_r12(const void *src, void *dst, int64_t links, hipStream_t s)
{
    static std::atomic<int> pad[kMaxDevices];
    const size_t p = occupancy_pad(reinterpret_cast<const void *>(pack_r12<V>), SU3_WAVES_PACK_R12, 64, pad);
    return launch_k(pack_r12<V>, dim3((unsigned)((links + 63) / 64)), dim3(64), s, p, (const u4 *)src, (u4 *)dst,
                    links);
}

// precision codes as in su3.h: 0 F64, 1 F32, 2 BF16, 3 R12_F32 (rows 0-1 FP32
// in, full FP32 out), 4 R12C_F32 (rows 0-1 FP32 in and out), 5 R12_F64 (rows
// 0-1 FP64 in, full FP64 out). Codes 3 and 4 share the storage of a.
hipError_t launch_pack(const void *src, void *dst, int64_t sites, int precision, hipStream_t s)
{
    const int64_t elems = sites * 36, links = sites * 4;
    switch (precision) {
    case 1:
        return launch_k(pack_f32<64>, dim3(grid_for(elems, 64, kOnePass)), dim3(64), s, 0, (const d2 *)src,
                        (f2 *)dst, elems);
    case 2:
        return launch_k(pack_bf16<128>, dim3(grid_for(elems, 128, kOnePass)), dim3(128), s, 0, (const d2 *)src,
                        (uint32_t *)dst, elems);
    case 3:
    case 4:
        return launch_pack_r12<f2>(src, dst, links, s);
    case 5:
        return launch_pack_r12<d2>(src, dst, links, s);
    default:
        return launch_stream_copy(src, dst, elems * 16, s);
    }
}

hipError_t launch_unpack(const void *src, void *dst, int64_t sites, int precision, hipStream_t s)
{
    const int64_t elems = sites * 36, links = sites * 4;
    switch (precision) {
    case 1:
        return launch_k(unpack_f32<64>, dim3(grid_for(elems, 64, kOnePass)), dim3(64), s, 0, (const f2 *)src, (d2 *)dst,
                        elems);
    case 2:
        return launch_k(unpack_bf16<256>, dim3(grid_for(elems / 2, 256, kOnePass)), dim3(256), s, 0, (const u2 *)src,
                        (d2 *)dst, elems / 2);
    case 3:
    case 4: {
        static std::atomic<int> pad[kMaxDevices];
        const size_t p = occupancy_pad(reinterpret_cast<const void *>(unpack_r12<f2>), SU3_WAVES_UNPACK_R12, 64, pad);
        return launch_k(unpack_r12<f2>, dim3((unsigned)((links + 63) / 64)), dim3(64), s, p, (const u4 *)src,
                        (u4 *)dst, links);
    }
    case 5: {
        static std::atomic<int> pad[kMaxDevices];
        const size_t p = occupancy_pad(reinterpret_cast<const void *>(unpack_r12<d2>), SU3_WAVES_UNPACK_R12, 64, pad);
        return launch_k(unpack_r12<d2>, dim3((unsigned)((links + 63) / 64)), dim3(64), s, p, (const u4 *)src,
                        (u4 *)dst, links);
    }
    default:
        return launch_stream_copy(src, dst, elems * 16, s);
    }
}

} // namespace su3
