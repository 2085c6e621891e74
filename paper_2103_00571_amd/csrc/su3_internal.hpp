// su3_internal.hpp -- device helpers and launcher declarations shared by the
// kernel files of libsu3 (gfx950). Not part of the public ABI (include/su3.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <tuple>

namespace su3 {

// 16-byte vector types as clang ext vectors, so that __builtin_nontemporal_*
// accept them and the compiler emits one global_load/store_dwordx4 each.
typedef double d2 __attribute__((ext_vector_type(2)));   // one complex double
typedef float f4 __attribute__((ext_vector_type(4)));    // two complex float
typedef float f2 __attribute__((ext_vector_type(2)));    // one complex float
typedef uint32_t u4 __attribute__((ext_vector_type(4))); // eight bf16
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

// Streaming accesses: a and c are touched once per call, so loads and stores
// carry the nontemporal hint (global_load/store ... nt) and do not displace
// the b links or other data from the caches.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) { __builtin_nontemporal_store(v, p); }

// complex multiply-accumulate acc += x * y, four fused multiply-adds
__device__ __forceinline__ void cmac(double &re, double &im, double xr, double xi, double yr, double yi)
{
    re = __builtin_fma(xr, yr, re);
    re = __builtin_fma(-xi, yi, re);
    im = __builtin_fma(xr, yi, im);
    im = __builtin_fma(xi, yr, im);
}
__device__ __forceinline__ void cmac(float &re, float &im, float xr, float xi, float yr, float yi)
{
    re = __builtin_fmaf(xr, yr, re);
    re = __builtin_fmaf(-xi, yi, re);
    im = __builtin_fmaf(xr, yi, im);
    im = __builtin_fmaf(xi, yr, im);
}

// BF16 <-> FP32. Widening is a shift; narrowing rounds to nearest even
// (v_cvt_pk_bf16_f32 on gfx950 under the default rounding mode).
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi)
{
    f2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2));
}

// XCD-contiguous tile order of a one-pass grid of nb workgroups. The
// dispatcher deals workgroups round-robin to MI355X's 8 XCDs (workgroup i to
// XCD i mod 8); here the k-th workgroup of XCD x takes tile
// x*q + min(x, r) + k (q = nb / 8, r = nb mod 8), so each XCD streams one
// contiguous eighth of the buffers in address order instead of every eighth
// tile. A bijection on [0, nb) for any nb: XCD x owns q tiles, plus one if
// x < r. The 8 is the XCD count of one device in the single-partition mode;
// under another partitioning the order is still a bijection, so results do
// not change, only the streaming rate may.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_order(int64_t bid, int64_t nb)
{
    const int64_t q = nb / kXcds, r = nb % kXcds, x = bid % kXcds;
    return x * q + (x < r ? x : r) + bid / kXcds;
}

// The tile of this workgroup in the site-major products, the matrix-vector
// product and the reconstruct-12 pack and unpack: XCD-contiguous (at L = 48
// it streams 3-5% faster than tile = workgroup index at the best cap of
// each). SU3_XCD_ORDER 0 restores tile = workgroup index.
#ifndef SU3_XCD_ORDER
#define SU3_XCD_ORDER 1
#endif
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t nb)
{
    return SU3_XCD_ORDER ? xcd_order(bid, nb) : bid;
}

// Store N whole-wavefront runs from a wavefront's LDS slice:
// dst[base + 64 i] = slice[64 i + lane] for i < N, where base already holds
// the lane's offset; positions at or past n are skipped unless the tile is
// whole (wave-uniform). Every LDS read is issued before the first store, so
// the wavefront waits for LDS once, and a whole tile stores without
// branches.
template <int N>
__device__ __forceinline__ void store_runs(u4 *__restrict__ dst, const u4 *slice, int64_t base, int lane, bool whole,
                                           int64_t n)
{
    u4 w[N];
#pragma unroll
    for (int i = 0; i < N; ++i)
        w[i] = slice[64 * i + lane];
    if (whole) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            st_stream(dst + base + 64 * i, w[i]);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (base + 64 * i < n)
                st_stream(dst + base + 64 * i, w[i]);
    }
}

// Threads per workgroup of the streaming kernels: four wave64s.
constexpr int kBlock = 256;

// Devices per process for the per-device caches.
constexpr int kMaxDevices = 64;

// Launch a kernel through hipLaunchKernel, which reports a failed launch in
// its return value; each argument is converted to the kernel's parameter type.
// dyn_lds is the dynamic LDS size in bytes.
template <typename... KArgs, typename... Args>
inline hipError_t launch_k(void (*k)(KArgs...), dim3 grid, dim3 block, hipStream_t s, size_t dyn_lds, Args... args)
{
    static_assert(sizeof...(KArgs) == sizeof...(Args), "argument count");
    struct Pack {
        std::tuple<KArgs...> t;
    };
    Pack p{std::tuple<KArgs...>(static_cast<KArgs>(args)...)};
    void *argv[sizeof...(KArgs)];
    std::apply([&](auto &...e) {
        int i = 0;
        ((argv[i++] = (void *)&e), ...);
    }, p.t);
    return hipLaunchKernel(reinterpret_cast<const void *>(k), grid, block, argv, dyn_lds, s);
}

// Dynamic LDS to add to each workgroup of `kernel` (block threads each) so
// that at most `waves` wavefronts are resident per CU; 0 for no cap. Cached
// per device in `cache` (entries start at 0).
size_t occupancy_pad(const void *kernel, int waves, int block, std::atomic<int> (&cache)[kMaxDevices]);
// The same pad for device `dev`, computed on every call (no cache).
size_t occupancy_pad_for(const void *kernel, int waves, int block, int dev);

// ---- launchers (each returns hipSuccess or the launch error) --------------
// Forward products. The grid covers the lattice once; *_grid report it.
int64_t fwd_aos_grid(int precision, int64_t sites);
int64_t fwd_soa_grid(int64_t sites, int64_t pitch, int elem_bytes);
// Plane pitch (elements) of the padded SoA layout that streams at the site-major rate.
int64_t soa_pitch(int64_t sites, int elem_bytes);
int soa_block_threads();
hipError_t launch_fwd_aos(const void *a, const void *b, void *c, int64_t sites, int precision, hipStream_t s);
// The a b^H and a^H b products (FP64 = 0, FP32 = 1).
int64_t fwd_an_grid(int precision, int64_t sites);
hipError_t launch_fwd_na(const void *a, const void *b, void *c, int64_t sites, int precision, hipStream_t s);
hipError_t launch_fwd_an(const void *a, const void *b, void *c, int64_t sites, int precision, hipStream_t s);
// Matrix times colour vector, w[s][j] = a[s][j] v[s] (FP64 = 0, FP32 = 1).
int64_t mat_vec_grid(int precision, int64_t sites);
hipError_t launch_mat_vec(const void *a, const void *v, void *w, int64_t sites, int precision, hipStream_t s);
// SoA product; plane p of a and c starts at element p * pitch (pitch >= sites).
hipError_t launch_fwd_soa(const void *a, const void *b, void *c, int64_t sites, int64_t pitch, int elem_bytes,
                          hipStream_t s);
int aos_block_threads();
// Layout and storage-form conversions.
hipError_t launch_aos_soa(const void *src, void *dst, int64_t sites, int64_t pitch, int elem_bytes, bool to_soa,
                          hipStream_t s);
hipError_t launch_pack(const void *src, void *dst, int64_t sites, int precision, hipStream_t s);
hipError_t launch_unpack(const void *src, void *dst, int64_t sites, int precision, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);
// Streaming probe of an access shape: per wavefront tile, in_a (and in_b)
// 16-byte chunks per lane read, out chunks per lane written. False for a
// shape it does not implement.
bool stream_shape_supported(int in_a, int in_b, int out);
hipError_t launch_stream_shape(const void *a, const void *b, void *c, int64_t tiles, int in_a, int in_b, int out,
                               int waves_per_cu, int tile_order, hipStream_t s);
// Adjoint: stage 1 writes per-workgroup partial sums of db into ws (72 x
// bwd_groups doubles, in 32-byte quads of components), stage 2 reduces them in a fixed order
// through run sums stored after them; bwd_workspace_doubles is the total.
int64_t bwd_groups(int64_t sites, int precision);
int64_t bwd_workspace_doubles(int64_t sites, int precision);
int bwd_block_threads();
hipError_t launch_bwd(const void *a, const void *b, const void *dc, void *da, double *db, int64_t sites,
                      int precision, double *ws, hipStream_t s);
hipError_t launch_bwd_zero(double *db, hipStream_t s);
// Bytes of the library-owned adjoint workspace (one static device array per
// device) and its device address on the current device, looked up on the
// first call per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t bwd_scratch(double **ptr);

} // namespace su3
