// su3_matvec.hip -- SU(3) matrix times colour vector over the lattice on
// gfx950: w[s][j] = a[s][j] v[s] for the four links of every site and the
// site's own colour vector (the matrix-vector building block the SU3_Bench
// paper names beside the matrix-matrix product, section Introduction).
//
// Per site the product reads a (576 B FP64 / 288 B FP32) and v (48 / 24 B)
// and writes w (192 / 96 B): 0.35 flop per byte in FP64, more strongly
// HBM-bound than the matrix-matrix product.
//
// A wavefront handles a tile of 64 units (FP64: one link; FP32: two links of
// one site), so 16 (FP64) or 32 (FP32) sites. It loads the tile's a with
// whole 1 KiB runs and the tile's 768 B of v as 8-byte words (a site's
// vector is only 8-byte aligned in FP32), transposes both through LDS to one
// unit per lane, writes the unit's output (48 B) back through LDS and stores
// it with whole 1 KiB runs. One tile per wavefront; the grid covers the
// lattice once.
#include "su3_internal.hpp"

// Resident wavefronts per CU: each carries 9.75 KiB of loads in flight; 9
// measured best at L=48 in the XCD-contiguous tile order (6.61 TB/s FP64).
#ifndef SU3_WAVES_MATVEC
#define SU3_WAVES_MATVEC 9
#endif

namespace su3 {

constexpr int kMvBlock = 64;    // one wavefront per workgroup

__device__ __forceinline__ void wave_sync_mv()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename S>
__global__ __launch_bounds__(kMvBlock) void mat_vec(const u4 *__restrict__ a, const uint64_t *__restrict__ v,
                                                    u4 *__restrict__ w, int64_t sites)
{
    typedef S SV __attribute__((ext_vector_type(16 / sizeof(S))));
    constexpr int PV = 16 / sizeof(S);           // scalars per 16-byte chunk
    constexpr int R = sizeof(S) == 8 ? 1 : 2;    // links per unit
    constexpr int kUnitsPerSite = 4 / R;
    constexpr int kWordsPerSite = 6 * (int)sizeof(S) / 8;   // 8-byte words of one v
    __shared__ u4 stage[64 * 9];
    __shared__ uint64_t vst[96];

    const int lane = threadIdx.x;
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t units = sites * kUnitsPerSite;
    const int64_t na = units * 9, nv = sites * kWordsPerSite, nw = units * 3;
    const bool whole = (t + 1) * 64 <= units;

    // loads: indices past the end re-read the last element (never used)
    u4 va[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int64_t g = t * 576 + 64 * i + lane;
        va[i] = ld_stream(a + (g < na ? g : na - 1));
    }
    uint64_t vv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t g = t * 96 + 64 * h + lane;
        vv[h] = ld_stream(v + (g < nv ? g : nv - 1));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        stage[64 * i + lane] = va[i];
    vst[lane] = vv[0];
    if (lane < 32)
        vst[64 + lane] = vv[1];
    wave_sync_mv();

    // the lane's unit: R links of site lane / kUnitsPerSite of the tile
    S x[18 * R], vec[6], o[6 * R];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const SV c = __builtin_bit_cast(SV, stage[9 * lane + i]);
#pragma unroll
        for (int e = 0; e < PV; ++e)
            x[PV * i + e] = c[e];
    }
    const int site = lane / kUnitsPerSite;
#pragma unroll
    for (int q = 0; q < kWordsPerSite; ++q) {
        typedef S SW __attribute__((ext_vector_type(8 / sizeof(S))));
        const SW c = __builtin_bit_cast(SW, vst[kWordsPerSite * site + q]);
#pragma unroll
        for (int e = 0; e < (int)(8 / sizeof(S)); ++e)
            vec[(8 / sizeof(S)) * q + e] = c[e];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            S re = 0, im = 0;
#pragma unroll
            for (int m = 0; m < 3; ++m)
                cmac(re, im, x[18 * r + 2 * (3 * k + m)], x[18 * r + 2 * (3 * k + m) + 1], vec[2 * m], vec[2 * m + 1]);
            o[6 * r + 2 * k] = re;
            o[6 * r + 2 * k + 1] = im;
        }
    wave_sync_mv();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        SV c;
#pragma unroll
        for (int e = 0; e < PV; ++e)
            c[e] = o[PV * i + e];
        stage[3 * lane + i] = __builtin_bit_cast(u4, c);
    }
    wave_sync_mv();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int64_t g = t * 192 + 64 * i + lane;
        if (whole || g < nw)
            st_stream(w + g, stage[64 * i + lane]);
    }
}

int64_t mat_vec_grid(int precision, int64_t sites)
{
    const int64_t units = sites * (precision == 0 ? 4 : 2);
    return (units + 63) / 64;
}

hipError_t launch_mat_vec(const void *a, const void *v, void *w, int64_t sites, int precision, hipStream_t s)
{
    static std::atomic<int> pad64[kMaxDevices], pad32[kMaxDevices];
    const dim3 grid((unsigned)mat_vec_grid(precision, sites));
    if (precision == 0) {
        const size_t pad =
            occupancy_pad(reinterpret_cast<const void *>(mat_vec<double>), SU3_WAVES_MATVEC, kMvBlock, pad64);
        return launch_k(mat_vec<double>, grid, dim3(kMvBlock), s, pad, (const u4 *)a, (const uint64_t *)v, (u4 *)w,
                        sites);
    }
    const size_t pad = occupancy_pad(reinterpret_cast<const void *>(mat_vec<float>), SU3_WAVES_MATVEC, kMvBlock, pad32);
    return launch_k(mat_vec<float>, grid, dim3(kMvBlock), s, pad, (const u4 *)a, (const uint64_t *)v, (u4 *)w, sites);
}

} // namespace su3
