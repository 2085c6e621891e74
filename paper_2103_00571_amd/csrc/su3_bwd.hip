// su3_bwd.hip -- adjoint of the SU(3) link multiply on gfx950.
//
// For the real loss Re sum conj(dC) * C with C[s][j] = A[s][j] B[j]:
//   dA[s][j] = dC[s][j] B[j]^H             (per site, streamed like the forward)
//   dB[j]    = sum_s A[s][j]^H dC[s][j]     (a sum over every site)
// The paper has no adjoint; these are the two contractions of its product.
//
// Stage 1 (bwd_rows): thread per output row (j, k), the same fixed-position,
// grid-stride mapping as the forward kernel. Each iteration reads row k of
// dC[s][j] and of A[s][j], writes row k of dA, and adds
// conj(A(k, m)) dC(k, l) to nine complex FP64 accumulators (the thread's k
// and j never change). At the end the workgroup adds its threads' partials in
// a fixed thread order through LDS and writes one 4x3x3 complex FP64 partial.
// Stage 2 (bwd_reduce): one workgroup per output component sums the G
// partials in a fixed strided order and then a fixed binary tree.
// G depends only on the number of sites, so the rounding sequence, and hence
// every bit of dB, is the same on every run and every device. No atomics.
#include "su3_internal.hpp"

namespace su3 {

template <typename S>
struct RowIO;

template <>
struct RowIO<double> {
    typedef d2 V;
};
template <>
struct RowIO<float> {
    typedef f2 V;
};

template <typename S>
__global__ __launch_bounds__(kBlock) void bwd_rows(const typename RowIO<S>::V *__restrict__ a,
                                                   const S *__restrict__ b,
                                                   const typename RowIO<S>::V *__restrict__ dc,
                                                   typename RowIO<S>::V *__restrict__ da, double *__restrict__ ws,
                                                   int64_t rows)
{
    typedef typename RowIO<S>::V V;
    __shared__ double part[kBlock][19]; // 18 used; odd stride spreads banks

    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    const int j = (int)((first % 12) / 3);
    S br[9], bi[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        br[q] = b[2 * (9 * j + q)];
        bi[q] = b[2 * (9 * j + q) + 1];
    }
    double accr[9], acci[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        accr[q] = 0.0;
        acci[q] = 0.0;
    }

    for (int64_t r = first; r < rows; r += step) {
        V g[3], x[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            g[l] = ld_stream(dc + 3 * r + l);
            x[l] = ld_stream(a + 3 * r + l);
        }
        // dA(k, m) = sum_l dC(k, l) conj(B(m, l))
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            S re = 0, im = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l)
                cmac(re, im, g[l].x, g[l].y, br[3 * m + l], -bi[3 * m + l]);
            V o = {re, im};
            st_stream(da + 3 * r + m, o);
        }
        // dB(m, l) += conj(A(k, m)) dC(k, l), in FP64
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int l = 0; l < 3; ++l)
                cmac(accr[3 * m + l], acci[3 * m + l], (double)x[m].x, -(double)x[m].y, (double)g[l].x,
                     (double)g[l].y);
    }

#pragma unroll
    for (int q = 0; q < 9; ++q) {
        part[threadIdx.x][2 * q] = accr[q];
        part[threadIdx.x][2 * q + 1] = acci[q];
    }
    __syncthreads();
    if (threadIdx.x < 72) {
        // component q = jj*18 + e of this workgroup's partial: the threads
        // whose link is jj, added in increasing thread order
        const int jj = threadIdx.x / 18, e = threadIdx.x % 18;
        const int64_t base = (int64_t)blockIdx.x * kBlock;
        double sum = 0.0;
        for (int t = 0; t < kBlock; ++t)
            if ((int)(((base + t) % 12) / 3) == jj)
                sum += part[t][e];
        ws[(int64_t)blockIdx.x * 72 + threadIdx.x] = sum;
    }
}

// grid = 72 workgroups, one per real component of dB
__global__ __launch_bounds__(kBlock) void bwd_reduce(const double *__restrict__ ws, double *__restrict__ db,
                                                     int64_t groups)
{
    __shared__ double red[kBlock];
    const int q = blockIdx.x;
    double sum = 0.0;
    for (int64_t g = threadIdx.x; g < groups; g += kBlock)
        sum += ws[g * 72 + q];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        db[q] = red[0];
}

hipError_t launch_bwd(const void *a, const void *b, const void *dc, void *da, double *db, int64_t sites,
                      int precision, double *ws, int64_t groups, hipStream_t s)
{
    hipError_t e;
    if (precision == 0)
        e = launch_k(bwd_rows<double>, dim3((unsigned)groups), dim3(kBlock), s, 0, (const d2 *)a, (const double *)b,
                     (const d2 *)dc, (d2 *)da, ws, sites * 12);
    else
        e = launch_k(bwd_rows<float>, dim3((unsigned)groups), dim3(kBlock), s, 0, (const f2 *)a, (const float *)b,
                     (const f2 *)dc, (f2 *)da, ws, sites * 12);
    if (e != hipSuccess)
        return e;
    return launch_k(bwd_reduce, dim3(72), dim3(kBlock), s, 0, (const double *)ws, db, groups);
}

// An empty lattice has dB = 0: the second stage over zero partials writes
// zeros (a kernel rather than a memset, so the call is safe to capture).
hipError_t launch_bwd_zero(double *db, hipStream_t s)
{
    return launch_k(bwd_reduce, dim3(72), dim3(kBlock), s, 0, (const double *)nullptr, db, (int64_t)0);
}

} // namespace su3
