// su3_bwd.hip -- adjoint of the SU(3) link multiply on gfx950.
//
// For the real loss Re sum conj(dC) * C with C[s][j] = A[s][j] B[j]:
//   dA[s][j] = dC[s][j] B[j]^H             (per site, streamed like the forward)
//   dB[j]    = sum_s A[s][j]^H dC[s][j]     (a sum over every site)
// The paper has no adjoint; these are the two contractions of its product.
//
// Stage 1 (bwd_tiles). A lane owns one row (3 complex) of a link at a time,
// 48 B in FP64 and 24 B in FP32, and a wavefront streams steps of 3 chunks
// per lane of dC and A (whole 1 KiB global runs; one 64-row tile in FP64,
// two in FP32), transposed to one row per lane through LDS. Per row k of
// link j it writes row k of dA and adds conj(A(k, m)) dC(k, l) (m, l = 0..2)
// to 18 FP64 accumulators. The tiles of a wavefront are spaced a multiple of
// 3 tiles (192 rows, a multiple of the 12 rows of a site) apart, so a lane
// keeps one row position, hence one link and one accumulator set, on every
// tile. A workgroup of 3 wavefronts takes kSteps steps each; in FP64 the
// workgroups are taken in batches of 256 and step k of every workgroup of a
// batch lies in one contiguous block (phase striping), which keeps the
// workgroups that run together on one contiguous front.
// At the end the lanes' accumulators are summed in a fixed order: per row
// position within the wavefront (lanes in increasing order), then per link
// over the workgroup's wavefronts and the link's three rows. Each workgroup
// writes one 4x3x3 complex FP64 partial. Partials are stored in quads of
// components: quad u = q / 4 holds, for every workgroup g, the 4 doubles of
// components 4u .. 4u+3 at 4 (u * groups + g), so each workgroup writes 18
// whole 32-byte sectors rather than 72 scattered doubles (a scattered
// 8-byte store costs a whole sector of HBM writes).
// Stage 2 reduces the partials of each of the 72 real components in two
// fixed-order levels: bwd_chunk_sums adds runs of kChunk consecutive partials
// of a quad's 4 components (8 per thread, then a shuffle tree per wavefront
// and the wavefronts in order), bwd_reduce adds the run sums, stored
// component-major (one wavefront per component: a strided loop, then a
// shuffle tree). With a single run per component the first level writes dB
// itself and the second is not launched. Both levels keep every load of a
// thread in flight at once, so stage 2 costs a few microseconds at any
// lattice size.
// The number of workgroups of every stage depends only on the number of sites
// and the form, so the rounding sequence, and every bit of dB, is the same on
// every run and every device. No atomics.
#include "su3_internal.hpp"

namespace su3 {

constexpr int kBwdWaves = 3;                 // wavefronts per workgroup
constexpr int kBwdThreads = 64 * kBwdWaves;
// Steps per wavefront and resident wavefronts per CU for stage 1 (0: as many
// as fit), from sweeps at L=32 over 1 to 128 steps, caps of 6, 9 and 12
// wavefronts and batches of 32 to 3072 workgroups (or none). More steps
// amortise the closing reduction and cut the partials stage 2 reads; fewer
// shorten the drain at the end of the grid and keep the workgroups from
// drifting apart in memory.
#ifndef SU3_BWD_TILES_F64
#define SU3_BWD_TILES_F64 4
#endif
#ifndef SU3_BWD_TILES_F32
#define SU3_BWD_TILES_F32 2
#endif
#ifndef SU3_BWD_WAVES_F64
#define SU3_BWD_WAVES_F64 9
#endif
#ifndef SU3_BWD_WAVES_F32
#define SU3_BWD_WAVES_F32 12
#endif
// Tile order of stage 1: 0, workgroup g takes tile group g; 1, the
// XCD-contiguous order of the forward kernels (xcd_order).
#ifndef SU3_BWD_XCD_ORDER
#define SU3_BWD_XCD_ORDER 0
#endif
// Phase striping of stage 1 (0: off): the workgroups are taken in batches
// of kBatch, and step k of every workgroup of a batch lies in one
// contiguous block of the batch's tiles, so the workgroups that run at the
// same time stream one contiguous front instead of each its own run.
#ifndef SU3_BWD_BATCH_F64
#define SU3_BWD_BATCH_F64 256
#endif
#ifndef SU3_BWD_BATCH_F32
#define SU3_BWD_BATCH_F32 0
#endif

// The two forms: kSub 64-row tiles per step (3 chunks per lane of each
// array), kSteps steps per wavefront, phase-striping batch kBatch.
struct BwdF64 {
    typedef double S;
    static constexpr int kSub = 1, kSteps = SU3_BWD_TILES_F64, kBatch = SU3_BWD_BATCH_F64;
};
struct BwdF32 {
    typedef float S;
    static constexpr int kSub = 2, kSteps = SU3_BWD_TILES_F32, kBatch = SU3_BWD_BATCH_F32;
};
constexpr int kRowsPerSite = 12;

// Stage 2, first level: threads per workgroup and partials per thread.
#ifndef SU3_BWD_CHUNK_THREADS
#define SU3_BWD_CHUNK_THREADS 256
#endif
#ifndef SU3_BWD_CHUNK_LOADS
#define SU3_BWD_CHUNK_LOADS 8
#endif
constexpr int kChunkThreads = SU3_BWD_CHUNK_THREADS;
constexpr int kChunkLoads = SU3_BWD_CHUNK_LOADS;
constexpr int64_t kChunk = (int64_t)kChunkThreads * kChunkLoads;

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync_bwd()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row `lane` of sub-tile q of a staged step, as 6 interleaved re/im values.
__device__ __forceinline__ void row_from_stage(const u4 *st, int q, int lane, double (&v)[6])
{
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const d2 w = __builtin_bit_cast(d2, st[192 * q + 3 * lane + e]);
        v[2 * e] = w.x;
        v[2 * e + 1] = w.y;
    }
}
__device__ __forceinline__ void row_from_stage(const u4 *st, int q, int lane, float (&v)[6])
{
    const f2 *p = reinterpret_cast<const f2 *>(st) + 192 * q + 3 * lane;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const f2 w = p[e];
        v[2 * e] = w.x;
        v[2 * e + 1] = w.y;
    }
}
__device__ __forceinline__ void row_to_stage(u4 *st, int q, int lane, const double (&v)[6])
{
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const d2 w = {v[2 * e], v[2 * e + 1]};
        st[192 * q + 3 * lane + e] = __builtin_bit_cast(u4, w);
    }
}
__device__ __forceinline__ void row_to_stage(u4 *st, int q, int lane, const float (&v)[6])
{
    f2 *p = reinterpret_cast<f2 *>(st) + 192 * q + 3 * lane;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const f2 w = {v[2 * e], v[2 * e + 1]};
        p[e] = w;
    }
}

template <class F>
__global__ __launch_bounds__(kBwdThreads) void bwd_tiles(const u4 *__restrict__ a, const typename F::S *__restrict__ b,
                                                         const u4 *__restrict__ dc, u4 *__restrict__ da,
                                                         double *__restrict__ ws, int64_t rows, int64_t groups)
{
    typedef typename F::S S;
    constexpr int kSub = F::kSub;                     // 64-row tiles per step
    constexpr int kSteps = F::kSteps;
    constexpr int CT = 64 * 6 * (int)sizeof(S) / 16;  // chunks per 64-row tile: 192 or 96
    constexpr int kStageBytes = 2 * 3 * 64 * 16;      // a and dC, 3 chunks per lane each
    constexpr int kRedBytes = 64 * 19 * 8;            // 18 accumulators per lane, padded
    constexpr int kBytes = kStageBytes > kRedBytes ? kStageBytes : kRedBytes;
    // per-wavefront LDS: step staging in the loop, reduction after it
    __shared__ __attribute__((aligned(16))) char tilebuf[kBwdWaves][kBytes];
    __shared__ double rowsum[kBwdWaves][kRowsPerSite * 18];
    __shared__ S bsh[72];

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    u4 *stg = reinterpret_cast<u4 *>(tilebuf[wv]);    // dC at [0, 192), A at [192, 384)
    double *red = reinterpret_cast<double *>(tilebuf[wv]);
    // this workgroup's tile group; its partial goes to slot grp
    const int64_t grp = SU3_BWD_XCD_ORDER ? xcd_order(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    // the wavefront's first 64-row tile t0; it takes t0 + D i for
    // i < kSub * kSteps (D a multiple of 3)
    constexpr int kPer = kBwdWaves * kSub * kSteps;   // tiles per workgroup
    int64_t t0, D;
    if constexpr (F::kBatch > 0) {
        constexpr int kB = F::kBatch;
        const int64_t bt = grp / kB, lam = grp - bt * kB;
        const int64_t nb = groups - bt * kB < kB ? groups - bt * kB : (int64_t)kB;
        t0 = bt * kPer * kB + kBwdWaves * lam + wv;
        D = kBwdWaves * nb;
    } else {
        t0 = grp * kPer + wv;
        D = kBwdWaves;
    }
    const int64_t nchunks = rows * 6 * (int64_t)sizeof(S) / 16;

    if (threadIdx.x < 72)
        bsh[threadIdx.x] = b[threadIdx.x];
    __syncthreads();

    const int pos = (int)((t0 * 64 + lane) % kRowsPerSite);   // row position in the site
    const int j = pos / 3;                                     // its link
    S br[9], bi[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        br[q] = bsh[2 * (9 * j + q)];
        bi[q] = bsh[2 * (9 * j + q) + 1];
    }
    double acc[18];
#pragma unroll
    for (int v = 0; v < 18; ++v)
        acc[v] = 0.0;

    // Global chunk of step-chunk c (c = 64 i + lane, i < 3) of the step that
    // starts at tile ts: sub-tile c / CT, chunk c mod CT of it.
    auto gchunk = [&](int64_t ts, int i) -> int64_t {
        const int c = 64 * i + lane, q = c / CT;
        return (ts + D * q) * CT + (c - q * CT);
    };
    // Step loads: chunks past the end re-read the last chunk (in bounds;
    // those rows store nothing and add nothing). The loads of the next step
    // are issued as soon as the current step sits in LDS, so they are in
    // flight while the current step is computed and stored.
    u4 va[3], vg[3];
    auto load_step = [&](int64_t ts) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int64_t g = gchunk(ts, i);
            const int64_t gc = g < nchunks ? g : nchunks - 1;
            vg[i] = ld_stream(dc + gc);
            va[i] = ld_stream(a + gc);
        }
    };
    if (t0 * 64 < rows)
        load_step(t0);
    for (int k = 0; k < kSteps; ++k) {
        const int64_t ts = t0 + D * kSub * k;   // the step's first tile
        if (ts * 64 >= rows)
            break;                              // wave-uniform
        // every row of the step's last tile is in the lattice
        const bool whole = (ts + D * (kSub - 1) + 1) * 64 <= rows;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            stg[64 * i + lane] = vg[i];
            stg[192 + 64 * i + lane] = va[i];
        }
        wave_sync_bwd();
        if (k + 1 < kSteps && (ts + D * kSub) * 64 < rows)
            load_step(ts + D * kSub);
        S o[kSub][6];
#pragma unroll
        for (int q = 0; q < kSub; ++q) {
            S g[6], x[6];     // interleaved re/im of dC and A row `lane` of sub-tile q
            row_from_stage(stg, q, lane, g);
            row_from_stage(stg + 192, q, lane, x);
            // dA(k, m) = sum_l dC(k, l) conj(B(m, l))
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                S re = 0, im = 0;
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    cmac(re, im, g[2 * l], g[2 * l + 1], br[3 * m + l], -bi[3 * m + l]);
                o[q][2 * m] = re;
                o[q][2 * m + 1] = im;
            }
            // dB(m, l) += conj(A(k, m)) dC(k, l), in FP64; rows past the end
            // of the lattice hold re-read data and add nothing
            const bool live = whole || (ts + D * q) * 64 + lane < rows;
#pragma unroll
            for (int h = 0; h < 6; ++h)
                x[h] = live ? x[h] : S(0);
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    cmac(acc[6 * m + 2 * l], acc[6 * m + 2 * l + 1], (double)x[2 * m], -(double)x[2 * m + 1],
                         (double)g[2 * l], (double)g[2 * l + 1]);
        }
        wave_sync_bwd();
#pragma unroll
        for (int q = 0; q < kSub; ++q)
            row_to_stage(stg, q, lane, o[q]);
        wave_sync_bwd();
        // store the dA step as 3 whole-wavefront runs, guarded past the end
        u4 w[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            w[i] = stg[64 * i + lane];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int64_t g = gchunk(ts, i);
            if (whole || g < nchunks)
                st_stream(da + g, w[i]);
        }
        wave_sync_bwd();
    }

    // ---- fixed-order reduction --------------------------------------------
    // The lanes' 18 accumulators go to LDS (row stride 19 doubles); then the
    // sums of the 12 row positions r are formed: output 18*r + e adds the
    // lanes at position r, (r - base) mod 12 and every 12th lane after it,
    // in increasing order. Every load of a lane is issued before the first
    // add (fixed trip counts; a lane index past 63 reads lane 63 and adds an
    // exact zero instead).
    const int base = (int)((t0 * 64) % kRowsPerSite);
    constexpr int kLanesPerPos = (64 + kRowsPerSite - 1) / kRowsPerSite;   // 6
    constexpr int kOut = kRowsPerSite * 18;                                 // 216
#pragma unroll
    for (int v = 0; v < 18; ++v)
        red[lane * 19 + v] = acc[v];
    wave_sync_bwd();
#pragma unroll
    for (int it = 0; it < (kOut + 63) / 64; ++it) {
        const int o3 = lane + 64 * it;
        if (o3 < kOut) {
            const int r = o3 / 18, e = o3 % 18;
            const int l0 = ((r - base) % kRowsPerSite + kRowsPerSite) % kRowsPerSite;
            double x[kLanesPerPos];
#pragma unroll
            for (int i = 0; i < kLanesPerPos; ++i) {
                const int l = l0 + kRowsPerSite * i;
                const double y = red[(l < 64 ? l : 63) * 19 + e];
                x[i] = l < 64 ? y : 0.0;
            }
            double sum = x[0];
#pragma unroll
            for (int i = 1; i < kLanesPerPos; ++i)
                sum += x[i];
            rowsum[wv][o3] = sum;
        }
    }
    __syncthreads();
    // workgroup partial of component q = 18*j + e: wavefronts in order, then
    // the link's three rows in order
    if (threadIdx.x < 72) {
        const int jj = threadIdx.x / 18, e = threadIdx.x % 18;
        double sum = 0.0;
        for (int w2 = 0; w2 < kBwdWaves; ++w2)
            for (int r = 3 * jj; r < 3 * jj + 3; ++r)
                sum += rowsum[w2][18 * r + e];
        ws[4 * ((int64_t)(threadIdx.x >> 2) * groups + grp) + (threadIdx.x & 3)] = sum;
    }
}

// grid = (chunks, 18): workgroup (c, u) adds partials c*kChunk .. c*kChunk +
// kChunk - 1 of the 4 components of quad u and writes run sums
// ws2[q * chunks + c] for q = 4u .. 4u+3. Thread t adds partials t,
// t + kChunkThreads, ... in order; then, per component, a binary tree across
// the lanes of each wavefront pairs lane t with t + w for w = 32, 16, ..., 1,
// and the wavefront sums are added in wavefront order.
__global__ __launch_bounds__(kChunkThreads) void bwd_chunk_sums(const double *__restrict__ ws,
                                                                double *__restrict__ ws2, int64_t groups,
                                                                int64_t chunks)
{
    constexpr int kW = kChunkThreads / 64;
    __shared__ double red[4][kW];
    const int64_t c = blockIdx.x;
    const d2 *src = reinterpret_cast<const d2 *>(ws + 4 * (int64_t)blockIdx.y * groups);
    d2 v[kChunkLoads][2];
#pragma unroll
    for (int i = 0; i < kChunkLoads; ++i) {
        const int64_t g = c * kChunk + (int64_t)kChunkThreads * i + threadIdx.x;
        const d2 z = {0.0, 0.0};
        v[i][0] = g < groups ? src[2 * g] : z;
        v[i][1] = g < groups ? src[2 * g + 1] : z;
    }
    double sum[4] = {v[0][0].x, v[0][0].y, v[0][1].x, v[0][1].y};
#pragma unroll
    for (int i = 1; i < kChunkLoads; ++i) {
        sum[0] += v[i][0].x;
        sum[1] += v[i][0].y;
        sum[2] += v[i][1].x;
        sum[3] += v[i][1].y;
    }
#pragma unroll
    for (int w = 32; w > 0; w >>= 1)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            sum[e] += __shfl_down(sum[e], w, 64);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (kW == 1) {
        // after the tree lane 0 holds the four sums
        if (lane == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ws2[(int64_t)(4 * blockIdx.y + e) * chunks + c] = sum[e];
        }
        return;
    }
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            red[e][wv] = sum[e];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = red[threadIdx.x][0];
#pragma unroll
        for (int w2 = 1; w2 < kW; ++w2)
            t += red[threadIdx.x][w2];
        ws2[(int64_t)(4 * blockIdx.y + threadIdx.x) * chunks + c] = t;
    }
}

// grid = 72 workgroups of one wavefront, one per real component of dB; the
// input holds `groups` values per component, component-major (the run sums
// of stage 2a). Lane t adds values t, t + 64, ... in order, then a binary
// tree across the lanes pairs lane t with t + w for w = 32, 16, ..., 1.
__global__ __launch_bounds__(64) void bwd_reduce(const double *__restrict__ ws, double *__restrict__ db,
                                                 int64_t groups)
{
    const int q = blockIdx.x;
    double sum = 0.0;
    for (int64_t g = threadIdx.x; g < groups; g += 64)
        sum += ws[(int64_t)q * groups + g];
#pragma unroll
    for (int w = 32; w > 0; w >>= 1)
        sum += __shfl_down(sum, w, 64);
    if (threadIdx.x == 0)
        db[q] = sum;
}
constexpr int kReduceThreads = 64;

// Workgroups of stage 1 for `sites` (a function of the size and form only).
int64_t bwd_groups(int64_t sites, int precision)
{
    const int64_t tiles = (sites * kRowsPerSite + 63) / 64;
    const int64_t per = (int64_t)kBwdWaves * (precision == 0 ? BwdF64::kSub * BwdF64::kSteps
                                                              : BwdF32::kSub * BwdF32::kSteps);
    return (tiles + per - 1) / per;
}

static int64_t bwd_chunks(int64_t groups) { return (groups + kChunk - 1) / kChunk; }

int64_t bwd_workspace_doubles(int64_t sites, int precision)
{
    const int64_t groups = bwd_groups(sites, precision);
    return 72 * (groups + bwd_chunks(groups));
}

int bwd_block_threads() { return kBwdThreads; }

hipError_t launch_bwd(const void *a, const void *b, const void *dc, void *da, double *db, int64_t sites,
                      int precision, double *ws, hipStream_t s)
{
    static std::atomic<int> pad64[kMaxDevices], pad32[kMaxDevices];
    const int64_t groups = bwd_groups(sites, precision), chunks = bwd_chunks(groups);
    double *ws2 = ws + 72 * groups;
    hipError_t e;
    if (precision == 0) {
        const size_t pad =
            occupancy_pad(reinterpret_cast<const void *>(bwd_tiles<BwdF64>), SU3_BWD_WAVES_F64, kBwdThreads, pad64);
        e = launch_k(bwd_tiles<BwdF64>, dim3((unsigned)groups), dim3(kBwdThreads), s, pad, (const u4 *)a,
                     (const double *)b, (const u4 *)dc, (u4 *)da, ws, sites * kRowsPerSite, groups);
    } else {
        const size_t pad =
            occupancy_pad(reinterpret_cast<const void *>(bwd_tiles<BwdF32>), SU3_BWD_WAVES_F32, kBwdThreads, pad32);
        e = launch_k(bwd_tiles<BwdF32>, dim3((unsigned)groups), dim3(kBwdThreads), s, pad, (const u4 *)a,
                     (const float *)b, (const u4 *)dc, (u4 *)da, ws, sites * kRowsPerSite, groups);
    }
    if (e != hipSuccess)
        return e;
    // With a single run per component (groups <= kChunk) the run sums are dB
    // itself, component-major: the first level writes them to db directly.
    if (chunks == 1)
        return launch_k(bwd_chunk_sums, dim3(1, 18), dim3(kChunkThreads), s, 0, (const double *)ws, db, groups,
                        (int64_t)1);
    e = launch_k(bwd_chunk_sums, dim3((unsigned)chunks, 18), dim3(kChunkThreads), s, 0, (const double *)ws, ws2,
                 groups, chunks);
    if (e != hipSuccess)
        return e;
    return launch_k(bwd_reduce, dim3(72), dim3(kReduceThreads), s, 0, (const double *)ws2, db, chunks);
}

// An empty lattice has dB = 0: the second stage over zero partials writes
// zeros (a kernel rather than a memset, so the call is safe to capture).
hipError_t launch_bwd_zero(double *db, hipStream_t s)
{
    return launch_k(bwd_reduce, dim3(72), dim3(kReduceThreads), s, 0, (const double *)nullptr, db, (int64_t)0);
}

// ---- the library-owned workspace of su3_mult_nn_bwd_noalloc ---------------
// A fixed device array (each device the library runs on holds its own copy
// until the process ends). Its name is only a host-side handle: host code
// uses the device address that hipGetSymbolAddress returns for the current
// device, kept per device in scratch_ptr.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
static std::atomic<double *> scratch_ptr[kMaxDevices];

hipError_t bwd_scratch(double **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    double *p = scratch_ptr[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        // racing first calls on one device get the same address
        e = hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (p == nullptr)
            return hipErrorInvalidSymbol;
        scratch_ptr[dev].store(p, std::memory_order_release);
    }
    *ptr = p;
    return hipSuccess;
}

} // namespace su3
