// su3_bwd.hip -- adjoint of the SU(3) link multiply on gfx950.
//
// For the real loss Re sum conj(dC) * C with C[s][j] = A[s][j] B[j]:
//   dA[s][j] = dC[s][j] B[j]^H             (per site, streamed like the forward)
//   dB[j]    = sum_s A[s][j]^H dC[s][j]     (a sum over every site)
// The paper has no adjoint; these are the two contractions of its product.
//
// Stage 1 (bwd_tiles). A thread owns one unit of output rows (FP64: one row,
// FP32: two rows), as in the forward kernel, and a wavefront streams tiles of
// 64 units: whole 1 KiB global runs of dC and A, transposed to one unit per
// lane through LDS. Per row k of link j it writes row k of dA and adds
// conj(A(k, m)) dC(k, l) (m, l = 0..2) to FP64 accumulators. A wavefront
// takes kTiles tiles spaced 3 tiles apart, so a lane keeps the same row
// position (and link) on every tile and its accumulators stay valid; a
// workgroup of 3 wavefronts covers 3*kTiles consecutive tiles.
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
// of a quad's 4 components (8 per thread, then a binary tree per component),
// bwd_reduce adds the run sums, stored component-major (one wavefront per
// component: a strided loop, then a binary tree across the lanes). Both
// levels keep every load of a thread in flight at once, so stage 2 costs a
// few microseconds at any lattice size.
// The number of workgroups of every stage depends only on the number of sites
// and the form, so the rounding sequence, and every bit of dB, is the same on
// every run and every device. No atomics.
#include "su3_internal.hpp"

namespace su3 {

constexpr int kBwdWaves = 3;                 // wavefronts per workgroup
constexpr int kBwdThreads = 64 * kBwdWaves;
// Tiles per wavefront and resident wavefronts per CU for stage 1 (0: as many
// as fit), measured at L=32 over 1, 2, 3, 4, 6, 8 and 16 tiles and 3, 6, 9 or
// 12 wavefronts.
// More tiles per wavefront amortise the closing reduction; fewer shorten the
// drain at the end of the grid.
#ifndef SU3_BWD_TILES_F64
#define SU3_BWD_TILES_F64 4
#endif
#ifndef SU3_BWD_TILES_F32
#define SU3_BWD_TILES_F32 4
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

// FP64: unit = one row (3 complex, 48 B); 12 units per site.
struct BwdF64 {
    typedef double S;
    static constexpr int kRows = 1, kUnitsPerSite = 12, kTiles = SU3_BWD_TILES_F64;
};
// FP32: unit = two rows (6 complex float, 48 B); 6 units per site.
struct BwdF32 {
    typedef float S;
    static constexpr int kRows = 2, kUnitsPerSite = 6, kTiles = SU3_BWD_TILES_F32;
};

// Stage 2, first level: partials per workgroup.
constexpr int kChunkLoads = 8;
constexpr int64_t kChunk = (int64_t)kBlock * kChunkLoads;

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync_bwd()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class F>
__global__ __launch_bounds__(kBwdThreads) void bwd_tiles(const u4 *__restrict__ a, const typename F::S *__restrict__ b,
                                                         const u4 *__restrict__ dc, u4 *__restrict__ da,
                                                         double *__restrict__ ws, int64_t units, int64_t groups)
{
    typedef typename F::S S;
    typedef S SV __attribute__((ext_vector_type(16 / sizeof(S))));
    constexpr int PV = 16 / sizeof(S);        // scalars per 16-byte chunk
    constexpr int R = F::kRows;
    constexpr int NV = 18 * R;                // accumulator doubles per lane
    constexpr int P = F::kUnitsPerSite;
    constexpr int kTiles = F::kTiles;
    constexpr int kStageBytes = 2 * 3 * 64 * 16;     // a and dC tiles
    constexpr int kRedBytes = 64 * 19 * 8;           // one row's 18 accumulators per lane, padded
    constexpr int kBytes = kStageBytes > kRedBytes ? kStageBytes : kRedBytes;
    // per-wavefront LDS: tile staging in the loop, reduction after it
    __shared__ __attribute__((aligned(16))) char tilebuf[kBwdWaves][kBytes];
    __shared__ double rowsum[kBwdWaves][12 * 18];
    __shared__ S bsh[72];

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    u4 *stage = reinterpret_cast<u4 *>(tilebuf[wv]);
    double *red = reinterpret_cast<double *>(tilebuf[wv]);
    // this workgroup's tile group; its partial goes to slot grp
    const int64_t grp = SU3_BWD_XCD_ORDER ? xcd_order(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t t0 = grp * kBwdWaves * kTiles + wv;
    const int64_t nchunks = units * 3;

    if (threadIdx.x < 72)
        bsh[threadIdx.x] = b[threadIdx.x];
    __syncthreads();

    const int pos = (int)((t0 * 64 + lane) % P);   // unit position in the site
    // row h of the unit is site row R*pos + h, which belongs to link (R*pos+h)/3
    S br[R][9], bi[R][9];
#pragma unroll
    for (int h = 0; h < R; ++h) {
        const int j = (R * pos + h) / 3;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            br[h][q] = bsh[2 * (9 * j + q)];
            bi[h][q] = bsh[2 * (9 * j + q) + 1];
        }
    }
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        acc[v] = 0.0;

    // Tile loads: chunk indices past the end re-read the last chunk (in
    // bounds; those lanes store nothing and add nothing). The loads of the
    // next tile are issued as soon as the current tile sits in LDS, so they
    // are in flight while the current tile is computed and stored.
    u4 va[3], vg[3];
    auto load_tile = [&](int64_t t) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int64_t g = t * 64 * 3 + lane + 64 * i;
            const int64_t gc = g < nchunks ? g : nchunks - 1;
            vg[i] = ld_stream(dc + gc);
            va[i] = ld_stream(a + gc);
        }
    };
    if (t0 * 64 < units)
        load_tile(t0);
    for (int k = 0; k < kTiles; ++k) {
        const int64_t t = t0 + (int64_t)kBwdWaves * k;
        if (t * 64 >= units)
            break;                                   // wave-uniform
        const bool whole = (t + 1) * 64 <= units;
        const int64_t g0 = t * 64 * 3 + lane;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            stage[64 * i + lane] = vg[i];
            stage[192 + 64 * i + lane] = va[i];
        }
        wave_sync_bwd();
        if (k + 1 < kTiles && (t + kBwdWaves) * 64 < units)
            load_tile(t + kBwdWaves);
        S g[6 * R], x[6 * R];   // interleaved re/im of the unit's R rows
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const SV wg = __builtin_bit_cast(SV, stage[3 * lane + i]);
            const SV wa = __builtin_bit_cast(SV, stage[192 + 3 * lane + i]);
#pragma unroll
            for (int e = 0; e < PV; ++e) {
                g[PV * i + e] = wg[e];
                x[PV * i + e] = wa[e];
            }
        }
        // dA(k, m) = sum_l dC(k, l) conj(B(m, l)), per row h of the unit
        S o[6 * R];
#pragma unroll
        for (int h = 0; h < R; ++h)
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                S re = 0, im = 0;
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    cmac(re, im, g[6 * h + 2 * l], g[6 * h + 2 * l + 1], br[h][3 * m + l], -bi[h][3 * m + l]);
                o[6 * h + 2 * m] = re;
                o[6 * h + 2 * m + 1] = im;
            }
        // dB(m, l) += conj(A(k, m)) dC(k, l), in FP64; lanes past the end of a
        // ragged last tile hold re-read data and add nothing
        const bool live = whole || t * 64 + lane < units;
#pragma unroll
        for (int h = 0; h < 6 * R; ++h)
            x[h] = live ? x[h] : S(0);
#pragma unroll
        for (int h = 0; h < R; ++h)
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    cmac(acc[18 * h + 6 * m + 2 * l], acc[18 * h + 6 * m + 2 * l + 1], (double)x[6 * h + 2 * m],
                         -(double)x[6 * h + 2 * m + 1], (double)g[6 * h + 2 * l], (double)g[6 * h + 2 * l + 1]);
        wave_sync_bwd();
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            SV w;
#pragma unroll
            for (int e = 0; e < PV; ++e)
                w[e] = o[PV * i + e];
            stage[3 * lane + i] = __builtin_bit_cast(u4, w);
        }
        wave_sync_bwd();
        store_runs<3>(da, stage, g0, lane, whole, nchunks);
        wave_sync_bwd();
    }

    // ---- fixed-order reduction --------------------------------------------
    // One pass per row h of the unit: the lanes' 18 accumulators of row h go
    // to LDS (row stride 19 doubles), then the row sums of the site rows
    // r = R*w + h (w = unit position 0..P-1) are formed: output 18*r + e adds
    // the lanes at position w, (w - base) mod P and every P-th lane after
    // it, in increasing order. Every load of a lane is issued before the
    // first add (fixed trip counts; a lane index past 63 reads lane 63 and
    // adds an exact zero instead).
    const int base = (int)((t0 * 64) % P);
    constexpr int kLanesPerPos = (64 + P - 1) / P;    // 6 (FP64) or 11 (FP32)
    constexpr int kPassOut = P * 18;                  // outputs per pass: 216 / R
#pragma unroll
    for (int h = 0; h < R; ++h) {
#pragma unroll
        for (int v = 0; v < 18; ++v)
            red[lane * 19 + v] = acc[18 * h + v];
        wave_sync_bwd();
#pragma unroll
        for (int it = 0; it < (kPassOut + 63) / 64; ++it) {
            const int o3 = lane + 64 * it;
            if (o3 < kPassOut) {
                const int w = o3 / 18, e = o3 % 18;
                const int l0 = ((w - base) % P + P) % P;
                double x[kLanesPerPos];
#pragma unroll
                for (int i = 0; i < kLanesPerPos; ++i) {
                    const int l = l0 + P * i;
                    const double y = red[(l < 64 ? l : 63) * 19 + e];
                    x[i] = l < 64 ? y : 0.0;
                }
                double sum = x[0];
#pragma unroll
                for (int i = 1; i < kLanesPerPos; ++i)
                    sum += x[i];
                rowsum[wv][18 * (R * w + h) + e] = sum;
            }
        }
        wave_sync_bwd();
    }
    __syncthreads();
    // workgroup partial of component q = 18*j + e: wavefronts in order, then
    // the link's three rows in order
    if (threadIdx.x < 72) {
        const int j = threadIdx.x / 18, e = threadIdx.x % 18;
        double sum = 0.0;
        for (int w2 = 0; w2 < kBwdWaves; ++w2)
            for (int r = 3 * j; r < 3 * j + 3; ++r)
                sum += rowsum[w2][18 * r + e];
        ws[4 * ((int64_t)(threadIdx.x >> 2) * groups + grp) + (threadIdx.x & 3)] = sum;
    }
}

// grid = (chunks, 18): workgroup (c, u) adds partials c*kChunk .. c*kChunk +
// kChunk - 1 of the 4 components of quad u (thread t takes t, t + kBlock,
// ... in order, then a tree per component) and writes run sums
// ws2[q * chunks + c] for q = 4u .. 4u+3.
__global__ __launch_bounds__(kBlock) void bwd_chunk_sums(const double *__restrict__ ws, double *__restrict__ ws2,
                                                         int64_t groups, int64_t chunks)
{
    __shared__ double red[4][kBlock];
    const int64_t c = blockIdx.x;
    const d2 *src = reinterpret_cast<const d2 *>(ws + 4 * (int64_t)blockIdx.y * groups);
    d2 v[kChunkLoads][2];
#pragma unroll
    for (int i = 0; i < kChunkLoads; ++i) {
        const int64_t g = c * kChunk + (int64_t)kBlock * i + threadIdx.x;
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
    for (int e = 0; e < 4; ++e)
        red[e][threadIdx.x] = sum[e];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                red[e][threadIdx.x] += red[e][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4)
        ws2[(int64_t)(4 * blockIdx.y + threadIdx.x) * chunks + c] = red[threadIdx.x][0];
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
    const int64_t units = sites * (precision == 0 ? BwdF64::kUnitsPerSite : BwdF32::kUnitsPerSite);
    const int64_t tiles = (units + 63) / 64;
    const int64_t per = (int64_t)kBwdWaves * (precision == 0 ? BwdF64::kTiles : BwdF32::kTiles);
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
                     (const double *)b, (const u4 *)dc, (u4 *)da, ws, sites * BwdF64::kUnitsPerSite, groups);
    } else {
        const size_t pad =
            occupancy_pad(reinterpret_cast<const void *>(bwd_tiles<BwdF32>), SU3_BWD_WAVES_F32, kBwdThreads, pad32);
        e = launch_k(bwd_tiles<BwdF32>, dim3((unsigned)groups), dim3(kBwdThreads), s, pad, (const u4 *)a,
                     (const float *)b, (const u4 *)dc, (u4 *)da, ws, sites * BwdF32::kUnitsPerSite, groups);
    }
    if (e != hipSuccess)
        return e;
    e = launch_k(bwd_chunk_sums, dim3((unsigned)chunks, 18), dim3(kBlock), s, 0, (const double *)ws, ws2, groups,
                 chunks);
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
