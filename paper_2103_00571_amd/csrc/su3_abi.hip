// su3_abi.hip -- the extern "C" entry points of libsu3 declared in su3.h:
// argument validation (before any HIP call), launch shape, dispatch.
#include "../../include/su3.h"
#include "su3_internal.hpp"

#include <atomic>

// Upper limit on resident workgroups per CU for the persistent kernels; the
// occupancy calculator usually sets a lower one.
#ifndef SU3_BLOCKS_PER_CU
#define SU3_BLOCKS_PER_CU 16
#endif

namespace {

using namespace su3;

// byte sizes per site of a and c, and of the four b links, per form
struct Form {
    int64_t a_site, c_site, b_total, b_align;
};

bool form_of(int precision, Form &f)
{
    switch (precision) {
    case SU3_F64: f = {576, 576, 576, 8}; return true;
    case SU3_F32: f = {288, 288, 288, 4}; return true;
    case SU3_BF16: f = {144, 144, 288, 4}; return true;
    case SU3_R12_F32: f = {192, 288, 288, 4}; return true;
    default: return false;
    }
}

// largest site count whose biggest array (R12 unpack writes 576 B per site,
// the adjoint touches four arrays) keeps every byte offset within int64
constexpr int64_t kMaxSites = INT64_MAX / 4096;

bool aligned(const void *p, int64_t n) { return ((uintptr_t)p % (uintptr_t)n) == 0; }

bool overlap(const void *p, int64_t pn, const void *q, int64_t qn)
{
    if (pn <= 0 || qn <= 0)
        return false;
    const uintptr_t a0 = (uintptr_t)p, a1 = a0 + (uintptr_t)pn;
    const uintptr_t b0 = (uintptr_t)q, b1 = b0 + (uintptr_t)qn;
    return a0 < b1 && b0 < a1;
}

int status_of(hipError_t e) { return e == hipSuccess ? SU3_OK : SU3_ERR_HIP; }

// compute units of the current device, cached per device
std::atomic<int> g_cus[kMaxDevices];

int device_cus(int *cus)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return SU3_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices)
        return SU3_ERR_HIP;
    int n = g_cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            return SU3_ERR_HIP;
        g_cus[dev].store(n, std::memory_order_relaxed);
    }
    *cus = n;
    return SU3_OK;
}

// Persistent grid for the streaming kernels. Every workgroup must be resident
// at once (a late wave of workgroups would double the tail), so the grid is
// at most CUs x resident-workgroups-per-CU. It is a multiple of 3, so that the
// grid-stride step is a whole number of sites for every form: rounded down
// when capped by residency, rounded up (with idle workgroups) otherwise.
int64_t persistent_grid(int64_t units, int cus, int resident)
{
    if (resident > SU3_BLOCKS_PER_CU)
        resident = SU3_BLOCKS_PER_CU;
    const int64_t need = (units + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * resident;
    if (need <= cap || cap < 3)
        return need < 1 ? 3 : (need + 2) / 3 * 3;
    return cap / 3 * 3;
}

int64_t units_per_site(int precision)
{
    switch (precision) {
    case SU3_F64: return 12;
    case SU3_F32: return 6;
    case SU3_BF16: return 3;
    default: return 2;
    }
}

// Adjoint stage-1 workgroups: a function of the site count only (never of the
// device), capped, and a multiple of 3.
// 1023 = 3 x 341 workgroups are resident at once on a 256-CU MI355X (four
// per CU, bounded by registers and LDS).
constexpr int64_t kBwdMaxGroups = 1023;

int64_t bwd_groups(int64_t sites)
{
    int64_t g = (sites * 12 + kBlock - 1) / kBlock;
    if (g > kBwdMaxGroups)
        g = kBwdMaxGroups;
    if (g < 1)
        g = 1;
    return (g + 2) / 3 * 3;
}

int check_lattice(const void *a, const void *b, const void *c, int64_t sites, int precision, Form &f)
{
    if (!form_of(precision, f))
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites)
        return SU3_ERR_SIZE;
    if (sites == 0)
        return SU3_OK;
    if (!a || !b || !c)
        return SU3_ERR_NULL;
    if (!aligned(a, 16) || !aligned(c, 16) || !aligned(b, f.b_align))
        return SU3_ERR_ALIGN;
    if (overlap(c, sites * f.c_site, a, sites * f.a_site) || overlap(c, sites * f.c_site, b, f.b_total))
        return SU3_ERR_OVERLAP;
    return SU3_OK;
}

} // namespace

extern "C" {

int su3_abi_version(void) { return SU3_ABI_VERSION; }

const char *su3_status_string(int status)
{
    switch (status) {
    case SU3_OK: return "SU3_OK: success";
    case SU3_ERR_NULL: return "SU3_ERR_NULL: a required pointer is NULL";
    case SU3_ERR_SIZE: return "SU3_ERR_SIZE: size out of range";
    case SU3_ERR_ALIGN: return "SU3_ERR_ALIGN: pointer not aligned (lattice arrays need 16 bytes)";
    case SU3_ERR_PRECISION: return "SU3_ERR_PRECISION: unknown or unsupported storage form";
    case SU3_ERR_OVERLAP: return "SU3_ERR_OVERLAP: an output overlaps an input";
    case SU3_ERR_WORKSPACE: return "SU3_ERR_WORKSPACE: workspace missing or too small";
    case SU3_ERR_HIP: return "SU3_ERR_HIP: HIP runtime call or kernel launch failed";
    default: return "unknown su3 status";
    }
}

int su3_launch_shape(int64_t sites, int precision, int64_t *grid, int *block)
{
    Form f;
    if (!form_of(precision, f))
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites)
        return SU3_ERR_SIZE;
    if (!grid || !block)
        return SU3_ERR_NULL;
    int cus = 0;
    int st = device_cus(&cus);
    if (st != SU3_OK)
        return st;
    const int res = fwd_resident_blocks(precision);
    if (res <= 0)
        return SU3_ERR_HIP;
    *grid = sites == 0 ? 0 : persistent_grid(sites * units_per_site(precision), cus, res);
    *block = kBlock;
    return SU3_OK;
}

int su3_mult_nn(const void *a, const void *b, void *c, int64_t sites, int precision, void *stream)
{
    Form f;
    int st = check_lattice(a, b, c, sites, precision, f);
    if (st != SU3_OK || sites == 0)
        return st;
    int cus = 0;
    if ((st = device_cus(&cus)) != SU3_OK)
        return st;
    const int res = fwd_resident_blocks(precision);
    if (res <= 0)
        return SU3_ERR_HIP;
    const int64_t grid = persistent_grid(sites * units_per_site(precision), cus, res);
    hipStream_t s = (hipStream_t)stream;
    switch (precision) {
    case SU3_F64: return status_of(launch_fwd_aos_f64(a, b, c, sites, grid, s));
    case SU3_F32: return status_of(launch_fwd_aos_f32(a, b, c, sites, grid, s));
    case SU3_BF16: return status_of(launch_fwd_aos_bf16(a, b, c, sites, grid, s));
    default: return status_of(launch_fwd_aos_r12(a, b, c, sites, grid, s));
    }
}

int su3_mult_nn_soa(const void *a, const void *b, void *c, int64_t sites, int precision, void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    Form f;
    int st = check_lattice(a, b, c, sites, precision, f);
    if (st != SU3_OK || sites == 0)
        return st;
    int cus = 0;
    if ((st = device_cus(&cus)) != SU3_OK)
        return st;
    // four link rows (grid.y) of gx workgroups; all resident at once
    const int eb = precision == SU3_F64 ? 16 : 8;
    int res = soa_resident_blocks(eb);
    if (res <= 0)
        return SU3_ERR_HIP;
    if (res > SU3_BLOCKS_PER_CU)
        res = SU3_BLOCKS_PER_CU;
    int64_t gx = (sites + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)cus * res / 4;
    if (gx > cap)
        gx = cap < 1 ? 1 : cap;
    return status_of(launch_fwd_soa(a, b, c, sites, eb, gx, (hipStream_t)stream));
}

static int transform(const void *src, void *dst, int64_t sites, int precision, bool to_soa, void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites)
        return SU3_ERR_SIZE;
    if (sites == 0)
        return SU3_OK;
    if (!src || !dst)
        return SU3_ERR_NULL;
    if (!aligned(src, 16) || !aligned(dst, 16))
        return SU3_ERR_ALIGN;
    const int64_t bytes = sites * (precision == SU3_F64 ? 576 : 288);
    if (overlap(src, bytes, dst, bytes))
        return SU3_ERR_OVERLAP;
    return status_of(launch_aos_soa(src, dst, sites, precision == SU3_F64 ? 16 : 8, to_soa, (hipStream_t)stream));
}

int su3_aos_to_soa(const void *src, void *dst, int64_t sites, int precision, void *stream)
{
    return transform(src, dst, sites, precision, true, stream);
}

int su3_soa_to_aos(const void *src, void *dst, int64_t sites, int precision, void *stream)
{
    return transform(src, dst, sites, precision, false, stream);
}

static int convert(const void *src, void *dst, int64_t sites, int precision, bool pack, void *stream)
{
    Form f;
    if (!form_of(precision, f))
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites)
        return SU3_ERR_SIZE;
    if (sites == 0)
        return SU3_OK;
    if (!src || !dst)
        return SU3_ERR_NULL;
    if (!aligned(src, 16) || !aligned(dst, 16))
        return SU3_ERR_ALIGN;
    const int64_t wide = sites * 576, narrow = sites * f.a_site;
    if (overlap(src, pack ? wide : narrow, dst, pack ? narrow : wide))
        return SU3_ERR_OVERLAP;
    hipStream_t s = (hipStream_t)stream;
    return status_of(pack ? launch_pack(src, dst, sites, precision, s) : launch_unpack(src, dst, sites, precision, s));
}

int su3_pack(const void *src_f64_aos, void *dst, int64_t sites, int precision, void *stream)
{
    return convert(src_f64_aos, dst, sites, precision, true, stream);
}

int su3_unpack(const void *src, void *dst_f64_aos, int64_t sites, int precision, void *stream)
{
    return convert(src, dst_f64_aos, sites, precision, false, stream);
}

size_t su3_mult_nn_bwd_workspace_bytes(int64_t sites, int precision)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return 0;
    if (sites <= 0 || sites > kMaxSites)
        return 0;
    return (size_t)bwd_groups(sites) * 72 * sizeof(double);
}

int su3_mult_nn_bwd(const void *a, const void *b, const void *dc, void *da, double *db_f64, int64_t sites,
                    int precision, void *ws, size_t ws_bytes, void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    Form f;
    form_of(precision, f);
    if (sites < 0 || sites > kMaxSites)
        return SU3_ERR_SIZE;
    if (!db_f64)
        return SU3_ERR_NULL;
    if (sites > 0 && (!a || !b || !dc || !da))
        return SU3_ERR_NULL;
    const size_t need = su3_mult_nn_bwd_workspace_bytes(sites, precision);
    if (sites > 0 && (!ws || ws_bytes < need))
        return SU3_ERR_WORKSPACE;
    if (!aligned(db_f64, 8))
        return SU3_ERR_ALIGN;
    if (sites > 0 && (!aligned(a, 16) || !aligned(dc, 16) || !aligned(da, 16) || !aligned(b, f.b_align) ||
                      !aligned(ws, 16)))
        return SU3_ERR_ALIGN;
    const int64_t n = sites * f.a_site;
    if (sites > 0 && (overlap(da, n, a, n) || overlap(da, n, dc, n) || overlap(da, n, b, f.b_total) ||
                      overlap(db_f64, 576, a, n) || overlap(db_f64, 576, dc, n) || overlap(db_f64, 576, da, n) ||
                      overlap(db_f64, 576, b, f.b_total) || overlap(ws, (int64_t)need, a, n) ||
                      overlap(ws, (int64_t)need, dc, n) || overlap(ws, (int64_t)need, da, n) ||
                      overlap(ws, (int64_t)need, b, f.b_total) || overlap(ws, (int64_t)need, db_f64, 576)))
        return SU3_ERR_OVERLAP;
    hipStream_t s = (hipStream_t)stream;
    if (sites == 0)
        return status_of(launch_bwd_zero(db_f64, s));
    return status_of(launch_bwd(a, b, dc, da, db_f64, sites, precision, (double *)ws, bwd_groups(sites), s));
}

int su3_stream_copy(const void *src, void *dst, int64_t bytes, void *stream)
{
    if (bytes < 0 || bytes % 16 != 0)
        return SU3_ERR_SIZE;
    if (bytes == 0)
        return SU3_OK;
    if (!src || !dst)
        return SU3_ERR_NULL;
    if (!aligned(src, 16) || !aligned(dst, 16))
        return SU3_ERR_ALIGN;
    if (overlap(src, bytes, dst, bytes))
        return SU3_ERR_OVERLAP;
    int cus = 0;
    int st = device_cus(&cus);
    if (st != SU3_OK)
        return st;
    const int res = copy_resident_blocks();
    if (res <= 0)
        return SU3_ERR_HIP;
    return status_of(
        launch_stream_copy(src, dst, bytes, persistent_grid(bytes / 16, cus, res), (hipStream_t)stream));
}

} // extern "C"
