// su3_abi.hip -- the extern "C" entry points of libsu3 declared in su3.h:
// argument validation (before any HIP call), launch shape, dispatch.
#include "../../include/su3.h"
#include "su3_internal.hpp"


namespace {

using namespace su3;

static_assert(SU3_BWD_SCRATCH_BYTES == kScratchBytes, "su3.h and the library disagree on the scratch size");

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
    case SU3_R12C_F32: f = {192, 192, 288, 4}; return true;
    case SU3_R12_F64: f = {384, 576, 576, 8}; return true;
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

// A grid that covers the lattice once must stay below 2^32 work-items per
// dimension (far beyond any lattice that fits in one GPU's memory).
constexpr int64_t kMaxGridThreads = (int64_t)1 << 32;

bool grid_fits(int64_t blocks, int64_t threads)
{
    // blocks * threads < 2^32, without forming the product
    return blocks >= 0 && threads > 0 && blocks <= (kMaxGridThreads - 1) / threads;
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
    *grid = sites == 0 ? 0 : fwd_aos_grid(precision, sites);
    *block = aos_block_threads();
    return grid_fits(*grid, *block) ? SU3_OK : SU3_ERR_SIZE;
}

int su3_mult_nn(const void *a, const void *b, void *c, int64_t sites, int precision, void *stream)
{
    Form f;
    int st = check_lattice(a, b, c, sites, precision, f);
    if (st != SU3_OK || sites == 0)
        return st;
    if (!grid_fits(fwd_aos_grid(precision, sites), aos_block_threads()))
        return SU3_ERR_SIZE;
    return status_of(launch_fwd_aos(a, b, c, sites, precision, (hipStream_t)stream));
}

// Validation of the SoA entries: planes of `pitch` elements (pitch >= sites).
static int check_soa(const void *a, const void *b, const void *c, int64_t sites, int64_t pitch, int precision)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites || pitch < sites || pitch > kMaxSites)
        return SU3_ERR_SIZE;
    if (sites == 0)
        return SU3_OK;
    if (!a || !b || !c)
        return SU3_ERR_NULL;
    Form f;
    form_of(precision, f);
    if (!aligned(a, 16) || !aligned(c, 16) || !aligned(b, f.b_align))
        return SU3_ERR_ALIGN;
    const int64_t es = precision == SU3_F64 ? 16 : 8, extent = 36 * pitch * es;
    if (overlap(c, extent, a, extent) || overlap(c, extent, b, f.b_total))
        return SU3_ERR_OVERLAP;
    return SU3_OK;
}

static int mult_soa(const void *a, const void *b, void *c, int64_t sites, int64_t pitch, int precision, void *stream)
{
    const int st = check_soa(a, b, c, sites, pitch, precision);
    if (st != SU3_OK || sites == 0)
        return st;
    const int es = precision == SU3_F64 ? 16 : 8;
    if (!grid_fits(fwd_soa_grid(sites, pitch, es), soa_block_threads()))
        return SU3_ERR_SIZE;
    return status_of(launch_fwd_soa(a, b, c, sites, pitch, es, (hipStream_t)stream));
}

int su3_mult_nn_soa(const void *a, const void *b, void *c, int64_t sites, int precision, void *stream)
{
    return mult_soa(a, b, c, sites, sites, precision, stream);
}

int su3_mult_nn_soa_pitched(const void *a, const void *b, void *c, int64_t sites, int64_t pitch, int precision,
                            void *stream)
{
    return mult_soa(a, b, c, sites, pitch, precision, stream);
}

int su3_soa_pitch(int64_t sites, int precision, int64_t *pitch)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites - 1024)
        return SU3_ERR_SIZE;
    if (!pitch)
        return SU3_ERR_NULL;
    *pitch = soa_pitch(sites, precision == SU3_F64 ? 16 : 8);
    return SU3_OK;
}

int su3_mult_na(const void *a, const void *b, void *c, int64_t sites, int precision, void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    Form f;
    int st = check_lattice(a, b, c, sites, precision, f);
    if (st != SU3_OK || sites == 0)
        return st;
    if (!grid_fits(fwd_aos_grid(precision, sites), aos_block_threads()))
        return SU3_ERR_SIZE;
    return status_of(launch_fwd_na(a, b, c, sites, precision, (hipStream_t)stream));
}

int su3_mult_an(const void *a, const void *b, void *c, int64_t sites, int precision, void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    Form f;
    int st = check_lattice(a, b, c, sites, precision, f);
    if (st != SU3_OK || sites == 0)
        return st;
    if (!grid_fits(fwd_an_grid(precision, sites), aos_block_threads()))
        return SU3_ERR_SIZE;
    return status_of(launch_fwd_an(a, b, c, sites, precision, (hipStream_t)stream));
}

int su3_mat_vec(const void *a, const void *v, void *w, int64_t sites, int precision, void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites)
        return SU3_ERR_SIZE;
    if (sites == 0)
        return SU3_OK;
    if (!a || !v || !w)
        return SU3_ERR_NULL;
    if (!aligned(a, 16) || !aligned(w, 16) || !aligned(v, 8))
        return SU3_ERR_ALIGN;
    const int64_t es = precision == SU3_F64 ? 16 : 8;   // bytes per complex
    if (overlap(w, sites * 12 * es, a, sites * 36 * es) || overlap(w, sites * 12 * es, v, sites * 3 * es))
        return SU3_ERR_OVERLAP;
    if (!grid_fits(mat_vec_grid(precision, sites), 64))
        return SU3_ERR_SIZE;
    return status_of(launch_mat_vec(a, v, w, sites, precision, (hipStream_t)stream));
}

static int transform(const void *src, void *dst, int64_t sites, int64_t pitch, int precision, bool to_soa,
                     void *stream)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    if (sites < 0 || sites > kMaxSites || pitch < sites || pitch > kMaxSites)
        return SU3_ERR_SIZE;
    if (sites == 0)
        return SU3_OK;
    if (!src || !dst)
        return SU3_ERR_NULL;
    if (!aligned(src, 16) || !aligned(dst, 16))
        return SU3_ERR_ALIGN;
    const int64_t es = precision == SU3_F64 ? 16 : 8;
    const int64_t aos = sites * 36 * es, soa = pitch * 36 * es;
    if (overlap(src, to_soa ? aos : soa, dst, to_soa ? soa : aos))
        return SU3_ERR_OVERLAP;
    return status_of(launch_aos_soa(src, dst, sites, pitch, (int)es, to_soa, (hipStream_t)stream));
}

int su3_aos_to_soa(const void *src, void *dst, int64_t sites, int precision, void *stream)
{
    return transform(src, dst, sites, sites, precision, true, stream);
}

int su3_soa_to_aos(const void *src, void *dst, int64_t sites, int precision, void *stream)
{
    return transform(src, dst, sites, sites, precision, false, stream);
}

int su3_aos_to_soa_pitched(const void *src, void *dst, int64_t sites, int64_t pitch, int precision, void *stream)
{
    return transform(src, dst, sites, pitch, precision, true, stream);
}

int su3_soa_to_aos_pitched(const void *src, void *dst, int64_t sites, int64_t pitch, int precision, void *stream)
{
    return transform(src, dst, sites, pitch, precision, false, stream);
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
    if (precision == SU3_F64 && !grid_fits(sites * 36, 1))
        return SU3_ERR_SIZE;
    // the reconstruct-12 pack and unpack cover the links once, 64 per workgroup
    if ((precision == SU3_R12_F32 || precision == SU3_R12C_F32 || precision == SU3_R12_F64) &&
        !grid_fits((sites * 4 + 63) / 64, 64))
        return SU3_ERR_SIZE;
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
    return (size_t)bwd_workspace_doubles(sites, precision) * sizeof(double);
}

// Validation shared by both adjoint entry points. ws is the caller's
// workspace (checked for size, alignment and overlap) unless own_ws is set,
// in which case the library's own array is used and only its size is checked.
static int check_bwd(const void *a, const void *b, const void *dc, const void *da, const double *db_f64, int64_t sites,
                     int precision, const void *ws, size_t ws_bytes, bool own_ws)
{
    if (precision != SU3_F64 && precision != SU3_F32)
        return SU3_ERR_PRECISION;
    Form f;
    form_of(precision, f);
    if (sites < 0 || sites > kMaxSites || !grid_fits(bwd_groups(sites, precision), bwd_block_threads()))
        return SU3_ERR_SIZE;
    if (!db_f64)
        return SU3_ERR_NULL;
    if (sites > 0 && (!a || !b || !dc || !da))
        return SU3_ERR_NULL;
    const size_t need = su3_mult_nn_bwd_workspace_bytes(sites, precision);
    if (own_ws) {
        if (need > kScratchBytes)
            return SU3_ERR_WORKSPACE;
    } else if (sites > 0 && (!ws || ws_bytes < need)) {
        return SU3_ERR_WORKSPACE;
    }
    if (!aligned(db_f64, 8))
        return SU3_ERR_ALIGN;
    if (sites > 0 && (!aligned(a, 16) || !aligned(dc, 16) || !aligned(da, 16) || !aligned(b, f.b_align) ||
                      (!own_ws && !aligned(ws, 16))))
        return SU3_ERR_ALIGN;
    const int64_t n = sites * f.a_site;
    if (sites > 0 && (overlap(da, n, a, n) || overlap(da, n, dc, n) || overlap(da, n, b, f.b_total) ||
                      overlap(db_f64, 576, a, n) || overlap(db_f64, 576, dc, n) || overlap(db_f64, 576, da, n) ||
                      overlap(db_f64, 576, b, f.b_total)))
        return SU3_ERR_OVERLAP;
    if (sites > 0 && !own_ws &&
        (overlap(ws, (int64_t)need, a, n) || overlap(ws, (int64_t)need, dc, n) || overlap(ws, (int64_t)need, da, n) ||
         overlap(ws, (int64_t)need, b, f.b_total) || overlap(ws, (int64_t)need, db_f64, 576)))
        return SU3_ERR_OVERLAP;
    return SU3_OK;
}

int su3_mult_nn_bwd(const void *a, const void *b, const void *dc, void *da, double *db_f64, int64_t sites,
                    int precision, void *ws, size_t ws_bytes, void *stream)
{
    const int st = check_bwd(a, b, dc, da, db_f64, sites, precision, ws, ws_bytes, false);
    if (st != SU3_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    if (sites == 0)
        return status_of(launch_bwd_zero(db_f64, s));
    return status_of(launch_bwd(a, b, dc, da, db_f64, sites, precision, (double *)ws, s));
}

int su3_mult_nn_bwd_noalloc(const void *a, const void *b, const void *dc, void *da, double *db_f64, int64_t sites,
                            int precision, void *stream)
{
    const int st = check_bwd(a, b, dc, da, db_f64, sites, precision, nullptr, 0, true);
    if (st != SU3_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    if (sites == 0)
        return status_of(launch_bwd_zero(db_f64, s));
    double *ws = nullptr;
    const hipError_t e = bwd_scratch(&ws);
    if (e != hipSuccess)
        return SU3_ERR_HIP;
    return status_of(launch_bwd(a, b, dc, da, db_f64, sites, precision, ws, s));
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
    if (!grid_fits(bytes / 16, 1))
        return SU3_ERR_SIZE;
    return status_of(launch_stream_copy(src, dst, bytes, (hipStream_t)stream));
}

int su3_stream_shape(const void *a, const void *b, void *c, int64_t tiles, int in_a, int in_b, int out,
                     int waves_per_cu, int tile_order, void *stream)
{
    if (!stream_shape_supported(in_a, in_b, out))
        return SU3_ERR_SIZE;
    // the grid check first: it bounds tiles (below 2^26), so the byte counts
    // below cannot overflow
    if (tiles < 0 || waves_per_cu < 0 || waves_per_cu > 32 || (tile_order != 0 && tile_order != 1) ||
        !grid_fits(tiles, 64))
        return SU3_ERR_SIZE;
    if (tiles == 0)
        return SU3_OK;
    if (!a || !c || (in_b > 0 && !b))
        return SU3_ERR_NULL;
    if (!aligned(a, 16) || !aligned(c, 16) || (in_b > 0 && !aligned(b, 16)))
        return SU3_ERR_ALIGN;
    const int64_t na = tiles * 1024 * in_a, nb = tiles * 1024 * in_b, nc = tiles * 1024 * out;
    if (overlap(c, nc, a, na) || (in_b > 0 && overlap(c, nc, b, nb)))
        return SU3_ERR_OVERLAP;
    return status_of(
        launch_stream_shape(a, b, c, tiles, in_a, in_b, out, waves_per_cu, tile_order, (hipStream_t)stream));
}

} // extern "C"
