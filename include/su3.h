/*
 * su3.h -- C ABI of libsu3, the MI355X (gfx950) SU(3) link-multiply library.
 *
 * The operation is the core kernel of SU3_Bench (arXiv 2103.00571, section
 * "Background", subsection SU3_Bench): over an L^4 lattice every site holds
 * four links, each a 3x3 complex matrix, and for every site s and link j
 *
 *     c[s].link[j] = a[s].link[j] * b[j]          (j = 0..3)
 *
 * where each output entry (k, l) is the dot product of row k of a[s].link[j]
 * with column l of b[j], and b is four matrices shared by every site.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named a, b, c, src, dst, dc, da are DEVICE pointers (memory the
 *    caller allocated with hipMalloc or any allocator of device memory on the
 *    current device). db_f64 is a device pointer too.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Every call is asynchronous on that stream: it only enqueues kernels and
 *    returns. No call allocates memory, synchronises, or keeps pointers after
 *    returning. The caller owns every buffer.
 *  - `sites` is the number of lattice sites (L^4 for an L^4 lattice).
 *    sites == 0 is valid and launches nothing, with one exception: the
 *    adjoint (su3_mult_nn_bwd) must still write db = 0, so for sites == 0 it
 *    enqueues one small kernel that zeroes the 72 doubles of db_f64 (a
 *    kernel, not a memset, so the call stays safe to capture in a graph).
 *  - Complex numbers are interleaved (re, im). A link is row-major 3x3:
 *    element (k, l) at complex offset 3k + l.
 *  - Site-major ("AoS") layout: link j of site s at complex offset
 *    (s*4 + j)*9; as a tensor, shape (sites, 4, 3, 3).
 *  - Structure-of-arrays ("SoA") layout: 36 planes of `sites` complex
 *    elements; element p = (j*3 + k)*3 + l of site s at complex offset
 *    p*sites + s; as a tensor, shape (4, 3, 3, sites).
 *  - Arguments are validated before anything is enqueued; on any error
 *    nothing is launched and the status says why. A failed launch returns
 *    SU3_ERR_HIP. Faults inside a kernel surface at the caller's next
 *    synchronisation, as with any HIP library.
 *  - Thread safety: calls may be made concurrently from several host threads.
 *
 * Storage forms (the `precision` argument)
 * ----------------------------------------
 *  code         a (per site)                b                 c (per site)
 *  SU3_F64      4x3x3 complex double, 576 B  4x3x3 cdouble     576 B, FP64
 *  SU3_F32      4x3x3 complex float,  288 B  4x3x3 cfloat      288 B, FP32
 *  SU3_BF16     4x3x3x(re,im) bf16,   144 B  4x3x3 cfloat      144 B, BF16
 *  SU3_R12_F32  rows 0-1 only: 4x2x3 cfloat, 4x3x3 cfloat      288 B, full FP32
 *               192 B; row 2 is rebuilt as
 *               conj(row0 x row1)
 *  SU3_R12C_F32 rows 0-1 only, as above  4x3x3 cfloat      rows 0-1 only: 4x2x3
 *               (192 B)                                     cfloat, 192 B
 *  SU3_R12_F64  rows 0-1 only: 4x2x3     4x3x3 cdouble     576 B, full FP64
 *               complex double, 384 B
 * FP32, BF16, R12_F32 and R12C_F32 compute in FP32; FP64 and R12_F64 compute
 * in FP64. BF16 results are rounded to nearest, ties to even. The
 * reconstruct-12 forms are valid for links in SU(3), for which the third row
 * equals the conjugate cross product of the first two. R12C_F32 keeps the
 * product compressed too: rows 0-1 of a*b are rows 0-1 of a times b, and the
 * product of SU(3) matrices is in SU(3), so its third row can be rebuilt the
 * same way (su3_unpack).
 */
#ifndef SU3_H
#define SU3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SU3_ABI_VERSION 6

/* storage form codes */
enum su3_precision {
    SU3_F64 = 0,
    SU3_F32 = 1,
    SU3_BF16 = 2,
    SU3_R12_F32 = 3,
    SU3_R12C_F32 = 4,
    SU3_R12_F64 = 5
};

/* status codes */
enum su3_status {
    SU3_OK = 0,
    SU3_ERR_NULL = -1,       /* a required pointer is NULL while sites > 0     */
    SU3_ERR_SIZE = -2,       /* sites < 0, or a byte count is out of range      */
    SU3_ERR_ALIGN = -3,      /* a lattice pointer is not 16-byte aligned        */
    SU3_ERR_PRECISION = -4,  /* unknown form, or a form this entry lacks        */
    SU3_ERR_OVERLAP = -5,    /* an output overlaps an input                     */
    SU3_ERR_WORKSPACE = -6,  /* workspace missing or smaller than required      */
    SU3_ERR_HIP = -7         /* a HIP runtime call or kernel launch failed      */
};

/* Library version of this header; a mismatch means the .so is stale. */
int su3_abi_version(void);

/* Human-readable text of a status code (static string, never NULL). */
const char *su3_status_string(int status);

/*
 * Forward product on the site-major layout (the paper's SU3_Bench kernel,
 * section "Background", subsection SU3_Bench):
 *   c[s][j](k, l) = sum_m a[s][j](k, m) * b[j](m, l).
 * a, c: AoS arrays in the form `precision` (table above), 16-byte aligned,
 * c must not overlap a or b (in-place is not supported). b: 4 links, in
 * complex double for SU3_F64 and complex float for every other form; b needs
 * only 8-byte alignment. c is overwritten, never accumulated.
 * Errors: SU3_ERR_NULL, SU3_ERR_SIZE, SU3_ERR_ALIGN, SU3_ERR_PRECISION,
 * SU3_ERR_OVERLAP, SU3_ERR_HIP.
 */
int su3_mult_nn(const void *a, const void *b, void *c, int64_t sites,
                int precision, void *stream);

/*
 * The two other link products of the MILC code the benchmark's kernel is
 * derived from (arXiv 2103.00571, section Introduction: SU(3) matrix-matrix
 * operations as a building block of lattice QCD); they are also the two
 * contractions of the adjoint (su3_mult_nn_bwd):
 *   su3_mult_na: c[s][j] = a[s][j] * b[j]^H,  c(k, l) = sum_m a(k, m) conj(b(l, m))
 *   su3_mult_an: c[s][j] = a[s][j]^H * b[j],  c(k, l) = sum_m conj(a(m, k)) b(m, l)
 * Site-major layout, SU3_F64 and SU3_F32 only (other forms return
 * SU3_ERR_PRECISION); arguments, alignment, overlap and errors as
 * su3_mult_nn.
 */
int su3_mult_na(const void *a, const void *b, void *c, int64_t sites,
                int precision, void *stream);
int su3_mult_an(const void *a, const void *b, void *c, int64_t sites,
                int precision, void *stream);

/*
 * SU(3) matrix times colour vector, the matrix-vector building block named
 * beside the matrix-matrix product (arXiv 2103.00571, section Introduction):
 * every link of a site applied to the site's own colour vector,
 *   w[s][j](k) = sum_m a[s][j](k, m) v[s](m),   j = 0..3.
 * a: site-major links, (sites, 4, 3, 3) complex, 16-byte aligned.
 * v: one colour vector per site, (sites, 3) complex, 8-byte aligned.
 * w: (sites, 4, 3) complex, 16-byte aligned, overlapping neither input.
 * SU3_F64 (complex double) and SU3_F32 (complex float) only.
 * Errors: SU3_ERR_NULL, SU3_ERR_SIZE, SU3_ERR_ALIGN, SU3_ERR_PRECISION,
 * SU3_ERR_OVERLAP, SU3_ERR_HIP.
 */
int su3_mat_vec(const void *a, const void *v, void *w, int64_t sites,
                int precision, void *stream);

/*
 * The same product on the SoA layout: a and c are 36 planes of `sites`
 * complex elements. The paper names remapping the data structures as the
 * main step in tuning SU3_Bench for wide SIMD machines (arXiv 2103.00571,
 * section Related Work); the SoA layout is that remapping, with every plane
 * access of a wavefront one contiguous run. Supports SU3_F64 and SU3_F32
 * (other forms return SU3_ERR_PRECISION). Same alignment, overlap and error
 * rules as su3_mult_nn.
 */
int su3_mult_nn_soa(const void *a, const void *b, void *c, int64_t sites,
                    int precision, void *stream);

/*
 * The SoA product on a padded SoA layout: plane p of a and c starts at
 * complex offset p*pitch (pitch >= sites); elements sites .. pitch-1 of each
 * plane are padding, never read or written. With pitch == sites this is
 * su3_mult_nn_soa. In the dense layout the three planes a row reads lie one
 * plane stride apart, and at some site counts (powers of two among them) the
 * same offsets of those planes collide in HBM; a padded stride avoids that,
 * the way lattice QCD codes pad their field strides. When the site count is
 * not a multiple of 8 (SU3_F64) or 16 (SU3_F32), dense planes also start off
 * 128-byte boundaries, and their partial-line writes cost the product and the
 * AoS -> SoA transform 10-25%; a pitch that is a multiple of 64 sites keeps
 * every plane aligned. su3_soa_pitch gives the pitch at which the product
 * streams at the site-major rate. Arguments,
 * alignment and errors as su3_mult_nn_soa; a and c each span 36*pitch
 * complex elements, c must not overlap a or b; pitch < sites returns
 * SU3_ERR_SIZE.
 */
int su3_mult_nn_soa_pitched(const void *a, const void *b, void *c, int64_t sites,
                            int64_t pitch, int precision, void *stream);

/*
 * Plane pitch (in complex elements) for a padded SoA layout of `sites`
 * sites: sites rounded up to a multiple of 64, plus 512 (SU3_F64) or 128
 * (SU3_F32); measured to stream at the site-major rate at every site count
 * tried. Writes *pitch. Errors: SU3_ERR_PRECISION (not SU3_F64 or SU3_F32),
 * SU3_ERR_SIZE (sites < 0 or too large), SU3_ERR_NULL.
 */
int su3_soa_pitch(int64_t sites, int precision, int64_t *pitch);

/*
 * Layout transforms between AoS and SoA for SU3_F64 and SU3_F32 (a pure
 * permutation of complex elements, bit-exact): the data-structure remapping
 * of arXiv 2103.00571, section Related Work, as an explicit step outside the
 * product. src and dst must not overlap and must be 16-byte aligned.
 * Errors: SU3_ERR_NULL, SU3_ERR_SIZE, SU3_ERR_ALIGN, SU3_ERR_PRECISION,
 * SU3_ERR_OVERLAP, SU3_ERR_HIP.
 */
int su3_aos_to_soa(const void *src, void *dst, int64_t sites, int precision,
                   void *stream);
int su3_soa_to_aos(const void *src, void *dst, int64_t sites, int precision,
                   void *stream);
/*
 * The same transforms to and from the padded SoA layout (plane p at complex
 * offset p*pitch, pitch >= sites): the SoA side spans 36*pitch elements and
 * its padding is neither read nor written. pitch < sites returns
 * SU3_ERR_SIZE; otherwise as above.
 */
int su3_aos_to_soa_pitched(const void *src, void *dst, int64_t sites,
                           int64_t pitch, int precision, void *stream);
int su3_soa_to_aos_pitched(const void *src, void *dst, int64_t sites,
                           int64_t pitch, int precision, void *stream);

/*
 * Conversion from FP64 AoS links to a storage form, and back. The paper has
 * no such step (its benchmark stores one precision); these entries belong to
 * the library's reduced storage forms, which cut the bytes the product
 * streams per site.
 *  su3_pack:   src is FP64 AoS; dst is the `precision` form of a
 *              (SU3_F32: round to nearest even; SU3_BF16: round to FP32, then
 *              to BF16, each to nearest even; SU3_R12_F32 and SU3_R12C_F32:
 *              rows 0 and 1 of every link rounded to FP32, 192 B per site;
 *              SU3_R12_F64: rows 0 and 1 kept in FP64, 384 B per site;
 *              SU3_F64: copy).
 *  su3_unpack: src is the `precision` form; dst is FP64 AoS. Widening is
 *              exact; for the reconstruct-12 forms row 2 is rebuilt in FP64
 *              as conj(row0 x row1) from the widened rows, each product and
 *              difference rounded separately (no fused multiply-add).
 * Both are bit-exact functions of their input.
 * Errors: SU3_ERR_NULL, SU3_ERR_SIZE, SU3_ERR_ALIGN, SU3_ERR_PRECISION,
 * SU3_ERR_OVERLAP, SU3_ERR_HIP.
 */
int su3_pack(const void *src_f64_aos, void *dst, int64_t sites, int precision,
             void *stream);
int su3_unpack(const void *src, void *dst_f64_aos, int64_t sites, int precision,
               void *stream);

/*
 * Adjoint of su3_mult_nn for SU3_F64 and SU3_F32 (AoS). The paper has no
 * adjoint; these are the two contractions that differentiate its product
 * (section Background, subsection SU3_Bench), added so that the product can
 * sit inside a differentiable program. For the real loss
 * Re sum conj(dc) * c, in the complex-gradient convention
 * dL/dRe(x) + i dL/dIm(x):
 *   da[s][j](k, m) = sum_l dc[s][j](k, l) * conj(b[j](m, l))      (dc b^H)
 *   db[j](m, l)    = sum_s sum_k conj(a[s][j](k, m)) * dc[s][j](k, l)
 * da has the form of a (FP64 or FP32). db_f64 receives 4x3x3 complex double
 * (72 doubles) in every form: the site sum is accumulated in FP64 by a
 * two-stage reduction whose order depends only on `sites`, so repeated calls
 * give bit-identical db on any device. ws is device scratch of at least
 * su3_mult_nn_bwd_workspace_bytes(sites, precision) bytes, 16-byte aligned,
 * owned by the caller, contents undefined on entry and exit.
 * da must not overlap a, b or dc; db_f64 and ws must not overlap anything.
 * sites == 0: a, b, dc, da and ws may be NULL; one kernel writes db = 0.
 * Errors: as su3_mult_nn, plus SU3_ERR_WORKSPACE.
 */
size_t su3_mult_nn_bwd_workspace_bytes(int64_t sites, int precision);
int su3_mult_nn_bwd(const void *a, const void *b, const void *dc, void *da,
                    double *db_f64, int64_t sites, int precision, void *ws,
                    size_t ws_bytes, void *stream);

/*
 * Allocation-free variant of su3_mult_nn_bwd, for callers that cannot
 * allocate device memory or pass a workspace: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The workspace is a
 * fixed array of SU3_BWD_SCRATCH_BYTES (64 MiB) in the library's device
 * memory, one per device, kept until the process ends; the call itself
 * allocates nothing. Arguments, results (bit for bit) and errors are those of
 * su3_mult_nn_bwd without ws and ws_bytes, except that SU3_ERR_WORKSPACE
 * means the lattice needs more workspace than the array holds:
 * su3_mult_nn_bwd_workspace_bytes(sites, precision) > SU3_BWD_SCRATCH_BYTES,
 * i.e. above about 7.4 million sites in FP64 and 14.9 million in FP32 (an
 * L = 48 lattice, 5,308,416 sites, fits in both). The array's device address
 * is looked up on the first call on each device, so make that first call
 * outside graph capture. Every call on a device shares that device's array:
 * calls that can overlap in time on one device (two streams, two host
 * threads, two graphs) race on it and must be ordered by the caller.
 */
#define SU3_BWD_SCRATCH_BYTES ((size_t)64 << 20)
int su3_mult_nn_bwd_noalloc(const void *a, const void *b, const void *dc, void *da,
                            double *db_f64, int64_t sites, int precision,
                            void *stream);

/*
 * Measurement aid: device-to-device copy of `bytes` bytes, one 16-byte
 * nontemporal load and store per thread over a grid that covers the buffer
 * once, the streaming pattern of the link multiply without the arithmetic. Used to
 * measure the HBM bandwidth the multiply is compared against. bytes must be
 * a multiple of 16; src and dst 16-byte aligned and non-overlapping.
 */
int su3_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);

/*
 * Measurement aid: the streaming ceiling of an access shape. Over `tiles`
 * wavefront tiles, tile w reads in_a 16-byte chunks per lane from a (bytes
 * w*1024*in_a .. (w+1)*1024*in_a - 1, as in_a whole-wavefront 1 KiB runs),
 * in_b chunks per lane from b likewise, and writes out chunks per lane to c
 * (bytes w*1024*out ..), with one 64-thread workgroup per tile and at most
 * waves_per_cu resident wavefronts per CU (0: no cap, at most 32).
 * tile_order picks which workgroup takes which tile: 0, workgroup i takes
 * tile i (the order of su3_stream_copy, su3_mult_nn_soa and the adjoint);
 * 1, XCD-contiguous, the order of the site-major products, the matrix-vector
 * product and the reconstruct-12 pack and unpack. MI355X deals workgroups
 * round-robin to its 8 XCDs, and order 1 gives XCD x (the workgroups i with
 * i mod 8 = x) one contiguous run of tiles: with q = tiles / 8 and
 * r = tiles mod 8, its k-th workgroup takes tile x*q + min(x, r) + k. The
 * values written are the XOR of the lane's loaded chunks with the chunk
 * number added to the first word. The shapes are those of the kernels:
 * (in_a, in_b, out) = (1, 0, 1) copy; (3, 0, 3) the FP64/FP32/BF16 forward;
 * (3, 3, 3) the adjoint; (6, 0, 9) reconstruct-12 with full output;
 * (9, 0, 9) a^H b. Sizes: a holds tiles*1024*in_a bytes, b tiles*1024*in_b
 * (b may be NULL when in_b is 0), c tiles*1024*out; 16-byte aligned; c must
 * not overlap a or b. Errors: SU3_ERR_SIZE for another shape, a negative
 * count, a cap above 32 or a tile_order other than 0 and 1; otherwise as
 * su3_stream_copy.
 */
int su3_stream_shape(const void *a, const void *b, void *c, int64_t tiles, int in_a, int in_b, int out,
                     int waves_per_cu, int tile_order, void *stream);

/*
 * Launch shape the library uses for su3_mult_nn on the current device:
 * writes the number of workgroups and threads per workgroup it would launch
 * for (sites, precision). Returns SU3_OK or an error code.
 */
int su3_launch_shape(int64_t sites, int precision, int64_t *grid, int *block);

#ifdef __cplusplus
}
#endif

#endif /* SU3_H */
