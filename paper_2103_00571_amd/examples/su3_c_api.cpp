// su3_c_api.cpp -- calling libsu3 through its C ABI alone (no Python, no
// torch): device buffers from hipMalloc, a HIP stream, the forward product
// in FP64, the adjoint with its caller-owned workspace, and the product on
// the padded SoA layout at the pitch the library recommends.
//
// With b[j] = I every product is an exact copy, so the program can check its
// results without any reference implementation: c must equal a bit for bit
// (also after AoS -> padded SoA, the SoA product and back), and dA = dC b^H
// must equal dC bit for bit. The entries of a and dC are
// small integers, so every partial sum of dB = sum_s a^H dC is an integer
// below 2^53 and exact in FP64: dB must equal the same sum formed in int64
// on the host. Exit status 0 and "ok" on success; the status string of the
// failing call otherwise.
//
//   su3_c_api [sites]          (default 100003)
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "su3.h"

#define HIP_OK(x)                                                                                                  \
    do {                                                                                                           \
        hipError_t e_ = (x);                                                                                       \
        if (e_ != hipSuccess) {                                                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                                         \
            return 2;                                                                                              \
        }                                                                                                          \
    } while (0)

#define SU3_OK_OR_FAIL(x)                                                                                          \
    do {                                                                                                           \
        int s_ = (x);                                                                                              \
        if (s_ != SU3_OK) {                                                                                        \
            std::fprintf(stderr, "%s: %s\n", #x, su3_status_string(s_));                                         \
            return 3;                                                                                              \
        }                                                                                                          \
    } while (0)

int main(int argc, char **argv)
{
    const int64_t sites = argc > 1 ? std::atoll(argv[1]) : 100003;
    if (sites <= 0)
        return 1;
    if (su3_abi_version() != SU3_ABI_VERSION) {
        std::fprintf(stderr, "libsu3 ABI %d, header %d\n", su3_abi_version(), SU3_ABI_VERSION);
        return 1;
    }
    const size_t n = (size_t)sites * 36 * 2;      // doubles per lattice (36 complex per site)
    std::vector<double> a(n), dc(n), b(72, 0.0), out(n);
    for (size_t i = 0; i < n; ++i) {               // any values: integers keep the check readable
        a[i] = (double)((int64_t)(i * 2654435761u % 2001) - 1000);
        dc[i] = (double)((int64_t)(i * 40503u % 1999) - 999);
    }
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 3; ++k)
            b[2 * (9 * j + 4 * k)] = 1.0;         // b[j] = identity

    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));
    double *d_a, *d_b, *d_c, *d_dc, *d_da, *d_db;
    void *d_ws;
    const size_t bytes = n * sizeof(double);
    const size_t ws_bytes = su3_mult_nn_bwd_workspace_bytes(sites, SU3_F64);
    HIP_OK(hipMalloc((void **)&d_a, bytes));
    HIP_OK(hipMalloc((void **)&d_c, bytes));
    HIP_OK(hipMalloc((void **)&d_dc, bytes));
    HIP_OK(hipMalloc((void **)&d_da, bytes));
    HIP_OK(hipMalloc((void **)&d_b, 72 * sizeof(double)));
    HIP_OK(hipMalloc((void **)&d_db, 72 * sizeof(double)));
    HIP_OK(hipMalloc(&d_ws, ws_bytes));
    HIP_OK(hipMemcpy(d_a, a.data(), bytes, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_dc, dc.data(), bytes, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_b, b.data(), 72 * sizeof(double), hipMemcpyHostToDevice));

    // c = a b (enqueued on `stream`; the call returns at once)
    SU3_OK_OR_FAIL(su3_mult_nn(d_a, d_b, d_c, sites, SU3_F64, stream));
    // dA = dC b^H and dB = sum_s a^H dC, with the caller's workspace
    SU3_OK_OR_FAIL(su3_mult_nn_bwd(d_a, d_b, d_dc, d_da, d_db, sites, SU3_F64, d_ws, ws_bytes, stream));
    // a rejected call launches nothing and says why
    if (su3_mult_nn(d_a, d_b, d_a, sites, SU3_F64, stream) != SU3_ERR_OVERLAP) {
        std::fprintf(stderr, "in-place call was not rejected\n");
        return 4;
    }
    HIP_OK(hipStreamSynchronize(stream));

    HIP_OK(hipMemcpy(out.data(), d_c, bytes, hipMemcpyDeviceToHost));
    if (std::memcmp(out.data(), a.data(), bytes) != 0) {
        std::fprintf(stderr, "c != a for b = I\n");
        return 5;
    }
    HIP_OK(hipMemcpy(out.data(), d_da, bytes, hipMemcpyDeviceToHost));
    if (std::memcmp(out.data(), dc.data(), bytes) != 0) {
        std::fprintf(stderr, "dA != dC for b = I\n");
        return 6;
    }
    // dB[j](m, l) = sum_s sum_k conj(a[s][j](k, m)) dC[s][j](k, l), in int64
    std::vector<int64_t> want(72, 0);
    for (int64_t s = 0; s < sites; ++s)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k)
                for (int m = 0; m < 3; ++m)
                    for (int l = 0; l < 3; ++l) {
                        const size_t ia = 2 * (size_t)(((s * 4 + j) * 3 + k) * 3 + m);
                        const size_t ig = 2 * (size_t)(((s * 4 + j) * 3 + k) * 3 + l);
                        const int64_t ar = (int64_t)a[ia], ai = (int64_t)a[ia + 1];
                        const int64_t gr = (int64_t)dc[ig], gi = (int64_t)dc[ig + 1];
                        want[2 * (9 * j + 3 * m + l)] += ar * gr + ai * gi;
                        want[2 * (9 * j + 3 * m + l) + 1] += ar * gi - ai * gr;
                    }
    std::vector<double> db(72);
    HIP_OK(hipMemcpy(db.data(), d_db, 72 * sizeof(double), hipMemcpyDeviceToHost));
    for (int q = 0; q < 72; ++q)
        if (db[q] != (double)want[q]) {
            std::fprintf(stderr, "dB[%d] = %.17g, exact sum %lld\n", q, db[q], (long long)want[q]);
            return 7;
        }

    // The padded SoA layout: plane p at complex offset p * pitch. a -> SoA,
    // c = a b on the SoA planes, c -> site-major; with b = I that is a again.
    int64_t pitch = 0;
    SU3_OK_OR_FAIL(su3_soa_pitch(sites, SU3_F64, &pitch));
    if (pitch < sites) {
        std::fprintf(stderr, "pitch %lld < sites\n", (long long)pitch);
        return 8;
    }
    const size_t soa_bytes = (size_t)pitch * 36 * 2 * sizeof(double);
    double *d_sa, *d_sc;
    HIP_OK(hipMalloc((void **)&d_sa, soa_bytes));
    HIP_OK(hipMalloc((void **)&d_sc, soa_bytes));
    HIP_OK(hipMemsetAsync(d_c, 0, bytes, stream));
    SU3_OK_OR_FAIL(su3_aos_to_soa_pitched(d_a, d_sa, sites, pitch, SU3_F64, stream));
    SU3_OK_OR_FAIL(su3_mult_nn_soa_pitched(d_sa, d_b, d_sc, sites, pitch, SU3_F64, stream));
    SU3_OK_OR_FAIL(su3_soa_to_aos_pitched(d_sc, d_c, sites, pitch, SU3_F64, stream));
    HIP_OK(hipStreamSynchronize(stream));
    HIP_OK(hipMemcpy(out.data(), d_c, bytes, hipMemcpyDeviceToHost));
    if (std::memcmp(out.data(), a.data(), bytes) != 0) {
        std::fprintf(stderr, "padded SoA round trip of c = a b != a for b = I\n");
        return 9;
    }
    for (void *p : {(void *)d_a, (void *)d_b, (void *)d_c, (void *)d_dc, (void *)d_da, (void *)d_db, d_ws,
                    (void *)d_sa, (void *)d_sc})
        HIP_OK(hipFree(p));
    HIP_OK(hipStreamDestroy(stream));
    std::printf("ok: %lld sites, forward, adjoint (dA and dB) and padded SoA (pitch %lld) through the C ABI\n",
                (long long)sites, (long long)pitch);
    return 0;
}
