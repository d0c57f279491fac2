/* A whole run through the C ABI from C, with device memory from hipMalloc and no PyTorch:
 * reads a two-star state (n, n1, params, then x y z vx vy vz as float arrays) from argv[1],
 * steps it argv[3] times in FP32 Kahan mode with the split request argv[4] (0 = the built-in
 * rule; see nb_tile_override) and band height argv[5], and writes the final positions and
 * velocities and the diagnostics
 * to argv[2]. Test infrastructure for tests/test_gpu_c_abi.py. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nbody.h"

#define CHECK(x)                                                         \
    do {                                                                 \
        int rc_ = (int)(x);                                              \
        if (rc_ != 0) {                                                  \
            fprintf(stderr, "%s failed: %d at line %d\n", #x, rc_, __LINE__); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 6) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[2];
    double prm[9];
    if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(prm, sizeof prm, 1, f) != 1) return 2;
    const int64_t n = hdr[0];
    if (n <= 0 || n > (1 << 24)) return 2;
    float *host = (float *)malloc((size_t)n * 6 * sizeof(float));
    if (!host || fread(host, sizeof(float), (size_t)n * 6, f) != (size_t)n * 6) return 2;
    fclose(f);

    nb_params p;
    memset(&p, 0, sizeof p);
    p.n = n;
    p.n1 = hdr[1];
    p.G = prm[0];
    p.m = prm[1];
    p.dt = prm[2];
    p.D1 = prm[3];
    p.D2 = prm[4];
    p.q = prm[5];
    p.a = prm[6];
    p.R2_0 = prm[7];
    p.growth_rate = prm[8];
    p.growth_on = 1;
    p.mode = NB_FP32_KAHAN;
    p.law = NB_LAW_CONTACT;

    CHECK(nb_tile_override(n, n, NB_FP32_KAHAN, NB_LAW_CONTACT, atoi(argv[4]), atoi(argv[5])));
    size_t scratch_bytes = 0;
    CHECK(nb_scratch_bytes(&p, &scratch_bytes));
    void *arr[9];
    for (int k = 0; k < 9; ++k) CHECK(hipMalloc(&arr[k], (size_t)n * sizeof(float)));
    void *side = NULL, *scratch = NULL;
    CHECK(hipMalloc(&side, (size_t)n));
    CHECK(hipMalloc(&scratch, scratch_bytes));  /* hipMalloc returns 256-byte aligned memory */
    for (int k = 0; k < 6; ++k) {
        CHECK(hipMemcpy(arr[k], host + (size_t)k * n, (size_t)n * sizeof(float),
                        hipMemcpyHostToDevice));
    }
    CHECK(hipMemset(side, 0, (size_t)n));
    hipStream_t st;
    CHECK(hipStreamCreate(&st));

    nb_buffers b;
    memset(&b, 0, sizeof b);
    b.x = arr[0];
    b.y = arr[1];
    b.z = arr[2];
    b.vx = arr[3];
    b.vy = arr[4];
    b.vz = arr[5];
    b.ax = arr[6];
    b.ay = arr[7];
    b.az = arr[8];
    b.side = side;
    b.scratch = scratch;
    b.scratch_bytes = scratch_bytes;
    nb_system *s = NULL;
    CHECK(nb_create(&p, &b, st, &s));
    CHECK(nb_step(&s, 1, atoi(argv[3]), st));
    nb_diag d;
    CHECK(nb_diagnostics(s, 1, &d, st));
    for (int k = 0; k < 6; ++k) {
        CHECK(hipMemcpy(host + (size_t)k * n, arr[k], (size_t)n * sizeof(float),
                        hipMemcpyDeviceToHost));
    }
    nb_destroy(s);
    CHECK(hipStreamDestroy(st));
    for (int k = 0; k < 9; ++k) CHECK(hipFree(arr[k]));
    CHECK(hipFree(side));
    CHECK(hipFree(scratch));

    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(host, sizeof(float), (size_t)n * 6, o);
    const double dv[4] = {d.KE, d.PE, d.D2, (double)d.step};
    fwrite(dv, sizeof dv, 1, o);
    fclose(o);
    free(host);
    return 0;
}
