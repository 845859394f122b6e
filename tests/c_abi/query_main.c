/* A plain C caller of the TPA C ABI (include/tpa.h), with no Python or torch:
 * build an R-MAT graph, preprocess it, run a batched query and a batch of
 * single-seed queries for the seeds given on the command line, and write the
 * outputs (float32, seed-major [k][n], first the batched rows, then the
 * single-seed rows) to a file.
 *
 * usage: query_main <scale> <samples> <rmat seed> <c> <S> <T> <out file> <seed>...
 * Device memory comes from hipMalloc; every call's status is checked, and a
 * failure prints tpa_last_error_message and exits with status 1. */
#include <stdio.h>
#include <stdlib.h>

#include "tpa.h"

#define CHECK_TPA(call)                                                                   \
    do {                                                                                  \
        tpa_status s_ = (call);                                                           \
        if (s_ != TPA_OK) {                                                               \
            fprintf(stderr, "%s: %s: %s\n", #call, tpa_status_string(s_), tpa_last_error_message()); \
            exit(1);                                                                      \
        }                                                                                 \
    } while (0)

#define CHECK_HIP(call)                                                        \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));         \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

int main(int argc, char **argv) {
    if (argc < 9) {
        fprintf(stderr, "usage: %s scale samples rmat_seed c S T out_file seed...\n", argv[0]);
        return 2;
    }
    const int scale = atoi(argv[1]);
    const int64_t samples = strtoll(argv[2], NULL, 0);
    const uint64_t rseed = strtoull(argv[3], NULL, 0);
    const double c = atof(argv[4]);
    const int S = atoi(argv[5]), T = atoi(argv[6]);
    const char *path = argv[7];
    const int64_t k = argc - 8;
    int32_t *seeds_h = (int32_t *)malloc(sizeof(int32_t) * k);
    for (int64_t j = 0; j < k; ++j) seeds_h[j] = (int32_t)atoi(argv[8 + j]);

    tpa_graph_t g = NULL;
    CHECK_TPA(tpa_graph_rmat(scale, 0, samples, rseed, 0.57, 0.19, 0.19, NULL, &g));
    int64_t n = 0, m = 0;
    CHECK_TPA(tpa_graph_info(g, &n, &m, NULL));
    CHECK_TPA(tpa_preprocess(g, c, T, NULL));

    int32_t *seeds_d = NULL;
    float *out_d = NULL;
    CHECK_HIP(hipMalloc((void **)&seeds_d, sizeof(int32_t) * k));
    CHECK_HIP(hipMalloc((void **)&out_d, sizeof(float) * 2 * k * n));
    CHECK_HIP(hipMemcpy(seeds_d, seeds_h, sizeof(int32_t) * k, hipMemcpyHostToDevice));
    CHECK_TPA(tpa_query(g, seeds_d, k, c, S, T, out_d, NULL));
    for (int64_t j = 0; j < k; ++j) CHECK_TPA(tpa_query(g, seeds_d + j, 1, c, S, T, out_d + (k + j) * n, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    CHECK_TPA(tpa_get_device_error(g, NULL));

    float *out_h = (float *)malloc(sizeof(float) * 2 * k * n);
    CHECK_HIP(hipMemcpy(out_h, out_d, sizeof(float) * 2 * k * n, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(out_h, sizeof(float), (size_t)(2 * k * n), f) != (size_t)(2 * k * n)) {
        fprintf(stderr, "cannot write %s\n", path);
        return 1;
    }
    fclose(f);
    printf("n=%lld m=%lld k=%lld\n", (long long)n, (long long)m, (long long)k);
    CHECK_HIP(hipFree(seeds_d));
    CHECK_HIP(hipFree(out_d));
    CHECK_TPA(tpa_graph_destroy(g));
    free(out_h);
    free(seeds_h);
    return 0;
}
