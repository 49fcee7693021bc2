/*
 * The C ABI used from plain C, with no Python: reads a graph ("n m" then m
 * lines "u v") from the file named by argv[1], and on the current HIP device
 *   1. solves it with cc_labels,
 *   2. solves it again with cc_labels_ex and opts.no_sync = 1 on its own
 *      stream, polling cc_stream_status until the work is done,
 *   3. solves two copies of it packed into one cc_labels_batch call,
 *   4. checks that an endpoint outside [0, n) gives CC_ERR_RANGE,
 * checks that 1-3 agree, and prints the labels of 1, one per line.
 * Exit status 0 on success.  Built by __graft_entry__.build().
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "hookcc.h"

#define HIP_OK(x)                                                            \
    do {                                                                     \
        if ((x) != hipSuccess) {                                             \
            fprintf(stderr, "HIP error at line %d\n", __LINE__);             \
            return 2;                                                        \
        }                                                                    \
    } while (0)
#define CC_OK_OR_FAIL(x)                                                     \
    do {                                                                     \
        int32_t rc_ = (x);                                                   \
        if (rc_ != CC_OK) {                                                  \
            fprintf(stderr, "line %d: status %d: %s\n", __LINE__, rc_, cc_last_error()); \
            return 3;                                                        \
        }                                                                    \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s graph.txt\n", argv[0]);
        return 1;
    }
    FILE* f = fopen(argv[1], "r");
    if (!f) return 1;
    long long n_in = 0, m_in = 0;
    if (fscanf(f, "%lld %lld", &n_in, &m_in) != 2 || n_in < 1 || m_in < 0) return 1;
    const int32_t n = (int32_t)n_in;
    const int64_t m = (int64_t)m_in;
    int32_t* hu = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(m + 1));
    int32_t* hv = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(m + 1));
    int32_t* h1 = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
    int32_t* h2 = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
    if (!hu || !hv || !h1 || !h2) return 1;
    for (int64_t i = 0; i < m; ++i) {
        int a, b;
        if (fscanf(f, "%d %d", &a, &b) != 2) return 1;
        hu[i] = a;
        hv[i] = b;
        hu[m + i] = a;  /* second copy for the batch: same local ids */
        hv[m + i] = b;
    }
    fclose(f);

    int32_t *du, *dv, *dout;
    HIP_OK(hipMalloc((void**)&du, sizeof(int32_t) * 2 * (size_t)(m + 1)));
    HIP_OK(hipMalloc((void**)&dv, sizeof(int32_t) * 2 * (size_t)(m + 1)));
    HIP_OK(hipMalloc((void**)&dout, sizeof(int32_t) * 2 * (size_t)n));
    HIP_OK(hipMemcpy(du, hu, sizeof(int32_t) * 2 * (size_t)m, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dv, hv, sizeof(int32_t) * 2 * (size_t)m, hipMemcpyHostToDevice));

    /* 1. synchronous solve */
    CC_OK_OR_FAIL(cc_labels(n, du, dv, m, dout));
    HIP_OK(hipMemcpy(h1, dout, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));

    /* 2. no-sync solve on a stream, status polled */
    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));
    HIP_OK(hipMemset(dout, 0xff, sizeof(int32_t) * (size_t)n));
    cc_options o;
    cc_options_init(&o);
    o.no_sync = 1;
    CC_OK_OR_FAIL(cc_labels_ex(n, du, dv, m, dout, &o, NULL, 0, (void*)s, NULL));
    int32_t st;
    while ((st = cc_stream_status((void*)s)) == CC_PENDING) {
    }
    CC_OK_OR_FAIL(st);
    HIP_OK(hipMemcpy(h2, dout, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    if (memcmp(h1, h2, sizeof(int32_t) * (size_t)n) != 0) {
        fprintf(stderr, "no-sync labels differ\n");
        return 4;
    }

    /* 3. two copies in one batch */
    int64_t vo[3] = {0, n, 2 * (int64_t)n};
    int64_t eo[3] = {0, m, 2 * m};
    CC_OK_OR_FAIL(cc_labels_batch(2, vo, eo, du, dv, dout));
    HIP_OK(hipMemcpy(h2, dout, sizeof(int32_t) * 2 * (size_t)n, hipMemcpyDeviceToHost));
    if (memcmp(h1, h2, sizeof(int32_t) * (size_t)n) != 0 ||
        memcmp(h1, h2 + n, sizeof(int32_t) * (size_t)n) != 0) {
        fprintf(stderr, "batch labels differ\n");
        return 5;
    }

    /* 4. an endpoint outside [0, n) */
    const int32_t bad = n;
    HIP_OK(hipMemcpy(du + 2 * m, &bad, sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dv + 2 * m, &bad, sizeof(int32_t), hipMemcpyHostToDevice));
    const int32_t rc = cc_labels(n, du + 2 * m, dv + 2 * m, 1, dout);
    if (rc != CC_ERR_RANGE || cc_last_error()[0] == '\0') {
        fprintf(stderr, "expected CC_ERR_RANGE, got %d\n", rc);
        return 6;
    }

    for (int32_t i = 0; i < n; ++i) printf("%d\n", h1[i]);
    HIP_OK(hipStreamDestroy(s));
    HIP_OK(hipFree(du));
    HIP_OK(hipFree(dv));
    HIP_OK(hipFree(dout));
    cc_release();
    free(hu);
    free(hv);
    free(h1);
    free(h2);
    return 0;
}
