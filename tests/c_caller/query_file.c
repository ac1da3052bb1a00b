/*
 * A plain C caller of liblumiq: no torch, no C++, the system HIP runtime.
 * It shows that the C ABI of include/lumiq.h is complete on its own for the
 * emission query (Sec. 4.1, Eqs. 3-5): the caller owns every device buffer,
 * the library owns the tree.
 *
 *   query_file TREE STORAGE RAYS N OUT
 *     TREE     plenoctree file (magic "LQOT", the loader's format)
 *     STORAGE  0 float32, 1 float16, 2 bfloat16
 *     RAYS     float32 origins[N][3] then directions[N][3], little-endian
 *     OUT      written: rgb[N][3] then alpha[N], float32, from
 *              lq_query_radiance (linear model, default flags)
 *
 * Besides the query it checks, and reports through its exit status, that
 * host pointers are refused with LQ_ERR_INVALID_ARG and that the
 * allocation-free entry point returns the same bits.  Exit status: 0 done,
 * 1 usage or file error, 2 library or HIP error, 3 a check failed.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "lumiq.h"

#define HIP_OK(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
            return 2;                                                         \
        }                                                                     \
    } while (0)

#define LQ_OK_OR(call)                                                        \
    do {                                                                      \
        lq_status s_ = (call);                                                \
        if (s_ != LQ_OK) {                                                    \
            fprintf(stderr, "%s: status %d\n", #call, (int)s_);               \
            return 2;                                                         \
        }                                                                     \
    } while (0)

static int run(const char *tree_path, int storage, const char *rays_path, int64_t n, const char *out_path) {
    const size_t vec_bytes = (size_t)n * 3 * sizeof(float);
    float *host = malloc(2 * vec_bytes + vec_bytes + (size_t)n * sizeof(float) + vec_bytes + (size_t)n * sizeof(float));
    if (!host) return 1;
    float *h_o = host, *h_d = host + 3 * n, *h_rgb = host + 6 * n, *h_alpha = host + 9 * n;
    float *h_rgb2 = host + 10 * n, *h_alpha2 = host + 13 * n;
    FILE *f = fopen(rays_path, "rb");
    if (!f) { perror(rays_path); return 1; }
    const size_t got = fread(host, 1, 2 * vec_bytes, f);
    fclose(f);
    if (got != 2 * vec_bytes) { fprintf(stderr, "short ray file\n"); return 1; }

    lq_octree *tree = NULL;
    LQ_OK_OR(lq_load_octree(tree_path, storage, 0, &tree));
    int64_t dev_bytes = 0;
    int32_t nn = 0, nl = 0, depth = 0, deg = 0, st = -1;
    LQ_OK_OR(lq_octree_info(tree, &dev_bytes, &nn, &nl, &depth, &deg, &st));
    printf("[c] tree: %d nodes, %d leaves, depth %d, SH degree %d, storage %d, %lld device bytes\n", nn, nl, depth,
           deg, st, (long long)dev_bytes);
    if (st != storage) { fprintf(stderr, "storage %d reported as %d\n", storage, st); return 3; }

    float *d_o, *d_d, *d_rgb, *d_alpha;
    HIP_OK(hipMalloc((void **)&d_o, vec_bytes));
    HIP_OK(hipMalloc((void **)&d_d, vec_bytes));
    HIP_OK(hipMalloc((void **)&d_rgb, vec_bytes));
    HIP_OK(hipMalloc((void **)&d_alpha, (size_t)n * sizeof(float)));
    HIP_OK(hipMemcpy(d_o, h_o, vec_bytes, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_d, h_d, vec_bytes, hipMemcpyHostToDevice));
    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));

    /* host buffers are refused before anything is launched */
    const lq_status bad = lq_query_radiance(tree, h_o, h_d, n, d_rgb, d_alpha, LQ_LINEAR, 0, s);
    if (bad != LQ_ERR_INVALID_ARG) { fprintf(stderr, "host origins: status %d\n", (int)bad); return 3; }

    LQ_OK_OR(lq_query_radiance(tree, d_o, d_d, n, d_rgb, d_alpha, LQ_LINEAR, 0, s));
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(h_rgb, d_rgb, vec_bytes, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_alpha, d_alpha, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));

    /* the allocation-free entry point: the same bits */
    LQ_OK_OR(lq_query_radiance_noalloc(tree, d_o, d_d, n, d_rgb, d_alpha, LQ_LINEAR, 0, s));
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(h_rgb2, d_rgb, vec_bytes, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_alpha2, d_alpha, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
    if (memcmp(h_rgb, h_rgb2, vec_bytes) || memcmp(h_alpha, h_alpha2, (size_t)n * sizeof(float))) {
        fprintf(stderr, "the allocation-free query differs\n");
        return 3;
    }

    f = fopen(out_path, "wb");
    if (!f) { perror(out_path); return 1; }
    const size_t put = fwrite(h_rgb, 1, vec_bytes, f) + fwrite(h_alpha, 1, (size_t)n * sizeof(float), f);
    fclose(f);
    if (put != vec_bytes + (size_t)n * sizeof(float)) return 1;

    HIP_OK(hipStreamDestroy(s));
    HIP_OK(hipFree(d_o));
    HIP_OK(hipFree(d_d));
    HIP_OK(hipFree(d_rgb));
    HIP_OK(hipFree(d_alpha));
    lq_free_octree(tree);
    free(host);
    printf("[c] %lld rays done\n", (long long)n);
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 6) {
        fprintf(stderr, "usage: %s TREE STORAGE RAYS N OUT\n", argv[0]);
        return 1;
    }
    const int storage = atoi(argv[2]);
    const long long n = atoll(argv[4]);
    if (storage < 0 || storage > 2 || n <= 0 || n > (1ll << 30)) {   /* host buffers: 56 B per ray */
        fprintf(stderr, "bad storage or count\n");
        return 1;
    }
    const int rc = run(argv[1], storage, argv[3], (int64_t)n, argv[5]);
    fflush(stdout);
    return rc;
}
