// proxy_shade.hip -- the consumer side of the emission query: irradiance at
// shading points from the light leaving the luminaire's proxy box.
//
// The radiance leaving the proxy along a ray is the luminaire's emission
// plus the scene light behind it seen through the luminaire's transparency
// (Sec. 3, Eq. 2): L_o = L_e + (1 - alpha) L_b, with alpha the opacity the
// query returns (Sec. 4.1, Eq. 5) and L_b one background colour.  The proxy
// is sampled uniformly over its surface (Sec. 6, Sampling): face
// f = floor(6 u0) of the six faces of area 4, point (2 u1 - 1, 2 u2 - 1) on
// it, area density 1/24.  A sample on a face that the shading point does not
// see from the front, or below its tangent plane, weighs 0; otherwise
//     w = cos(theta_x) cos(theta_y) / (|y - x|^2 / 24),
// and the estimate is the mean of w L_o over the point's samples.
//
// Three stream-ordered steps: k_proxy_rays weighs every sample and lists the
// live ones (weight > 0) with their rays, the persistent emission query
// marches the listed rays only, k_proxy_reduce blends and sums per point in
// sample order (FP64 sums).  Listing first matters: rays that need no march
// interleaved with live ones would make the query's refills draw again and
// again from its shared ray counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "lq_internal.h"

namespace lq {
namespace {

constexpr int kShadeBlock = 256;
constexpr int kSamplesPerThread = 8;
constexpr int kSamplesPerBlock = kShadeBlock * kSamplesPerThread;
constexpr float kInvAreaDensity = 24.0f;   // total area of the faces of [-1,1]^3

__global__ void k_proxy_zero(unsigned long long *p) { p[0] = 0ull; }

// Samples j = blockIdx.x * kSamplesPerBlock + k * kShadeBlock + threadIdx.x
// (k < kSamplesPerThread) of the flattened [point][sample] grid: each
// sample's weight, and for the samples that weigh more than 0 (live) the ray
// and a place in the live list (one atomic per block).  Inside a block the
// live samples are listed grouped by the cell of the proxy they aim at (face
// x 4 x 4 cells), so that the rays one wave marches come from neighbouring
// shading points toward the same part of the luminaire.  The list's order
// (across blocks, and within a cell) is arbitrary; no ray's result depends
// on it.
constexpr int kCellsPerSide = 4;
constexpr int kAimCells = 6 * kCellsPerSide * kCellsPerSide;
__global__ __launch_bounds__(kShadeBlock) void k_proxy_rays(const float *points, const float *normals, int64_t m,
                                                            int S, const float *u, float *o, float *d, float *w,
                                                            int64_t *live, unsigned long long *n_live) {
    __shared__ unsigned s_cell[kAimCells];
    __shared__ unsigned long long s_base;
    for (int c = threadIdx.x; c < kAimCells; c += kShadeBlock) s_cell[c] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * kSamplesPerBlock + threadIdx.x;
    int cell[kSamplesPerThread];              // aim cell of a live sample, -1 for a dead one
    unsigned rank[kSamplesPerThread];         // its place among the block's samples of that cell
#pragma unroll
    for (int k = 0; k < kSamplesPerThread; ++k) {
        const int64_t j = j0 + (int64_t)k * kShadeBlock;
        cell[k] = -1;
        rank[k] = 0;
        if (j < m) {
            const int64_t i = j / S;
            const float x0 = points[3 * i], x1 = points[3 * i + 1], x2 = points[3 * i + 2];
            const float n0 = normals[3 * i], n1 = normals[3 * i + 1], n2 = normals[3 * i + 2];
            const float u0 = u[3 * j], u1 = u[3 * j + 1], u2 = u[3 * j + 2];
            int f = (int)(u0 * 6.0f);
            f = f < 0 ? 0 : (f > 5 ? 5 : f);
            const int axis = f >> 1;
            const float sgn = (f & 1) ? 1.0f : -1.0f;
            const float a = u1 * 2.0f - 1.0f, b = u2 * 2.0f - 1.0f;
            // the face point: sgn on `axis`, then a and b on the next two axes (cyclic)
            const float y0 = axis == 0 ? sgn : (axis == 1 ? b : a);
            const float y1 = axis == 1 ? sgn : (axis == 2 ? b : a);
            const float y2 = axis == 2 ? sgn : (axis == 0 ? b : a);
            const float d0 = y0 - x0, d1 = y1 - x1, d2 = y2 - x2;
            const float xa = axis == 0 ? x0 : (axis == 1 ? x1 : x2);
            const float h = sgn * xa - 1.0f;          // height of x in front of the face's plane
            const float dist2 = d0 * d0 + d1 * d1 + d2 * d2;
            const float nlen = sqrtf(n0 * n0 + n1 * n1 + n2 * n2);
            const float ndot = n0 * d0 + n1 * d1 + n2 * d2;
            float wt = 0.0f;
            if (h > 0.0f && ndot > 0.0f && dist2 > 0.0f && nlen > 0.0f) {
                const float dist = sqrtf(dist2);
                const float cos_x = ndot / (nlen * dist), cos_y = h / dist;
                wt = cos_x * cos_y / dist2 * kInvAreaDensity;
            }
            w[j] = wt;
            if (wt > 0.0f) {
                o[3 * j] = x0;
                o[3 * j + 1] = x1;
                o[3 * j + 2] = x2;
                d[3 * j] = d0;
                d[3 * j + 1] = d1;
                d[3 * j + 2] = d2;
                int ca = (int)((a + 1.0f) * (0.5f * kCellsPerSide));
                int cb = (int)((b + 1.0f) * (0.5f * kCellsPerSide));
                ca = ca < 0 ? 0 : (ca >= kCellsPerSide ? kCellsPerSide - 1 : ca);
                cb = cb < 0 ? 0 : (cb >= kCellsPerSide ? kCellsPerSide - 1 : cb);
                cell[k] = (f * kCellsPerSide + ca) * kCellsPerSide + cb;
                rank[k] = atomicAdd(&s_cell[cell[k]], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {                   // cell counts -> offsets in the block's part of the list
        unsigned tot = 0;
        for (int c = 0; c < kAimCells; ++c) {
            const unsigned n = s_cell[c];
            s_cell[c] = tot;
            tot += n;
        }
        s_base = tot ? atomicAdd(n_live, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSamplesPerThread; ++k)
        if (cell[k] >= 0) live[s_base + s_cell[cell[k]] + rank[k]] = j0 + (int64_t)k * kShadeBlock;
}

// Blend and per-point sums.  Block b takes points [b P, b P + P) with
// P = min(kShadeBlock, max(1, kReduceChunk / S)), so that their samples fit
// one chunk of kReduceChunk (a point with more samples is summed chunk by
// chunk).  The terms w (L_e + (1 - alpha) L_b) of a chunk are computed from
// coalesced loads into LDS; one thread per point then adds its terms in
// sample order (FP64 partial sums per chunk, added in chunk order): the same
// order for every launch.
constexpr int kReduceChunk = kSamplesPerBlock;

__global__ __launch_bounds__(kShadeBlock) void k_proxy_reduce(const float *rgb, const float *alpha, const float *w,
                                                              int64_t n_points, int S, int P, float b0, float b1,
                                                              float b2, float *irradiance, float *terms) {
    __shared__ float s_t[3][kReduceChunk];
    const int64_t p0 = (int64_t)blockIdx.x * P;
    const int np = (int)(n_points - p0 < P ? n_points - p0 : P);
    const int64_t span = (int64_t)np * S;            // samples of this block's points
    const int64_t j_first = p0 * S;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t c0 = 0; c0 < span; c0 += kReduceChunk) {
        const int len = (int)(span - c0 < kReduceChunk ? span - c0 : kReduceChunk);
        for (int t = threadIdx.x; t < len; t += kShadeBlock) {
            const int64_t j = j_first + c0 + t;
            const float wt = w[j];
            float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f;
            if (wt > 0.0f) {                      // only live samples were queried
                const float tr = 1.0f - alpha[j];
                t0 = wt * (rgb[3 * j] + tr * b0);
                t1 = wt * (rgb[3 * j + 1] + tr * b1);
                t2 = wt * (rgb[3 * j + 2] + tr * b2);
            }
            if (terms) {
                terms[3 * j] = t0;
                terms[3 * j + 1] = t1;
                terms[3 * j + 2] = t2;
            }
            s_t[0][t] = t0;
            s_t[1][t] = t1;
            s_t[2][t] = t2;
        }
        __syncthreads();
        if ((int)threadIdx.x < np) {             // thread q sums point p0 + q (P <= kShadeBlock)
            const int64_t q = threadIdx.x;
            // this point's samples within the chunk, in order
            const int64_t lo = q * S > c0 ? q * S : c0;
            const int64_t hi = q * S + S < c0 + len ? q * S + S : c0 + len;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int64_t k = lo; k < hi; ++k) {
                s0 += s_t[0][k - c0];
                s1 += s_t[1][k - c0];
                s2 += s_t[2][k - c0];
            }
            a0 += s0;
            a1 += s1;
            a2 += s2;
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < np) {
        const int64_t i = p0 + threadIdx.x;
        irradiance[3 * i] = (float)(a0 / S);
        irradiance[3 * i + 1] = (float)(a1 / S);
        irradiance[3 * i + 2] = (float)(a2 / S);
    }
}

lq_status shade_fail(lq_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" lq_status lq_proxy_irradiance(const lq_octree *tree, const float *points, const float *normals,
                                         int64_t n_points, const float *u, int32_t n_samples,
                                         const float *background_rgb, int model, float *irradiance,
                                         float *sample_terms, void *hip_stream) {
    if (!tree) return shade_fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    if (n_points < 0) return shade_fail(LQ_ERR_INVALID_ARG, "n_points must be >= 0");
    if (n_samples < 1 || n_samples > 65536) return shade_fail(LQ_ERR_INVALID_ARG, "n_samples must be in 1..65536");
    if (model != LQ_LINEAR && model != LQ_EXP) return shade_fail(LQ_ERR_INVALID_ARG, "model must be LQ_LINEAR or LQ_EXP");
    if (n_points > ((int64_t)1 << 36) / n_samples) return shade_fail(LQ_ERR_INVALID_ARG, "n_points * n_samples too large");
    if (n_points == 0) return LQ_OK;
    const float b0 = background_rgb ? background_rgb[0] : 0.0f;
    const float b1 = background_rgb ? background_rgb[1] : 0.0f;
    const float b2 = background_rgb ? background_rgb[2] : 0.0f;
    const int dev = octree_device(tree);
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return shade_fail(LQ_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    const int64_t m = n_points * n_samples;
    lq_status st;
    if ((st = check_device_array(points, (size_t)n_points * 12, dev, "points")) != LQ_OK) return st;
    if ((st = check_device_array(normals, (size_t)n_points * 12, dev, "normals")) != LQ_OK) return st;
    if ((st = check_device_array(u, (size_t)m * 12, dev, "u")) != LQ_OK) return st;
    if ((st = check_device_array(irradiance, (size_t)n_points * 12, dev, "irradiance")) != LQ_OK) return st;
    if (sample_terms && (st = check_device_array(sample_terms, (size_t)m * 12, dev, "sample_terms")) != LQ_OK)
        return st;
    hipStream_t s = (hipStream_t)hip_stream;
    // stream-ordered scratch: the live-ray counter (256 B), then per sample a
    // list slot (8 B), a ray (24 B), its weight (4 B), its radiance and opacity (16 B)
    unsigned char *buf = nullptr;
    if ((e = hipMallocAsync((void **)&buf, 256 + (size_t)m * 52, s)) != hipSuccess)
        return shade_fail(LQ_ERR_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    unsigned long long *n_live = reinterpret_cast<unsigned long long *>(buf);
    int64_t *live = reinterpret_cast<int64_t *>(buf + 256);
    float *o = reinterpret_cast<float *>(buf + 256 + (size_t)m * 8);
    float *d = o + 3 * m, *w = o + 6 * m, *rgb = o + 7 * m, *alpha = o + 10 * m;
    hipLaunchKernelGGL(k_proxy_zero, dim3(1), dim3(1), 0, s, n_live);
    hipLaunchKernelGGL(k_proxy_rays, dim3((unsigned)((m + kSamplesPerBlock - 1) / kSamplesPerBlock)),
                       dim3(kShadeBlock), 0, s, points, normals, m, (int)n_samples, u, o, d, w, live, n_live);
    e = hipGetLastError();
    st = LQ_OK;
    if (e != hipSuccess) {
        st = shade_fail(LQ_ERR_HIP, std::string("launching the proxy samples: ") + hipGetErrorString(e));
    } else {
        st = query_scratch(tree, o, d, m, live, n_live, rgb, alpha, model, s);
        if (st == LQ_OK) {
            const int P = n_samples >= kReduceChunk ? 1 : std::min(kShadeBlock, kReduceChunk / n_samples);
            hipLaunchKernelGGL(k_proxy_reduce, dim3((unsigned)((n_points + P - 1) / P)), dim3(kShadeBlock), 0, s,
                               rgb, alpha, w, n_points, (int)n_samples, P, b0, b1, b2, irradiance, sample_terms);
            if ((e = hipGetLastError()) != hipSuccess)
                st = shade_fail(LQ_ERR_HIP, std::string("launching the proxy reduction: ") + hipGetErrorString(e));
        }
    }
    hipError_t f = hipFreeAsync(buf, s);
    if (st == LQ_OK && f != hipSuccess) st = shade_fail(LQ_ERR_HIP, std::string("hipFreeAsync: ") + hipGetErrorString(f));
    return st;
}
