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
// Guided sampling (cdf != null): the sample picks a cell of the faces its
// point sees from the front (the others contribute nothing), the face by
// guide mass mixed with the face-centre geometry and the cell by the face's
// table (guide_cell below); u1, u2 give the point in the cell, and the
// weight divides by the cell's area density.
struct Guide {
    const double *cdf;    // [D^2][n_cells + 1], or null: uniform sampling
    const double *prob;   // [D^2][n_cells]
    int G, n_cells, D;    // D x D direction bins per cell
    float step;           // 2 / G (float32)
    double area;          // (2 / G)^2
};

// Tangent bin 0..D-1 of a direction with tangent component v and squared
// length l2: the number of thresholds 2 j / D - 1 (j = 1..D-1) that
// v / sqrt(l2) reaches, decided on squares in FP64 (no square root).
__device__ inline int direction_bin(double v, double l2, int D) {
    int i = 0;
    for (int j = 1; j < D; ++j) {
        const double th = (2.0 * j) / D - 1.0;
        bool ok;
        if (th < 0.0) ok = v >= 0.0 || v * v <= (th * th) * l2;
        else if (th == 0.0) ok = v >= 0.0;
        else ok = v >= 0.0 && v * v >= (th * th) * l2;
        i = ok ? j : i;
    }
    return i;
}

// Bin i1 D + i2 of an outward direction w through a face of axis a: i1, i2
// the tangent bins of its components on axes a + 1 and a + 2 (cyclic); the
// squared length summed in axis order.
__device__ inline int face_direction_bin(int a, double w0, double w1, double w2, int D) {
    const double l2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double t1 = a == 0 ? w1 : (a == 1 ? w2 : w0);
    const double t2 = a == 0 ? w2 : (a == 1 ? w0 : w1);
    return direction_bin(t1, l2, D) * D + direction_bin(t2, l2, D);
}

constexpr double kFaceMix = 0.5;   // share of the face choice weighted by the face-centre geometry

// Picks the cell of a guided sample.  The point x (normal n) sees the faces
// with side * x_axis > 1.  On face f it uses table b_f, the direction bin
// of x - c_f (c_f the face's centre); P_f = cdf_b_f[(f + 1) G^2] -
// cdf_b_f[f G^2] is the face's guide mass, P_vis their sum,
// g_f = max(0, n.(c_f - x)) (side x_axis - 1) / |c_f - x|^4 the irradiance
// integrand cos cos / r^2 at the face centre (up to the constant 1/|n|)
// and S the sum of P_f g_f.  Face f is taken with probability
// Q_f = kFaceMix P_f g_f / S + (1 - kFaceMix) P_f / P_vis (P_f / P_vis when
// S = 0), the cell within it by inverting its table.  All of it in FP64
// from the float32 inputs, sums in axis and face order, so that the choice
// is reproducible bit for bit.  Returns the cell (-1 when no face is visible
// or P_vis = 0), its table in `bin` and Q_f / P_f in `factor`: the
// sample's area density is prob_bin[k] factor / A_cell.
template <bool DIR>
__device__ inline int guide_cell(const Guide &g, float x0, float x1, float x2, float n0, float n1, float n2,
                                 float u0, int &bin, double &factor) {
    const int gg = g.G * g.G;
    const int stride = g.n_cells + 1;
    const double xd[3] = {(double)x0, (double)x1, (double)x2};
    const double nd[3] = {(double)n0, (double)n1, (double)n2};
    bool vis[6];
    int fb[6];
    double P[6], Q[6], gf[6];
    double pv = 0.0, gs = 0.0;
    int last = -1;
    factor = 0.0;
    bin = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int ax = f >> 1;
        const float xa = ax == 0 ? x0 : (ax == 1 ? x1 : x2);
        vis[f] = ((f & 1) ? xa : -xa) > 1.0f;
        P[f] = 0.0;
        gf[f] = 0.0;
        fb[f] = 0;
        if (vis[f]) {
            const double sg = (f & 1) ? 1.0 : -1.0;
            double d[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) d[b] = (b == ax ? sg : 0.0) - xd[b];
            // the outward direction x - c_f is -d
            if constexpr (DIR) fb[f] = face_direction_bin(ax, -d[0], -d[1], -d[2], g.D);
            const double *c = g.cdf + (size_t)fb[f] * stride;
            P[f] = c[(f + 1) * gg] - c[f * gg];
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double ndot = nd[0] * d[0] + nd[1] * d[1] + nd[2] * d[2];
            const double h = sg * xd[ax] - 1.0;
            gf[f] = ndot > 0.0 ? (ndot * h) / (r2 * r2) : 0.0;
            pv += P[f];
            gs += P[f] * gf[f];
            last = f;
        }
    }
    if (!(pv > 0.0)) return -1;
#pragma unroll
    for (int f = 0; f < 6; ++f)
        Q[f] = !vis[f] ? 0.0
                       : (gs > 0.0 ? kFaceMix * (P[f] * gf[f] / gs) + (1.0 - kFaceMix) * (P[f] / pv) : P[f] / pv);
    double t = (double)u0;
    for (int f = 0; f < 6; ++f) {
        if (!vis[f]) continue;
        if (t < Q[f] || f == last) {
            const double *c = g.cdf + (size_t)fb[f] * stride;
            const double r = Q[f] > 0.0 ? t / Q[f] : 0.0;
            const double target = c[f * gg] + r * P[f];
            int lo = f * gg, hi = f * gg + gg - 1;   // c[lo] <= target holds for lo = f gg
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (c[mid] <= target) lo = mid;
                else hi = mid - 1;
            }
            factor = P[f] > 0.0 ? Q[f] / P[f] : 0.0;
            bin = fb[f];
            return lo;
        }
        t -= Q[f];
    }
    return -1;
}

// DIR: a direction-binned guide (D > 1); the direction-averaged and the
// uniform samplers are compiled without the bin decisions.
template <bool DIR>
__global__ __launch_bounds__(kShadeBlock) void k_proxy_rays(const float *points, const float *normals, int64_t m,
                                                            int S, const float *u, float *o, float *d, float *w,
                                                            int64_t *live, unsigned long long *n_live,
                                                            const Guide g) {
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
            int f;
            float a, b, inv_density = kInvAreaDensity;
            if (g.cdf) {
                double factor = 0.0;
                int bin = 0;
                int k = guide_cell<DIR>(g, x0, x1, x2, n0, n1, n2, u0, bin, factor);
                const double pa = k >= 0 ? g.prob[(size_t)bin * g.n_cells + k] * factor / g.area : 0.0;
                inv_density = pa > 0.0 ? (float)(1.0 / pa) : 0.0f;
                k = k < 0 ? 0 : k;                    // a dead sample: any cell, weight 0
                const int gg = g.G * g.G;
                f = k / gg;
                const int ca = (k / g.G) % g.G, cb = k % g.G;
                a = ((float)ca + u1) * g.step - 1.0f;
                b = ((float)cb + u2) * g.step - 1.0f;
            } else {
                f = (int)(u0 * 6.0f);
                f = f < 0 ? 0 : (f > 5 ? 5 : f);
                a = u1 * 2.0f - 1.0f;
                b = u2 * 2.0f - 1.0f;
            }
            const int axis = f >> 1;
            const float sgn = (f & 1) ? 1.0f : -1.0f;
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
            if (h > 0.0f && ndot > 0.0f && dist2 > 0.0f && nlen > 0.0f && inv_density > 0.0f) {
                const float dist = sqrtf(dist2);
                const float cos_x = ndot / (nlen * dist), cos_y = h / dist;
                wt = cos_x * cos_y / dist2 * inv_density;
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

// Probe rays of the guide: probe j of cell c = j / R starts at a uniform
// point of the cell (u0, u1) and aims at a uniform point of the box (u2..u4).
__global__ void k_guide_rays(int G, int R, int64_t n, const float *u, float step, float *o, float *d) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int c = (int)(j / R);
    const int gg = G * G;
    const int f = c / gg, ca = (c / G) % G, cb = c % G;
    const int axis = f >> 1;
    const float sgn = (f & 1) ? 1.0f : -1.0f;
    const float *uj = u + 5 * j;
    const float a = ((float)ca + uj[0]) * step - 1.0f;
    const float b = ((float)cb + uj[1]) * step - 1.0f;
    const float y0 = axis == 0 ? sgn : (axis == 1 ? b : a);
    const float y1 = axis == 1 ? sgn : (axis == 2 ? b : a);
    const float y2 = axis == 2 ? sgn : (axis == 0 ? b : a);
    const float t0 = uj[2] * 2.0f - 1.0f, t1 = uj[3] * 2.0f - 1.0f, t2 = uj[4] * 2.0f - 1.0f;
    o[3 * j] = y0;
    o[3 * j + 1] = y1;
    o[3 * j + 2] = y2;
    d[3 * j] = t0 - y0;
    d[3 * j + 1] = t1 - y1;
    d[3 * j + 2] = t2 - y2;
}

// Guide weights, D^2 per cell (cell-major), one wave per cell: per bin, the
// mean luminance (channel mean) of the cell's probes whose outward direction
// -d falls in the bin, summed in FP64 (each lane over its probes in order,
// then the lanes by a fixed butterfly: deterministic); a bin none of them
// fell in takes the mean over all R probes (D = 1: that mean alone).
constexpr int kGuideReduceBlock = 256;

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline double probe_luminance(const float *rgb, int64_t j) {
    const float *q = rgb + 3 * j;
    return ((double)q[0] + (double)q[1] + (double)q[2]) / 3.0;
}

__global__ __launch_bounds__(kGuideReduceBlock) void k_guide_reduce(const float *rgb, const float *d, int R,
                                                                    int n_cells, int G, int D, float *weights) {
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t c = (int64_t)blockIdx.x * (kGuideReduceBlock / 64) + (threadIdx.x >> 6);
    if (c >= n_cells) return;   // wave-uniform: the shuffles below see whole waves
    const int nb = D * D;
    const int a = (int)(c / ((int64_t)G * G)) >> 1;
    const int64_t j0 = c * R;
    double tot = 0.0;
    for (int r = lane; r < R; r += 64) tot += probe_luminance(rgb, j0 + r);
    tot = wave_sum_f64(tot);
    for (int b = 0; b < nb; ++b) {
        double s = 0.0, cnt = 0.0;
        if (D > 1) {
            for (int r = lane; r < R; r += 64) {
                const float *dj = d + 3 * (j0 + r);
                if (face_direction_bin(a, -(double)dj[0], -(double)dj[1], -(double)dj[2], D) == b) {
                    s += probe_luminance(rgb, j0 + r);
                    cnt += 1.0;
                }
            }
        }
        s = wave_sum_f64(s);
        cnt = wave_sum_f64(cnt);
        if (lane == 0) weights[c * nb + b] = (float)(cnt > 0.0 ? s / cnt : tot / R);
    }
}

// The cell probabilities and their running sums, in cell order (FP64):
// W = sum w, p_k = (1 - beta) (w_k / W) + beta / n (1 / n each when W = 0),
// cdf[0] = 0, cdf[k + 1] = cdf[k] + p_k.  The sums are sequential (their
// order fixes the FP64 results); one block stages the weights in LDS chunk
// by chunk with coalesced loads, computes a chunk's p_k in parallel, and
// thread 0 runs the sums over LDS.
constexpr int kCdfBlock = 256;
constexpr int kCdfChunk = 2048;   // cells staged in LDS at a time

// a cell's weight as the table uses it: negative, NaN and infinite weights
// count as 0
__device__ inline double guide_weight(float w) { return w > 0.0f && w < INFINITY ? (double)w : 0.0; }

__global__ __launch_bounds__(kCdfBlock) void k_guide_cdf(const float *weights, int n, int D, double beta, double *prob,
                                                         double *cdf) {
    __shared__ double s_v[kCdfChunk];
    __shared__ double s_W;
    const int t = threadIdx.x;
    const int nb = D * D, b = blockIdx.x;   // block b builds the table of direction bin b
    prob += (size_t)b * n;
    cdf += (size_t)b * (n + 1);
    double W = 0.0;   // thread 0 only
    for (int c0 = 0; c0 < n; c0 += kCdfChunk) {
        const int m = min(kCdfChunk, n - c0);
        for (int i = t; i < m; i += kCdfBlock) s_v[i] = guide_weight(weights[(size_t)(c0 + i) * nb + b]);
        __syncthreads();
        if (t == 0)
            for (int i = 0; i < m; ++i) W += s_v[i];
        __syncthreads();
    }
    if (t == 0) {
        s_W = W;
        cdf[0] = 0.0;
    }
    __syncthreads();
    W = s_W;
    double run = 0.0;   // thread 0 only
    for (int c0 = 0; c0 < n; c0 += kCdfChunk) {
        const int m = min(kCdfChunk, n - c0);
        for (int i = t; i < m; i += kCdfBlock) {
            const double p =
                W > 0.0 ? (1.0 - beta) * (guide_weight(weights[(size_t)(c0 + i) * nb + b]) / W) + beta / n : 1.0 / n;
            prob[c0 + i] = p;
            s_v[i] = p;
        }
        __syncthreads();
        if (t == 0)
            for (int i = 0; i < m; ++i) {
                run += s_v[i];
                s_v[i] = run;
            }
        __syncthreads();
        for (int i = t; i < m; i += kCdfBlock) cdf[c0 + i + 1] = s_v[i];
        __syncthreads();
    }
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

namespace lq {
namespace {

lq_status proxy_common(const lq_octree *tree, const float *points, const float *normals, int64_t n_points,
                       const float *u, int32_t n_samples, const float *weights, int32_t grid, int32_t dir_res,
                       float defensive,
                       const float *background_rgb, int model, float *irradiance, float *sample_terms,
                       void *hip_stream) {
    if (!tree) return shade_fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    if (n_points < 0) return shade_fail(LQ_ERR_INVALID_ARG, "n_points must be >= 0");
    if (n_samples < 1 || n_samples > 65536) return shade_fail(LQ_ERR_INVALID_ARG, "n_samples must be in 1..65536");
    if (model != LQ_LINEAR && model != LQ_EXP) return shade_fail(LQ_ERR_INVALID_ARG, "model must be LQ_LINEAR or LQ_EXP");
    if (n_points > ((int64_t)1 << 36) / n_samples) return shade_fail(LQ_ERR_INVALID_ARG, "n_points * n_samples too large");
    const bool guided = weights != nullptr;
    if (guided && (grid < 1 || grid > 256)) return shade_fail(LQ_ERR_INVALID_ARG, "grid must be in 1..256");
    if (guided && (dir_res < 1 || dir_res > 4)) return shade_fail(LQ_ERR_INVALID_ARG, "dir_res must be in 1..4");
    if (guided && !(defensive >= 0.0f && defensive <= 1.0f))
        return shade_fail(LQ_ERR_INVALID_ARG, "defensive must be in [0, 1]");
    if (n_points == 0) return LQ_OK;
    const float b0 = background_rgb ? background_rgb[0] : 0.0f;
    const float b1 = background_rgb ? background_rgb[1] : 0.0f;
    const float b2 = background_rgb ? background_rgb[2] : 0.0f;
    const int dev = octree_device(tree);
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return shade_fail(LQ_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    const int64_t m = n_points * n_samples;
    const int n_cells = guided ? 6 * grid * grid : 0;
    const int n_bins = guided ? dir_res * dir_res : 0;
    lq_status st;
    if ((st = check_device_array(points, (size_t)n_points * 12, dev, "points")) != LQ_OK) return st;
    if ((st = check_device_array(normals, (size_t)n_points * 12, dev, "normals")) != LQ_OK) return st;
    if ((st = check_device_array(u, (size_t)m * 12, dev, "u")) != LQ_OK) return st;
    if ((st = check_device_array(irradiance, (size_t)n_points * 12, dev, "irradiance")) != LQ_OK) return st;
    if (sample_terms && (st = check_device_array(sample_terms, (size_t)m * 12, dev, "sample_terms")) != LQ_OK)
        return st;
    if (guided && (st = check_device_array(weights, (size_t)n_cells * n_bins * 4, dev, "weights")) != LQ_OK)
        return st;
    hipStream_t s = (hipStream_t)hip_stream;
    // stream-ordered scratch: the live-ray counter (256 B), then per sample a
    // list slot (8 B), a ray (24 B), its weight (4 B), its radiance and
    // opacity (16 B); guided, the cell probabilities and running sums of
    // every direction bin
    const size_t guide_bytes = guided ? (size_t)n_bins * (2 * n_cells + 1) * 8 : 0;
    const size_t guide_at = (256 + (size_t)m * 52 + 255) & ~(size_t)255;   // 8-byte (here 256) aligned
    unsigned char *buf = nullptr;
    if ((e = hipMallocAsync((void **)&buf, guide_at + guide_bytes, s)) != hipSuccess)
        return shade_fail(LQ_ERR_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    unsigned long long *n_live = reinterpret_cast<unsigned long long *>(buf);
    int64_t *live = reinterpret_cast<int64_t *>(buf + 256);
    float *o = reinterpret_cast<float *>(buf + 256 + (size_t)m * 8);
    float *d = o + 3 * m, *w = o + 6 * m, *rgb = o + 7 * m, *alpha = o + 10 * m;
    Guide g{};
    if (guided) {
        double *gd = reinterpret_cast<double *>(buf + guide_at);
        g.prob = gd;
        g.cdf = gd + (size_t)n_bins * n_cells;
        g.G = grid;
        g.n_cells = n_cells;
        g.D = dir_res;
        g.step = (float)(2.0 / grid);
        g.area = (2.0 / grid) * (2.0 / grid);
        hipLaunchKernelGGL(k_guide_cdf, dim3((unsigned)n_bins), dim3(kCdfBlock), 0, s, weights, n_cells, dir_res,
                           (double)defensive,
                           const_cast<double *>(g.prob), const_cast<double *>(g.cdf));
    }
    hipLaunchKernelGGL(k_proxy_zero, dim3(1), dim3(1), 0, s, n_live);
    {
        auto kern = guided && dir_res > 1 ? k_proxy_rays<true> : k_proxy_rays<false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)((m + kSamplesPerBlock - 1) / kSamplesPerBlock)), dim3(kShadeBlock), 0,
                           s, points, normals, m, (int)n_samples, u, o, d, w, live, n_live, g);
    }
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

}  // namespace
}  // namespace lq

extern "C" lq_status lq_proxy_irradiance(const lq_octree *tree, const float *points, const float *normals,
                                         int64_t n_points, const float *u, int32_t n_samples,
                                         const float *background_rgb, int model, float *irradiance,
                                         float *sample_terms, void *hip_stream) {
    return proxy_common(tree, points, normals, n_points, u, n_samples, nullptr, 0, 1, 0.0f, background_rgb, model,
                        irradiance, sample_terms, hip_stream);
}

extern "C" lq_status lq_proxy_irradiance_guided(const lq_octree *tree, const float *points, const float *normals,
                                                int64_t n_points, const float *u, int32_t n_samples,
                                                const float *weights, int32_t grid, int32_t dir_res,
                                                float defensive, const float *background_rgb, int model,
                                                float *irradiance, float *sample_terms, void *hip_stream) {
    if (!weights) return shade_fail(LQ_ERR_INVALID_ARG, "weights is NULL");
    return proxy_common(tree, points, normals, n_points, u, n_samples, weights, grid, dir_res, defensive,
                        background_rgb, model, irradiance, sample_terms, hip_stream);
}

extern "C" lq_status lq_proxy_guide(const lq_octree *tree, int32_t grid, int32_t dir_res, int32_t n_probes,
                                    const float *u_probe, int model, float *weights, void *hip_stream) {
    if (!tree) return shade_fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    if (grid < 1 || grid > 256) return shade_fail(LQ_ERR_INVALID_ARG, "grid must be in 1..256");
    if (dir_res < 1 || dir_res > 4) return shade_fail(LQ_ERR_INVALID_ARG, "dir_res must be in 1..4");
    if (n_probes < 1 || n_probes > 65536) return shade_fail(LQ_ERR_INVALID_ARG, "n_probes must be in 1..65536");
    if (model != LQ_LINEAR && model != LQ_EXP) return shade_fail(LQ_ERR_INVALID_ARG, "model must be LQ_LINEAR or LQ_EXP");
    const int dev = octree_device(tree);
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return shade_fail(LQ_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    const int n_cells = 6 * grid * grid;
    const int64_t n = (int64_t)n_cells * n_probes;
    lq_status st;
    if ((st = check_device_array(u_probe, (size_t)n * 20, dev, "u_probe")) != LQ_OK) return st;
    if ((st = check_device_array(weights, (size_t)n_cells * dir_res * dir_res * 4, dev, "weights")) != LQ_OK)
        return st;
    hipStream_t s = (hipStream_t)hip_stream;
    float *buf = nullptr;    // probe rays (24 B) and their radiance (12 B)
    if ((e = hipMallocAsync((void **)&buf, (size_t)n * 36, s)) != hipSuccess)
        return shade_fail(LQ_ERR_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    float *o = buf, *d = buf + 3 * n, *rgb = buf + 6 * n;
    hipLaunchKernelGGL(k_guide_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, grid, n_probes, n, u_probe,
                       (float)(2.0 / grid), o, d);
    st = LQ_OK;
    if ((e = hipGetLastError()) != hipSuccess) {
        st = shade_fail(LQ_ERR_HIP, std::string("launching the guide probes: ") + hipGetErrorString(e));
    } else {
        st = query_scratch(tree, o, d, n, nullptr, nullptr, rgb, nullptr, model, s);
        if (st == LQ_OK) {
            constexpr int cells_per_block = kGuideReduceBlock / 64;
            hipLaunchKernelGGL(k_guide_reduce, dim3((unsigned)((n_cells + cells_per_block - 1) / cells_per_block)),
                               dim3(kGuideReduceBlock), 0, s, rgb, d, n_probes, n_cells, grid, dir_res, weights);
            if ((e = hipGetLastError()) != hipSuccess)
                st = shade_fail(LQ_ERR_HIP, std::string("launching the guide reduction: ") + hipGetErrorString(e));
        }
    }
    hipError_t f = hipFreeAsync(buf, s);
    if (st == LQ_OK && f != hipSuccess) st = shade_fail(LQ_ERR_HIP, std::string("hipFreeAsync: ") + hipGetErrorString(f));
    return st;
}
