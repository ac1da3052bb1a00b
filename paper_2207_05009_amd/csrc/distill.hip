// distill.hip -- plenoctree distillation from a continuous radiance field
// (Sec. 5, "Creating the plenoctree"): one density sample at the centre of
// every voxel of the finest grid, pruning of the voxels whose centre density
// is below a threshold (0.01 in the paper), the mean density and mean SH
// coefficients of a number of uniformly random positions inside every voxel
// kept (256 in the paper: averaging against aliasing at discontinuities),
// and the octree over the kept voxels with its empty octants collapsed
// bottom-up.
//
// The field (the stand-in for a trained radiance field) is a sum of
// Gaussian blobs in log-density, clamped, with thin spherical shells of
// constant density; its SH emission coefficients are blended by the
// normalised blob weights w_k (a softmax of -|x - c_k|^2 / (2 r_k^2)): the
// DC coefficient is logit(E_c / L_max) / Y_00 with E_c = sum_k w_k e_kc, the
// others sum_k w_k h_kcj (lq_field_desc in include/lumiq.h).
//
// Kernels, stream-ordered:
//   k_centre_bits     voxels in Morton order, 64 per wave: the centre test
//                     in FP64 (its decision is an integer), one 64-bit
//                     ballot word per 64 voxels, a count per chunk;
//   k_scan_counts     exclusive scan of the chunk counts (one block);
//   k_centre_compact  the Morton codes of the kept voxels, ascending;
//   k_distill<NB>     one lane per kept voxel: n_samples positions from
//                     Philox4x32-10 (counter = code, sample index, 0, 0;
//                     key = seed), the blob exponents in FP64, their
//                     exponentials and the per-sample sums in float32 with
//                     every blob's weight kept in registers (NB >= blobs,
//                     fully unrolled), shell membership as in FP64 (a
//                     decision), and the means.  The higher SH coefficients
//                     are linear in the weights, so their mean is
//                     sum_k mean(w_k) h_k: the lane averages the NB weights
//                     and combines them with h once at the end (the same
//                     value as averaging the per-sample coefficients, in
//                     other rounding);
//   tree build        per level, bottom-up: run heads of the parent codes,
//                     a scan for the parents' positions, their compaction;
//                     then the child table, breadth-first, Morton order
//                     within a level.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lq_internal.h"

namespace lq {
namespace {

constexpr int kMaxBlobs = 32;
constexpr int kMaxShells = 8;
constexpr int kThreads = 256;
constexpr int kWordsPerChunk = 256;          // 64-bit occupancy words per chunk (16,384 voxels)
constexpr int kScanBlock = 1024;

// The field as kernel arguments: float32 copies for the samples, FP64 for
// the decisions (centre occupancy, shell membership).
struct FieldArgs {
    int nb, ns, K, pad;
    float cx[kMaxBlobs], cy[kMaxBlobs], cz[kMaxBlobs], inv2r2[kMaxBlobs], amp[kMaxBlobs];
    float cxl[kMaxBlobs], cyl[kMaxBlobs], czl[kMaxBlobs];     // centre = float32 + lower part
    float er[kMaxBlobs], eg[kMaxBlobs], eb[kMaxBlobs];
    float sx[kMaxShells], sy[kMaxShells], sz[kMaxShells], sr[kMaxShells];
    float sxl[kMaxShells], syl[kMaxShells], szl[kMaxShells];
    float log_base, sigma_max, l_max, half_width, threshold, pad2[3];
    double dcx[kMaxBlobs], dcy[kMaxBlobs], dcz[kMaxBlobs], dinv2r2[kMaxBlobs], damp[kMaxBlobs];
    double dsx[kMaxShells], dsy[kMaxShells], dsz[kMaxShells], dsr[kMaxShells];
    double dhalf_width, dthreshold;   // density(centre) >= prune  <=>  S >= dthreshold
};
static_assert(sizeof(FieldArgs) < 4000, "kernel argument space");

__device__ inline uint32_t compact3(uint32_t v) {   // every third bit, from bit 0
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Shell membership, decided as in FP64: a float32 distance first (centres
// as a float32 pair, so each difference is within 2 ulp of its own value;
// positions and centres within [-2, 2]: the distance is off by under
// 2e-6), and FP64 only when its margin to a shell boundary is below 1e-5.
__device__ inline bool in_shell_f64(const FieldArgs &f, int j, double x, double y, double z) {
    const double dx = x - f.dsx[j], dy = y - f.dsy[j], dz = z - f.dsz[j];
    const double dist = sqrt(dx * dx + dy * dy + dz * dz);
    return fabs(dist - f.dsr[j]) < f.dhalf_width;
}

__device__ inline bool in_shell(const FieldArgs &f, double x, double y, double z) {
    const float xf = (float)x, yf = (float)y, zf = (float)z;
    bool in = false;
    for (int j = 0; j < f.ns; ++j) {
        const float dx = (xf - f.sx[j]) - f.sxl[j], dy = (yf - f.sy[j]) - f.syl[j], dz = (zf - f.sz[j]) - f.szl[j];
        const float dist = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        const float m = fabsf(dist - f.sr[j]) - f.half_width;
        if (fabsf(m) > 1e-5f) in = in || m < 0.0f;
        else in = in || in_shell_f64(f, j, x, y, z);
    }
    return in;
}

__device__ inline bool centre_kept_f64(const FieldArgs &f, double x, double y, double z) {
    double S = 0.0;
    for (int k = 0; k < f.nb; ++k) {
        const double dx = x - f.dcx[k], dy = y - f.dcy[k], dz = z - f.dcz[k];
        const double d2 = dx * dx + dy * dy + dz * dz;
        S += f.damp[k] * exp(-d2 * f.dinv2r2[k]);
    }
    return S >= f.dthreshold;
}

// The centre test, decided as in FP64: S in float32 first, FP64 only when
// S_32 lies within 4e-3 of the threshold.  Bound: voxel centres are exact
// in float32 and blob centres are float32 pairs, so every difference, the
// squared distance and lw = -d^2 / (2 r^2) carry under 6 ulp of relative
// error, and exp2 one more: each term a g is off by under
// |a| (6 |lw| + 2) 2^-24 <= |a| (6 / e + 2) 2^-24 (g |lw| <= 1 / e), under
// 1.1e-4 for 32 blobs of |a| <= 12; the running sum adds under
// 32 2^-24 sum |a| g <= 7.4e-4.
__device__ inline bool centre_kept(const FieldArgs &f, double x, double y, double z) {
    if (in_shell(f, x, y, z)) return true;
    const float xf = (float)x, yf = (float)y, zf = (float)z;
    float S = 0.0f;
    for (int k = 0; k < f.nb; ++k) {
        const float dx = (xf - f.cx[k]) - f.cxl[k], dy = (yf - f.cy[k]) - f.cyl[k], dz = (zf - f.cz[k]) - f.czl[k];
        const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        S = fmaf(f.amp[k], __builtin_amdgcn_exp2f(-d2 * f.inv2r2[k] * 1.4426950408889634f), S);
    }
    const float m = S - f.threshold;
    if (fabsf(m) > 4e-3f) return m >= 0.0f;
    return centre_kept_f64(f, x, y, z);
}

// Occupancy of the voxels [chunk * kWordsPerChunk * 64, ...) in Morton
// order: bits[word] bit l = voxel 64 word + l kept; counts[chunk] = kept.
__global__ __launch_bounds__(kThreads) void k_centre_bits(const FieldArgs f, int depth, uint64_t n_vox,
                                                          unsigned long long *bits, uint32_t *counts) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double h = 2.0 / (double)(1 << depth);
    uint32_t cnt = 0;
    for (int it = wave; it < kWordsPerChunk; it += kThreads / 64) {
        const uint64_t word = (uint64_t)blockIdx.x * kWordsPerChunk + it;
        const uint64_t code = word * 64 + lane;
        bool kept = false;
        if (code < n_vox) {
            const uint32_t c = (uint32_t)code;
            const double x = -1.0 + ((double)compact3(c) + 0.5) * h;
            const double y = -1.0 + ((double)compact3(c >> 1) + 0.5) * h;
            const double z = -1.0 + ((double)compact3(c >> 2) + 0.5) * h;
            kept = centre_kept(f, x, y, z);
        }
        const unsigned long long m = __ballot(kept);
        if (word * 64 < n_vox && lane == 0) bits[word] = m;
        cnt += (uint32_t)__popcll(m);
    }
    if (lane == 0) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_cnt;
}

// Exclusive scan of n counts by one block; total in *total.
__global__ __launch_bounds__(kScanBlock) void k_scan_counts(const uint32_t *counts, uint32_t n, uint32_t *offsets,
                                                            uint32_t *total) {
    __shared__ uint32_t s[kScanBlock];
    const uint32_t per = (n + kScanBlock - 1) / kScanBlock;
    const uint32_t a = threadIdx.x * per, b = min(n, a + per);
    uint32_t sum = 0;
    for (uint32_t i = a; i < b; ++i) sum += counts[i];
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {   // Hillis-Steele, inclusive
        const uint32_t v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - sum;
    for (uint32_t i = a; i < b; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == kScanBlock - 1) *total = s[kScanBlock - 1];
}

// Codes of the kept voxels of a chunk at its offset, ascending.  Writes
// only below cap (the caller's capacity).
__global__ __launch_bounds__(kWordsPerChunk) void k_centre_compact(const unsigned long long *bits, uint64_t n_words,
                                                                   const uint32_t *offsets, uint32_t *codes,
                                                                   uint64_t cap) {
    __shared__ uint32_t s[kWordsPerChunk];
    const uint64_t word = (uint64_t)blockIdx.x * kWordsPerChunk + threadIdx.x;
    const unsigned long long m = word < n_words ? bits[word] : 0ull;
    const uint32_t c = (uint32_t)__popcll(m);
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kWordsPerChunk; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t pos = (uint64_t)offsets[blockIdx.x] + s[threadIdx.x] - c;
    unsigned long long r = m;
    while (r) {
        const int bit = __ffsll(r) - 1;
        r &= r - 1;
        if (pos < cap) codes[pos] = (uint32_t)(word * 64 + bit);
        ++pos;
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): 10 rounds of two
// 32x32 -> 64-bit multiplications with the key bumped by the Weyl constants.
// Each product is one 64-bit multiply (a single v_mad_u64_u32).
__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                     uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        c1 = (uint32_t)p1;
        c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// One lane per kept voxel i < n: the means over n_samples positions.
// sh_out[i][c][k]; hi [nb][3][K - 1] (device, FP64).  rec: NB records of
// four doubles (centre, -log2(e) / (2 r^2)), then NB float4 records
// (amplitude, radiance); those past nb are padded so that their terms
// vanish (exp2 of a huge negative argument is exactly 0).
//
// Precision: the exponent t_k = -log2(e) |x - c_k|^2 / (2 r_k^2) is taken in
// FP64 (full rate on this chip, like float32 without packing): a softmax
// weight depends on the absolute error of t_k - max_j t_j, and at points far
// from every blob (|t| in the hundreds, on the shells) float32 would leave
// relative errors of 1e-4 in the weights.  exp2, log2 and the per-sample
// sums are float32; the sums over samples run in blocks of kBlock samples
// (float32 inside a block, FP64 across blocks), and the higher coefficients
// sum_k mean(w_k) h_k are formed in FP64 once per voxel.
//
// The records are read inside the sample loop through an offset the
// compiler cannot prove constant (zero is 0), so they arrive by scalar
// loads from cache each sample instead of being held across the loop, where
// they would overflow the scalar register file; groups of four blobs are
// separated by scheduling barriers so that the loads are not all issued at
// once.  The Philox round keys are likewise recomputed by scalar adds.
constexpr int kBlock = 16;

template <int NB>
__global__ __launch_bounds__(kThreads) void k_distill(const FieldArgs f, const double *__restrict__ rec,
                                                      uint32_t zero, const double *hi, int depth, int n_samples,
                                                      uint32_t key0, uint32_t key1, const uint32_t *codes,
                                                      uint64_t n, float *sigma_out, float *sh_out) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t code = codes[i];
    const double hd = 2.0 / (double)(1 << depth);
    const double lox = -1.0 + (double)compact3(code) * hd;
    const double loy = -1.0 + (double)compact3(code >> 1) * hd;
    const double loz = -1.0 + (double)compact3(code >> 2) * hd;
    constexpr float kLog2e = 1.4426950408889634f;
    constexpr float kLn2InvY00 = 0.69314718055994531f * 3.5449077018110318f;
    const float log_base2 = f.log_base * kLog2e;
    double wsum[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) wsum[k] = 0.0;
    double sig_sum = 0.0, dc0_sum = 0.0, dc1_sum = 0.0, dc2_sum = 0.0;
    for (int j0 = 0; j0 < n_samples; j0 += kBlock) {
        const int j1 = min(n_samples, j0 + kBlock);
        float wb[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) wb[k] = 0.0f;
        float sig_acc = 0.0f, dc0 = 0.0f, dc1 = 0.0f, dc2 = 0.0f;
        for (int j = j0; j < j1; ++j) {
            const uint32_t jz = (uint32_t)j & zero;   // 0, opaque to the compiler
            const double4 *qa = reinterpret_cast<const double4 *>(rec) + jz;
            const float4 *qb = reinterpret_cast<const float4 *>(qa + NB);
            uint32_t u[4];
            philox4x32_10(code, (uint32_t)j, 0u, 0u, key0 + jz, key1 + jz, u);
            // the position exactly in FP64 (cell + offset: 34 bits)
            const double x = lox + (double)(u[0] >> 8) * 0x1p-24 * hd;
            const double y = loy + (double)(u[1] >> 8) * 0x1p-24 * hd;
            const double z = loz + (double)(u[2] >> 8) * 0x1p-24 * hd;
            // t_k = log2 of blob k's Gaussian, m = max_k t_k (FP64)
            double t[NB];
            double m = -INFINITY;
#pragma unroll
            for (int g = 0; g < NB; g += 4) {
#pragma unroll
                for (int k = g; k < g + 4; ++k) {
                    const double4 a = qa[k];
                    const double dx = x - a.x, dy = y - a.y, dz = z - a.z;
                    t[k] = fma(dz, dz, fma(dy, dy, dx * dx)) * a.w;
                    m = fmax(m, t[k]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            float e[NB];
            float s = 0.0f, sa = 0.0f, e0 = 0.0f, e1 = 0.0f, e2 = 0.0f;
#pragma unroll
            for (int g = 0; g < NB; g += 4) {
#pragma unroll
                for (int k = g; k < g + 4; ++k) {
                    const float4 b = qb[k];
                    e[k] = __builtin_amdgcn_exp2f((float)(t[k] - m));
                    s += e[k];
                    sa = fmaf(b.x, e[k], sa);
                    e0 = fmaf(b.y, e[k], e0);
                    e1 = fmaf(b.z, e[k], e1);
                    e2 = fmaf(b.w, e[k], e2);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            const float inv = __builtin_amdgcn_rcpf(s);
#pragma unroll
            for (int k = 0; k < NB; ++k) wb[k] = fmaf(e[k], inv, wb[k]);
            // density: exp(log_base + sum_k a_k g_k), sum_k a_k g_k = 2^m sa
            float sg = fminf(
                __builtin_amdgcn_exp2f(fmaf(__builtin_amdgcn_exp2f((float)m) * kLog2e, sa, log_base2)),
                f.sigma_max);
            if (f.ns > 0 && in_shell(f, x, y, z)) sg = f.sigma_max;
            sig_acc += sg;
            // DC: logit(E / L_max) / Y_00 = ln(E / (L_max - E)) 2 sqrt(pi),
            // E = e_c / s: log2(e_c / (L_max s - e_c)) ln 2 2 sqrt(pi)
            const float ls = f.l_max * s;
            dc0 = fmaf(__builtin_amdgcn_logf(e0 * __builtin_amdgcn_rcpf(ls - e0)), kLn2InvY00, dc0);
            dc1 = fmaf(__builtin_amdgcn_logf(e1 * __builtin_amdgcn_rcpf(ls - e1)), kLn2InvY00, dc1);
            dc2 = fmaf(__builtin_amdgcn_logf(e2 * __builtin_amdgcn_rcpf(ls - e2)), kLn2InvY00, dc2);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) wsum[k] += (double)wb[k];
        sig_sum += (double)sig_acc;
        dc0_sum += (double)dc0;
        dc1_sum += (double)dc1;
        dc2_sum += (double)dc2;
    }
    const double invn = 1.0 / (double)n_samples;
    sigma_out[i] = (float)(sig_sum * invn);
    const int K = f.K;
    float *row = sh_out + i * (uint64_t)(3 * K);
    row[0] = (float)(dc0_sum * invn);
    row[K] = (float)(dc1_sum * invn);
    row[2 * K] = (float)(dc2_sum * invn);
    for (int c = 0; c < 3; ++c)
        for (int j = 1; j < K; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (k < f.nb) acc = fma(wsum[k], hi[(k * 3 + c) * (K - 1) + (j - 1)], acc);
            row[c * K + j] = (float)(acc * invn);
        }
}

// ---- octree build (bottom-up collapse) ---------------------------------
// generic exclusive scan of n uint32 values (n < 2^31): block sums, one
// block scanning them, per-block scans plus the block's offset
__global__ __launch_bounds__(kScanBlock) void k_block_sums(const uint32_t *v, uint64_t n, uint32_t *sums) {
    __shared__ uint32_t s[kScanBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
    s[threadIdx.x] = i < n ? v[i] : 0u;
    __syncthreads();
    for (int off = kScanBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kScanBlock) void k_block_scan(const uint32_t *v, uint64_t n, const uint32_t *block_off,
                                                           uint32_t *out) {
    __shared__ uint32_t s[kScanBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const uint32_t x = i < n ? v[i] : 0u;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const uint32_t y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < n) out[i] = block_off[blockIdx.x] + s[threadIdx.x] - x;
}

// run heads of the parent codes of a sorted level
__global__ void k_parent_heads(const uint32_t *kids, uint64_t n, uint32_t *head) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = (i == 0 || (kids[i] >> 3) != (kids[i - 1] >> 3)) ? 1u : 0u;
}

// parents[pos[i]] = kids[i] >> 3 at run heads; pidx[i] = the parent's position
__global__ void k_parent_compact(const uint32_t *kids, uint64_t n, const uint32_t *head, const uint32_t *pos,
                                 uint32_t *parents, uint32_t *pidx) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = pos[i] + head[i] - 1u;   // inclusive count of heads, minus one
    pidx[i] = p;
    if (head[i]) parents[p] = kids[i] >> 3;
}

// codes strictly ascending and below 8^depth?  (flag set on a violation)
__global__ void k_check_codes(const uint32_t *codes, uint64_t n, uint64_t limit, uint32_t *bad) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (codes[i] >= limit || (i > 0 && codes[i] <= codes[i - 1])) atomicOr(bad, 1u);
}

__global__ void k_child_write(const uint32_t *kids, uint64_t n, const uint32_t *pidx, int32_t base_parent,
                              int32_t base_kids, int leaves, int32_t *child) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = leaves ? -(int32_t)(i + 1) : base_kids + (int32_t)i;
    child[(uint64_t)(base_parent + (int32_t)pidx[i]) * 8u + (kids[i] & 7u)] = v;
}

__global__ void k_fill_i32(int32_t *p, uint64_t n, int32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

lq_status dfail(lq_status s, const std::string &m) {
    set_error(m);
    return s;
}
lq_status dhip(hipError_t e, const char *what) {
    return dfail(LQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device buffers freed at scope exit (after the stream is synchronised).
struct DevBufs {
    std::vector<void *> p;
    ~DevBufs() {
        for (void *q : p) (void)hipFree(q);
    }
    template <class T>
    hipError_t alloc(T **out, size_t count) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) p.push_back(q);
        *out = static_cast<T *>(q);
        return e;
    }
};

// exclusive scan of v[0..n) into out (device), total on the host
hipError_t scan_u32(const uint32_t *v, uint64_t n, uint32_t *out, uint32_t *total_host, DevBufs &b, hipStream_t s) {
    const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
    uint32_t *sums, *offs, *tot;
    hipError_t e;
    if ((e = b.alloc(&sums, nb)) != hipSuccess || (e = b.alloc(&offs, nb)) != hipSuccess ||
        (e = b.alloc(&tot, 1)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(kScanBlock), 0, s, v, n, sums);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kScanBlock), 0, s, sums, (uint32_t)nb, offs, tot);
    hipLaunchKernelGGL(k_block_scan, dim3((unsigned)nb), dim3(kScanBlock), 0, s, v, n, offs, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(total_host, tot, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

lq_status field_args(const lq_field_desc *fd, int depth, float prune_sigma, FieldArgs &f) {
    if (!fd) return dfail(LQ_ERR_INVALID_ARG, "field is NULL");
    if (fd->n_blobs < 1 || fd->n_blobs > kMaxBlobs) return dfail(LQ_ERR_UNSUPPORTED, "n_blobs must be in [1, 32]");
    if (fd->n_shells < 0 || fd->n_shells > kMaxShells) return dfail(LQ_ERR_UNSUPPORTED, "n_shells must be in [0, 8]");
    if (fd->sh_degree < 0 || fd->sh_degree > 4) return dfail(LQ_ERR_UNSUPPORTED, "sh_degree must be in [0, 4]");
    if (depth < 1 || depth > 10) return dfail(LQ_ERR_INVALID_ARG, "max_depth must be in [1, 10]");
    if (!(prune_sigma > 0.0f) || !std::isfinite(prune_sigma)) return dfail(LQ_ERR_INVALID_ARG, "prune_sigma must be > 0");
    if (!fd->blobs || (fd->n_shells && !fd->shells)) return dfail(LQ_ERR_INVALID_ARG, "field arrays are NULL");
    const int K = (fd->sh_degree + 1) * (fd->sh_degree + 1);
    if (K > 1 && !fd->blob_sh) return dfail(LQ_ERR_INVALID_ARG, "blob_sh is NULL");
    if (!(fd->l_max > 0.0) || !(fd->sigma_max > 0.0) || !std::isfinite(fd->log_density_base) ||
        !(fd->shell_half_width >= 0.0))
        return dfail(LQ_ERR_INVALID_ARG, "bad field scalars");
    memset(&f, 0, sizeof(f));
    f.nb = fd->n_blobs;
    f.ns = fd->n_shells;
    f.K = K;
    for (int k = 0; k < f.nb; ++k) {
        const double *b = fd->blobs + 8 * k;
        if (!(b[3] >= 1e-3 && b[3] <= 4.0) || !std::isfinite(b[0] + b[1] + b[2] + b[4]) || std::fabs(b[0]) > 2.0 ||
            std::fabs(b[1]) > 2.0 || std::fabs(b[2]) > 2.0 || std::fabs(b[4]) > 12.0)
            return dfail(LQ_ERR_INVALID_ARG,
                         "a blob needs a centre in [-2, 2]^3, a radius in [1e-3, 4] and |amplitude| <= 12");
        for (int c = 0; c < 3; ++c)
            if (!(b[5 + c] > 0.0) || !(b[5 + c] < fd->l_max))
                return dfail(LQ_ERR_INVALID_ARG, "blob radiance must be in (0, l_max)");
        const double inv = 1.0 / (2.0 * b[3] * b[3]);
        f.dcx[k] = b[0];
        f.dcy[k] = b[1];
        f.dcz[k] = b[2];
        f.dinv2r2[k] = inv;
        f.damp[k] = b[4];
        f.cx[k] = (float)b[0];
        f.cy[k] = (float)b[1];
        f.cz[k] = (float)b[2];
        f.cxl[k] = (float)(b[0] - (double)f.cx[k]);
        f.cyl[k] = (float)(b[1] - (double)f.cy[k]);
        f.czl[k] = (float)(b[2] - (double)f.cz[k]);
        f.inv2r2[k] = (float)inv;
        f.amp[k] = (float)b[4];
        f.er[k] = (float)b[5];
        f.eg[k] = (float)b[6];
        f.eb[k] = (float)b[7];
    }
    for (int j = 0; j < f.ns; ++j) {
        for (int a = 0; a < 4; ++a)
            if (!std::isfinite(fd->shells[4 * j + a]) || std::fabs(fd->shells[4 * j + a]) > 2.0)
                return dfail(LQ_ERR_INVALID_ARG, "shell centres and radii must lie in [-2, 2]");
        f.dsx[j] = fd->shells[4 * j];
        f.dsy[j] = fd->shells[4 * j + 1];
        f.dsz[j] = fd->shells[4 * j + 2];
        f.dsr[j] = fd->shells[4 * j + 3];
        f.sx[j] = (float)f.dsx[j];
        f.sy[j] = (float)f.dsy[j];
        f.sz[j] = (float)f.dsz[j];
        f.sr[j] = (float)f.dsr[j];
        f.sxl[j] = (float)(f.dsx[j] - (double)f.sx[j]);
        f.syl[j] = (float)(f.dsy[j] - (double)f.sy[j]);
        f.szl[j] = (float)(f.dsz[j] - (double)f.sz[j]);
    }
    f.dhalf_width = fd->shell_half_width;
    f.half_width = (float)fd->shell_half_width;
    f.dthreshold = log((double)prune_sigma) - fd->log_density_base;
    f.threshold = (float)f.dthreshold;
    f.log_base = (float)fd->log_density_base;
    f.sigma_max = (float)fd->sigma_max;
    f.l_max = (float)fd->l_max;
    return LQ_OK;
}


// The sample loop's blob records (k_distill), as bytes: NB x {cx, cy, cz,
// -log2(e) / (2 r^2)} in FP64, then NB x {amplitude, radiance} in float32;
// the records past nb sit far outside the field with a huge falloff, so
// their exp2 terms are exactly 0, and their amplitude and radiance are 0.
std::vector<unsigned char> blob_records(const FieldArgs &f, int NB) {
    std::vector<unsigned char> r((size_t)NB * 48, 0);
    for (int k = 0; k < NB; ++k) {
        double q[4] = {1000.0, 1000.0, 1000.0, -1e300};
        float w[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (k < f.nb) {
            q[0] = f.dcx[k], q[1] = f.dcy[k], q[2] = f.dcz[k];
            q[3] = -f.dinv2r2[k] * 1.4426950408889634;
            w[0] = f.amp[k], w[1] = f.er[k], w[2] = f.eg[k], w[3] = f.eb[k];
        }
        memcpy(r.data() + 32 * k, q, 32);
        memcpy(r.data() + 32 * NB + 16 * k, w, 16);
    }
    return r;
}

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" {

lq_status lq_distill_leaves(const lq_field_desc *field, int32_t max_depth, float prune_sigma, int32_t n_samples,
                            uint64_t seed, int device, int64_t capacity, uint32_t *codes, float *sigma, float *sh,
                            int64_t *n_leaves, void *hip_stream) {
    if (!n_leaves) return dfail(LQ_ERR_INVALID_ARG, "n_leaves is NULL");
    *n_leaves = 0;
    FieldArgs f;
    lq_status st = field_args(field, max_depth, prune_sigma, f);
    if (st != LQ_OK) return st;
    if (n_samples < 1 || n_samples > (1 << 20)) return dfail(LQ_ERR_INVALID_ARG, "n_samples must be in [1, 2^20]");
    if (capacity < 0) return dfail(LQ_ERR_INVALID_ARG, "capacity must be >= 0");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return dhip(e, "hipSetDevice");
    const int K = f.K;
    if (capacity > 0) {
        if ((st = check_device_array(codes, (size_t)capacity * 4, device, "codes")) != LQ_OK) return st;
        if ((st = check_device_array(sigma, (size_t)capacity * 4, device, "sigma")) != LQ_OK) return st;
        if ((st = check_device_array(sh, (size_t)capacity * 12 * K, device, "sh")) != LQ_OK) return st;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const uint64_t n_vox = 1ull << (3 * max_depth);
    const uint64_t n_words = (n_vox + 63) / 64;
    const uint64_t n_chunks = (n_words + kWordsPerChunk - 1) / kWordsPerChunk;
    DevBufs b;
    unsigned long long *bits;
    uint32_t *counts, *offs, *tot;
    double *d_hi = nullptr;
    if ((e = b.alloc(&bits, n_words)) != hipSuccess || (e = b.alloc(&counts, n_chunks)) != hipSuccess ||
        (e = b.alloc(&offs, n_chunks)) != hipSuccess || (e = b.alloc(&tot, 1)) != hipSuccess)
        return dfail(LQ_ERR_OOM, "device scratch of the distillation");
    if (K > 1) {
        const size_t nh = (size_t)f.nb * 3 * (K - 1);
        if ((e = b.alloc(&d_hi, nh)) != hipSuccess) return dfail(LQ_ERR_OOM, "device copy of blob_sh");
        if ((e = hipMemcpy(d_hi, field->blob_sh, nh * 8, hipMemcpyHostToDevice)) != hipSuccess)
            return dhip(e, "copying blob_sh");
    }
    hipLaunchKernelGGL(k_centre_bits, dim3((unsigned)n_chunks), dim3(kThreads), 0, s, f, max_depth, n_vox, bits,
                       counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kScanBlock), 0, s, counts, (uint32_t)n_chunks, offs, tot);
    if ((e = hipGetLastError()) != hipSuccess) return dhip(e, "launching the centre test");
    uint32_t total = 0;
    if ((e = hipMemcpyAsync(&total, tot, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return dhip(e, "the centre test");
    *n_leaves = total;
    if (capacity == 0 || total == 0) return LQ_OK;
    if ((int64_t)total > capacity) return dfail(LQ_ERR_INVALID_ARG, "more kept voxels than capacity (n_leaves set)");
    hipLaunchKernelGGL(k_centre_compact, dim3((unsigned)n_chunks), dim3(kWordsPerChunk), 0, s, bits, n_words, offs,
                       codes, (uint64_t)capacity);
    const unsigned nb = (unsigned)((total + kThreads - 1) / kThreads);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int NB = f.nb <= 8 ? 8 : f.nb <= 16 ? 16 : 32;
    std::vector<unsigned char> rec = blob_records(f, NB);
    double *d_rec;
    if ((e = b.alloc(&d_rec, rec.size() / 8)) != hipSuccess) return dfail(LQ_ERR_OOM, "device copy of the blobs");
    if ((e = hipMemcpy(d_rec, rec.data(), rec.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return dhip(e, "copying the blobs");
    if (NB == 8)
        hipLaunchKernelGGL(k_distill<8>, dim3(nb), dim3(kThreads), 0, s, f, d_rec, 0u, d_hi, max_depth, n_samples,
                           k0, k1, codes, (uint64_t)total, sigma, sh);
    else if (NB == 16)
        hipLaunchKernelGGL(k_distill<16>, dim3(nb), dim3(kThreads), 0, s, f, d_rec, 0u, d_hi, max_depth, n_samples,
                           k0, k1, codes, (uint64_t)total, sigma, sh);
    else
        hipLaunchKernelGGL(k_distill<32>, dim3(nb), dim3(kThreads), 0, s, f, d_rec, 0u, d_hi, max_depth, n_samples,
                           k0, k1, codes, (uint64_t)total, sigma, sh);
    if ((e = hipGetLastError()) != hipSuccess) return dhip(e, "launching the distillation");
    // the scratch above is freed on return: wait for its last use
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return dhip(e, "the distillation");
    return LQ_OK;
}

lq_status lq_octree_from_leaves(int32_t max_depth, int32_t sh_degree, const uint32_t *codes, const float *sigma,
                                const float *sh, int64_t n_leaves, float l_max, float sigma_min, float alpha_max,
                                int storage, int device, lq_octree **out) {
    if (!out) return dfail(LQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_depth < 1 || max_depth > 10) return dfail(LQ_ERR_INVALID_ARG, "max_depth must be in [1, 10]");
    if (sh_degree < 0 || sh_degree > 4) return dfail(LQ_ERR_INVALID_ARG, "sh_degree must be in [0, 4]");
    if (n_leaves < 0 || n_leaves > (int64_t)1 << 30) return dfail(LQ_ERR_INVALID_ARG, "n_leaves out of range");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return dhip(e, "hipSetDevice");
    const int K = (sh_degree + 1) * (sh_degree + 1);
    lq_status st;
    if (n_leaves > 0) {
        if ((st = check_device_array(codes, (size_t)n_leaves * 4, device, "codes")) != LQ_OK) return st;
        if ((st = check_device_array(sigma, (size_t)n_leaves * 4, device, "sigma")) != LQ_OK) return st;
        if ((st = check_device_array(sh, (size_t)n_leaves * 12 * K, device, "sh")) != LQ_OK) return st;
    }
    hipStream_t s = nullptr;
    DevBufs b;
    const uint64_t n = (uint64_t)n_leaves;
    const unsigned tb = 256;
    auto grid = [&](uint64_t m) { return dim3((unsigned)std::max<uint64_t>(1, (m + tb - 1) / tb)); };
    if (n > 0) {
        uint32_t *bad;
        if ((e = b.alloc(&bad, 1)) != hipSuccess) return dfail(LQ_ERR_OOM, "device scratch");
        uint32_t hbad = 0;
        if ((e = hipMemcpy(bad, &hbad, 4, hipMemcpyHostToDevice)) != hipSuccess) return dhip(e, "scratch");
        hipLaunchKernelGGL(k_check_codes, grid(n), dim3(tb), 0, s, codes, n, 1ull << (3 * max_depth), bad);
        if ((e = hipMemcpy(&hbad, bad, 4, hipMemcpyDeviceToHost)) != hipSuccess) return dhip(e, "checking codes");
        if (hbad) return dfail(LQ_ERR_FORMAT, "codes must be strictly ascending Morton codes below 8^max_depth");
    }
    // levels bottom-up: level[max_depth] = the leaves' codes
    std::vector<const uint32_t *> level(max_depth + 1, nullptr);
    std::vector<uint32_t *> pidx(max_depth + 1, nullptr);
    std::vector<uint64_t> count(max_depth + 1, 0);
    level[max_depth] = codes;
    count[max_depth] = n;
    for (int l = max_depth - 1; l >= 0; --l) {
        const uint64_t m = count[l + 1];
        if (m == 0) {
            count[l] = l == 0 ? 1 : 0;
            continue;
        }
        uint32_t *head, *pos, *par, *pi;
        if ((e = b.alloc(&head, m)) != hipSuccess || (e = b.alloc(&pos, m)) != hipSuccess ||
            (e = b.alloc(&par, m)) != hipSuccess || (e = b.alloc(&pi, m)) != hipSuccess)
            return dfail(LQ_ERR_OOM, "device scratch of the octree build");
        hipLaunchKernelGGL(k_parent_heads, grid(m), dim3(tb), 0, s, level[l + 1], m, head);
        uint32_t total = 0;
        if ((e = scan_u32(head, m, pos, &total, b, s)) != hipSuccess) return dhip(e, "scanning a level");
        hipLaunchKernelGGL(k_parent_compact, grid(m), dim3(tb), 0, s, level[l + 1], m, head, pos, par, pi);
        level[l] = par;
        pidx[l + 1] = pi;
        count[l] = total;
    }
    // the root always exists (level 0 holds code 0 when any leaf exists)
    count[0] = 1;
    std::vector<int64_t> base(max_depth + 1, 0);
    int64_t n_nodes = 0;
    for (int l = 0; l < max_depth; ++l) {
        base[l] = n_nodes;
        n_nodes += (int64_t)count[l];
    }
    if (n_nodes >= (1 << 29)) return dfail(LQ_ERR_UNSUPPORTED, "too many nodes");
    int32_t *child;
    if ((e = b.alloc(&child, (size_t)n_nodes * 8)) != hipSuccess) return dfail(LQ_ERR_OOM, "device child table");
    hipLaunchKernelGGL(k_fill_i32, grid((uint64_t)n_nodes * 8), dim3(tb), 0, s, child, (uint64_t)n_nodes * 8, 0);
    for (int l = 0; l < max_depth; ++l) {
        const uint64_t m = count[l + 1];
        if (m == 0 || !pidx[l + 1]) continue;
        hipLaunchKernelGGL(k_child_write, grid(m), dim3(tb), 0, s, level[l + 1], m, pidx[l + 1], (int32_t)base[l],
                           (int32_t)base[l + 1], l + 1 == max_depth ? 1 : 0, child);
    }
    if ((e = hipGetLastError()) != hipSuccess) return dhip(e, "launching the octree build");
    // the device table and leaves become an octree through the loader
    // (validation, storage conversion, the sigma_min-pruned table, top grids)
    std::vector<int32_t> hchild((size_t)n_nodes * 8);
    std::vector<float> hsig(n), hsh(n * 3 * K);
    if ((e = hipMemcpy(hchild.data(), child, hchild.size() * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (n && (e = hipMemcpy(hsig.data(), sigma, n * 4, hipMemcpyDeviceToHost)) != hipSuccess) ||
        (n && (e = hipMemcpy(hsh.data(), sh, n * 12 * K, hipMemcpyDeviceToHost)) != hipSuccess))
        return dhip(e, "reading the built octree");
    lq_octree_desc d;
    d.max_depth = max_depth;
    d.sh_degree = sh_degree;
    d.n_nodes = (int32_t)n_nodes;
    d.n_leaves = (int32_t)n;
    d.l_max = l_max;
    d.sigma_min = sigma_min;
    d.alpha_max = alpha_max;
    d.child = hchild.data();
    d.sigma = hsig.data();
    d.sh = hsh.data();
    return lq_load_octree_desc(&d, storage, device, out);
}

}  // extern "C"
