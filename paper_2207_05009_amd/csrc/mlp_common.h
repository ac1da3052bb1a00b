// mlp_common.h -- shapes, parameter layout and device helpers of the
// learned surrogate (a Fourier-feature MLP that stands in for the octree
// march on incoherent shading queries).
//
//   ray -> x6 = (e / sqrt(3), d/|d|), e = near hit of the ray's line with the
//          sphere of radius sqrt(3) that bounds the proxy box (the 5D light
//          field coordinates of Sec. 3, Eq. 1)
//   x6  -> 126 Fourier features [v, sin(2^k pi v), cos(2^k pi v)]_{k<10}
//          (the positional encoding of Sec. 4.2), zero padded to 128
//   128 -> 64 -> 64 -> 64 -> 64 (ReLU) -> 3: y = log(L + 1e-2)
//
// Parameters (float32 master copy) are one flat vector: per layer W[out][in]
// row-major, then b[out].  The GEMMs run on MFMA in bfloat16 with float32
// accumulation; their operands are a bfloat16 image of the weights (W[out][in]
// with the last layer padded to 16 rows) and bfloat16 activations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lq {
namespace mlp {

constexpr int kFeat = 128;          // 126 features + 2 zeros
constexpr int kFeatUsed = 126;
constexpr int kHidden = 64;
constexpr int kOut = 3;
constexpr int kOutPad = 16;
constexpr int kFreq = 10;
constexpr float kEpsOut = 1e-2f;    // L = exp(y) - kEpsOut
constexpr float kLossEps = 1e-2f;   // Eq. 8 regulariser
constexpr float kR2 = 3.0f;         // squared radius of the bounding sphere

// flat parameter offsets
constexpr int kW1 = 0, kB1 = kW1 + kHidden * kFeat;            // 8192
constexpr int kW2 = kB1 + kHidden, kB2 = kW2 + kHidden * kHidden;
constexpr int kW3 = kB2 + kHidden, kB3 = kW3 + kHidden * kHidden;
constexpr int kW4 = kB3 + kHidden, kB4 = kW4 + kHidden * kHidden;
constexpr int kW5 = kB4 + kHidden, kB5 = kW5 + kOut * kHidden;
constexpr int kParams = kB5 + kOut;                              // 20931

constexpr int kBiasPad = 4 * kHidden + kOutPad;                  // 272 floats

// trust map: octahedral 32x32 cells for the entry direction and for the ray
// direction (1,048,576 bins)
constexpr int kOctRes = 32;
constexpr int kTrustBins = kOctRes * kOctRes * kOctRes * kOctRes;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline uint16_t f2bf(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __host__ inline float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// D += A * B for 16x16x16 blocks (bf16 in, f32 accumulate).  Lane l holds
//   a[i] = A[l % 16][4 (l / 16) + i],  b[i] = B[4 (l / 16) + i][l % 16],
//   d[i] = D[4 (l / 16) + i][l % 16].
__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// sphere parameterisation of the line o + t d; returns false on a miss
// (a direction whose squared length is zero -- also by underflow -- or not
// finite, or a line that misses the sphere).  x6 is
// written in every case, branch-free; after a miss its values mean nothing
// and need not be finite.  Hardware reciprocal square root and square root,
// within a few units in the last place: the features are rounded to
// bfloat16 afterwards.
__device__ inline bool sphere_x6(const float *o, const float *d, float *x6) {
    const float dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const float inv = __builtin_amdgcn_rsqf(dd);
    const float dn0 = d[0] * inv, dn1 = d[1] * inv, dn2 = d[2] * inv;
    const float b = o[0] * dn0 + o[1] * dn1 + o[2] * dn2;
    const float c = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - kR2;
    const float disc = b * b - c;
    const float t = -b - __builtin_amdgcn_sqrtf(fmaxf(disc, 0.0f));
    const float s = 0.57735026918962576f;   // 1 / sqrt(3)
    x6[0] = (o[0] + t * dn0) * s;
    x6[1] = (o[1] + t * dn1) * s;
    x6[2] = (o[2] + t * dn2) * s;
    x6[3] = dn0;
    x6[4] = dn1;
    x6[5] = dn2;
    return dd > 0.0f && isfinite(dd) && disc > 0.0f;
}

// Which path answers a ray of the hybrid query.  The network models the
// radiance of a whole line (the chord of the proxy box it crosses), keyed by
// where the line enters the bounding sphere; a ray sees that whole chord
// only when the sphere -- and so the box inside it -- lies wholly ahead of
// its origin.  kRouteZero: the line misses the sphere, or the sphere lies
// wholly behind the origin (radiance 0, as the octree gives).  kRouteOctree:
// the origin is inside the sphere (it may be inside the box, or see a part
// of the chord only).  kRouteNet: the sphere lies ahead.
enum { kRouteNet = 0, kRouteOctree = 1, kRouteZero = 2 };

__device__ inline int sphere_route(const float *o, const float *d, float *x6) {
    if (!sphere_x6(o, d, x6)) return kRouteZero;
    const float c = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - kR2;
    const float od = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    if (!(c > 0.0f)) return kRouteOctree;
    // outside the sphere, both crossings lie on the side where o.d < 0
    return od < 0.0f ? kRouteNet : kRouteZero;
}

// octahedral cell (0..kOctRes^2-1) of a unit vector
__device__ inline int oct_cell(float x, float y, float z) {
    const float s = fabsf(x) + fabsf(y) + fabsf(z);
    float u = x / s, v = y / s;
    if (z < 0.0f) {
        const float uu = (1.0f - fabsf(v)) * (u >= 0.0f ? 1.0f : -1.0f);
        const float vv = (1.0f - fabsf(u)) * (v >= 0.0f ? 1.0f : -1.0f);
        u = uu;
        v = vv;
    }
    int iu = (int)((u + 1.0f) * (0.5f * kOctRes));
    int iv = (int)((v + 1.0f) * (0.5f * kOctRes));
    iu = iu < 0 ? 0 : (iu >= kOctRes ? kOctRes - 1 : iu);
    iv = iv < 0 ? 0 : (iv >= kOctRes ? kOctRes - 1 : iv);
    return iv * kOctRes + iu;
}

__device__ inline int trust_bin(const float *x6) {
    return oct_cell(x6[0], x6[1], x6[2]) * (kOctRes * kOctRes) + oct_cell(x6[3], x6[4], x6[5]);
}

}  // namespace mlp
}  // namespace lq
