// mlp.hip -- training and inference of the learned surrogate on gfx950.
//
// Inference (k_infer): weights staged in LDS in MFMA lane order, 16 rays per
// MFMA tile, activations in registers; see the comment above the kernel.
//
// Training step (one launch + one reduction launch):
//   k_train_step: a workgroup of 4 waves stages the bfloat16 weights in LDS in
//   MFMA lane order (forward and transposed) and processes tiles of 64
//   samples.  Per tile, each wave takes 16 samples through the sphere
//   parameterisation and the Fourier features, then the forward GEMMs and the
//   backward data GEMMs (MFMA 16x16x32 bf16, weights as the A operand, so one
//   layer's output registers are the next layer's B operand), with the loss
//   of Eq. 8 in between.  Features, activations and output gradients are also
//   written to LDS, one row per feature, and after a barrier the 84 16x16
//   blocks of the weight gradients (K = the tile's 64 samples) are split over
//   the 4 waves and accumulate in registers across the workgroup's tiles;
//   bias gradients are row sums.  Each workgroup writes one partial gradient
//   row.
//   k_reduce_adam: sums the rows in a fixed order (deterministic), applies
//   Adam to the float32 master weights and scatters them to the bfloat16
//   lane-ordered copy the kernels stage.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lq_internal.h"
#include "mlp_common.h"

using namespace lq::mlp;

namespace lq {
namespace {

constexpr int kWaves = 4;
constexpr int kTile = 64;                   // samples per tile (16 per wave)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// v[j], v[j + 1] as bfloat16 (nearest even) in one word, v[j] in the low
// half; converted as a two-element vector, which the compiler turns into one
// packed conversion (element by element it converts each value alone and
// merges the halves afterwards: three instructions per pair instead of one)
template <int J>
__device__ inline unsigned pk2(f32x4 v) {
    const f32x2 p = __builtin_shufflevector(v, v, J, J + 1);
    return __builtin_bit_cast(unsigned, __builtin_convertvector(p, bf16x2));
}

// the eight values lo[0..3], hi[0..3] as bfloat16, in that order
__device__ inline s16x8 pack8(f32x4 lo, f32x4 hi) {
    const u32x4 w = {pk2<0>(lo), pk2<2>(lo), pk2<0>(hi), pk2<2>(hi)};
    return __builtin_bit_cast(s16x8, w);
}

// bfloat16 of relu(x) for eight values: round first, then clear the negative
// ones as signed 16-bit integers (a bfloat16 with its sign bit set is negative
// as an int16), which equals rounding relu(x) and takes one packed max per pair
__device__ inline bf16x8 relu_pack(f32x4 lo, f32x4 hi) {
    const s16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    return __builtin_bit_cast(bf16x8, __builtin_elementwise_max(pack8(lo, hi), zero));
}

// variable whose 10 frequencies lane group g evaluates, the variable of its
// run of 5 and the first frequency of that run
__host__ __device__ constexpr int run_a(int g) { return g == 0 ? 0 : g == 1 ? 2 : g == 2 ? 3 : 5; }
__host__ __device__ constexpr int run_b(int g) { return g < 2 ? 1 : 4; }
__host__ __device__ constexpr int run_b0(int g) { return (g & 1) ? 5 : 0; }

// feature (index of the Fourier encoding, 0..127) that slot j (0..31) of lane
// group g holds: j < 20 sin/cos of the 10-run, 20 <= j < 30 the 5-run,
// j = 30, 31 the raw variables 2g, 2g + 1 (group 3: the two zero pads)
__host__ __device__ constexpr int slot_feature(int g, int j) {
    return j < 20   ? (1 + 2 * kFreq) * run_a(g) + 1 + j
           : j < 30 ? (1 + 2 * kFreq) * run_b(g) + 1 + 2 * run_b0(g) + (j - 20)
           : g == 3 ? kFeatUsed + (j - 30)
                    : (1 + 2 * kFreq) * (2 * g + (j - 30));
}
constexpr bool slots_are_a_permutation() {
    bool seen[kFeat] = {};
    for (int g = 0; g < 4; ++g)
        for (int j = 0; j < 32; ++j) {
            const int c = slot_feature(g, j);
            if (c < 0 || c >= kFeat || seen[c]) return false;
            seen[c] = true;
        }
    return true;
}
static_assert(slots_are_a_permutation(), "the feature slots must cover the encoding once");

// x[i] for a lane-dependent i, by selects on the six values (an indexed
// read of a private array would put the array in memory)
__device__ inline float pick6(float a0, float a1, float a2, float a3, float a4, float a5, int i) {
    return i == 0 ? a0 : i == 1 ? a1 : i == 2 ? a2 : i == 3 ? a3 : i == 4 ? a4 : a5;
}

// sin, cos of pi 2^k x for k = 0..4 into f[0..10) (x already scaled by the
// run's first frequency, |x| <= 32): the hardware sine and cosine of the
// argument reduced exactly to [-1/2, 1/2] turn (within 1.3e-7 of the exact
// values over this range), then sin 2a = 2 sin a cos a and
// cos 2a = 1 - 2 sin^2 a (three operations per doubling, sharing 2 sin a).
// Four doublings grow the initial error about 30-fold: under 5e-6 (measured
// in float32 over |x| <= 32), far under the bfloat16 feature rounding.
__device__ inline void sincos_run5(float x, float *f) {
    const float h = 0.5f * x;          // turns
    const float r = h - rintf(h);      // exact for |h| < 2^23
    float sn = __builtin_amdgcn_sinf(r), cs = __builtin_amdgcn_cosf(r);
    f[0] = sn;
    f[1] = cs;
#pragma unroll
    for (int k = 1; k < 5; ++k) {
        const float t = 2.0f * sn;
        const float s2 = t * cs;
        const float c2 = fmaf(-t, sn, 1.0f);
        sn = s2;
        cs = c2;
        f[2 * k] = sn;
        f[2 * k + 1] = cs;
    }
}

// ------------------------------------------------------------ training
// One workgroup of 4 waves processes tiles of 64 samples (16 per wave).
// Phase A, per wave: features, the forward GEMMs and the backward data GEMMs
// chained in registers exactly like inference (MFMA 16x16x32, weights -- and
// for the backward, the transposed weights -- staged in LDS in lane order;
// the ReLU masks come from the activations the lane still holds).  Every
// GEMM input of the weight gradients (features, activations H_l, output
// gradients dZ_l, dY) is also written to LDS feature-major, one row of 64
// samples per feature.  Phase B, per workgroup: the weight gradients
// dW_l = dZ_l H_{l-1}^T contract over the tile's 64 samples, so each MFMA
// operand is 8 consecutive samples of one row (one ds_read_b128); their 84
// 16x16 blocks are split over the 4 waves and accumulate in registers across
// the workgroup's tiles; bias gradients are row sums.
constexpr int kRS = 72;                              // LDS row stride (bf16): 64 samples + 8
constexpr int kRowX = 0, kRowH = kRowX + kFeat;      // X: 128 rows, H1..H4: 64 rows each
constexpr int kRowDZ = kRowH + 4 * kHidden;          // dZ1..dZ4: 64 rows each
constexpr int kRowDY = kRowDZ + 4 * kHidden;         // dY: 4 rows (outputs 0..2, row 3 zero)
constexpr int kRows = kRowDY + 4;
constexpr int kTW1 = 0;                              // bf16x8 [4 fb][4 kb][64]
constexpr int kTWh = kTW1 + 16 * 64 * 16;            // bf16x8 [3 l][4 fb][2 kb][64] + output [2 kb][64]
constexpr int kTWt = kTWh + 26 * 64 * 16;            // bf16x8 [3 l][4 ib][2 kb][64]: transposed W2..W4
constexpr int kTW5t = kTWt + 24 * 64 * 16;           // bf16x4 [4 ib][64]: transposed W5 (K = 16)
constexpr int kTB = kTW5t + 4 * 64 * 8;              // float [kBiasPad]
constexpr int kTAct = kTB + kBiasPad * 4;            // bf16 [kRows][kRS]
constexpr int kTLoss = kTAct + kRows * kRS * 2;      // float [kWaves]
constexpr int kTrainLds = kTLoss + kWaves * 4;
static_assert(kTrainLds <= 160 * 1024, "training LDS carve exceeds the CU's LDS");

// The bfloat16 weights are kept on the device in the byte order the kernels
// stage into LDS (the first kTB bytes of the training carve: W1, W2..W5 as
// the forward A operands, W2..W4 and W5 transposed as the backward ones), so
// a workgroup stages them with contiguous 16-byte copies.  Positions are in
// bfloat16 elements.
constexpr int kLaneElems = kTB / 2;

// slot (32 g + j) of feature f: the inverse of slot_feature
__host__ __device__ constexpr int slot_of_feature(int f) {
    if (f >= kFeatUsed) return 3 * 32 + 30 + (f - kFeatUsed);
    const int v = f / (1 + 2 * kFreq), r = f % (1 + 2 * kFreq);
    if (r == 0) return (v >> 1) * 32 + 30 + (v & 1);
    const int k = r - 1;
    if (v == 0 || v == 2 || v == 3 || v == 5) return (v == 0 ? 0 : v == 2 ? 1 : v == 3 ? 2 : 3) * 32 + k;
    return ((v == 1 ? 0 : 2) + (k >= kFreq)) * 32 + 20 + (k >= kFreq ? k - kFreq : k);
}
constexpr bool slot_inverse_holds() {
    for (int g = 0; g < 4; ++g)
        for (int j = 0; j < 32; ++j)
            if (slot_of_feature(slot_feature(g, j)) != 32 * g + j) return false;
    return true;
}
static_assert(slot_inverse_holds(), "slot_of_feature must invert slot_feature");

// parameter held at lane-image position u (-1: padding, kept zero)
__host__ __device__ constexpr int lane_param(int u) {
    if (u < kTWh / 2) {                                   // W1: [fb][kb][lane] x 8
        const int e = u & 7, ln = (u >> 3) & 63, blk = u >> 9;
        return kW1 + ((blk >> 2) * 16 + (ln & 15)) * kFeat + slot_feature(ln >> 4, (blk & 3) * 8 + e);
    }
    if (u < kTWt / 2) {                                   // W2..W4, W5: [blk][lane] x 8
        const int v = u - kTWh / 2, e = v & 7, ln = (v >> 3) & 63, blk = v >> 9;
        const int r = ln & 15, kb = blk < 24 ? (blk & 1) : blk - 24;
        const int in = 32 * kb + 16 * (e >> 2) + 4 * (ln >> 4) + (e & 3);
        if (blk < 24) return kW2 + (blk >> 3) * (kW3 - kW2) + (((blk >> 1) & 3) * 16 + r) * kHidden + in;
        return r < kOut ? kW5 + r * kHidden + in : -1;
    }
    if (u < kTW5t / 2) {                                  // W2..W4 transposed: [l][ib][kb][lane] x 8
        const int v = u - kTWt / 2, e = v & 7, ln = (v >> 3) & 63, blk = v >> 9;
        const int out = (2 * (blk & 1) + (e >> 2)) * 16 + 4 * (ln >> 4) + (e & 3);
        return kW2 + (blk >> 3) * (kW3 - kW2) + out * kHidden + ((blk >> 1) & 3) * 16 + (ln & 15);
    }
    const int v = u - kTW5t / 2, e = v & 3, ln = (v >> 2) & 63, ib = v >> 8;   // W5 transposed, x 4
    const int o = 4 * (ln >> 4) + e;
    return o < kOut ? kW5 + o * kHidden + ib * 16 + (ln & 15) : -1;
}

// lane-image positions of parameter p (W2..W5 appear twice, W1 once, biases
// not at all; -1 where there is none)
__host__ __device__ constexpr void lane_positions(int p, int &u0, int &u1) {
    u0 = u1 = -1;
    if (p < kB1) {
        const int out = p / kFeat, sl = slot_of_feature(p % kFeat), j = sl & 31;
        u0 = kTW1 / 2 + (((out >> 4) * 4 + (j >> 3)) * 64 + (sl >> 5) * 16 + (out & 15)) * 8 + (j & 7);
        return;
    }
    int l = -1, q = 0;
    if (p >= kW2 && p < kB2) { l = 0; q = p - kW2; }
    else if (p >= kW3 && p < kB3) { l = 1; q = p - kW3; }
    else if (p >= kW4 && p < kB4) { l = 2; q = p - kW4; }
    if (l >= 0) {
        const int out = q / kHidden, in = q % kHidden;
        u0 = kTWh / 2 + (((l * 4 + (out >> 4)) * 2 + (in >> 5)) * 64 + ((in & 15) >> 2) * 16 + (out & 15)) * 8 +
             4 * ((in >> 4) & 1) + (in & 3);
        u1 = kTWt / 2 + (((l * 4 + (in >> 4)) * 2 + (out >> 5)) * 64 + ((out & 15) >> 2) * 16 + (in & 15)) * 8 +
             4 * ((out >> 4) & 1) + (out & 3);
        return;
    }
    if (p >= kW5 && p < kB5) {
        const int o = (p - kW5) / kHidden, in = (p - kW5) % kHidden;
        u0 = kTWh / 2 + ((24 + (in >> 5)) * 64 + ((in & 15) >> 2) * 16 + o) * 8 + 4 * ((in >> 4) & 1) + (in & 3);
        u1 = kTW5t / 2 + ((in >> 4) * 64 + (in & 15)) * 4 + o;
    }
}

// every position's parameter lists that position, every weight's positions
// hold that weight (checked in ranges to stay within the constexpr step limit)
constexpr bool lane_forward_agrees(int u_begin, int u_end) {
    for (int u = u_begin; u < u_end; ++u) {
        const int p = lane_param(u);
        if (p < 0) continue;
        int u0 = 0, u1 = 0;
        lane_positions(p, u0, u1);
        if (u != u0 && u != u1) return false;
    }
    return true;
}
constexpr bool lane_inverse_agrees(int p_begin, int p_end) {
    for (int p = p_begin; p < p_end; ++p) {
        int u0 = 0, u1 = 0;
        lane_positions(p, u0, u1);
        const bool weight = p < kB1 || (p >= kW2 && p < kB2) || (p >= kW3 && p < kB3) || (p >= kW4 && p < kB4) ||
                            (p >= kW5 && p < kB5);
        if (weight != (u0 >= 0)) return false;
        if (u0 >= 0 && (u0 >= kLaneElems || lane_param(u0) != p)) return false;
        if (u1 >= 0 && (u1 >= kLaneElems || lane_param(u1) != p)) return false;
        if ((u1 >= 0) != (weight && p >= kW2)) return false;
    }
    return true;
}
static_assert(lane_forward_agrees(0, 4096) && lane_forward_agrees(4096, 8192), "lane image map, W1");
static_assert(lane_forward_agrees(8192, 12288) && lane_forward_agrees(12288, 16384), "lane image map, W2..W5");
static_assert(lane_forward_agrees(16384, 20480) && lane_forward_agrees(20480, 24576), "lane image map, W2..W5");
static_assert(lane_forward_agrees(24576, 28672) && lane_forward_agrees(28672, 32768), "lane image map, transposed");
static_assert(lane_forward_agrees(32768, kLaneElems), "lane image map, W5 transposed");
static_assert(lane_inverse_agrees(0, 4096) && lane_inverse_agrees(4096, 8192), "lane image inverse, W1");
static_assert(lane_inverse_agrees(8192, 12288) && lane_inverse_agrees(12288, 16384), "lane image inverse");
static_assert(lane_inverse_agrees(16384, kParams), "lane image inverse");

typedef __bf16 bf16x4b __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mfma16b(bf16x4b a, bf16x4b b, f32x4 c) {
    return mfma16(__builtin_bit_cast(bf16x4, a), __builtin_bit_cast(bf16x4, b), c);
}

// bfloat16 of x where the activation h (bfloat16, h layout) is positive, else
// 0: the mask min(max(h, 0), 1) per 16-bit half, negated to all ones
__device__ inline bf16x8 mask_pack(f32x4 lo, f32x4 hi, bf16x8 h) {
    const s16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0}, one = {1, 1, 1, 1, 1, 1, 1, 1};
    const s16x8 pos = __builtin_elementwise_min(__builtin_elementwise_max(__builtin_bit_cast(s16x8, h), zero), one);
    return __builtin_bit_cast(bf16x8, pack8(lo, hi) & (zero - pos));
}

// write the h-layout pair hv (features 16 (2 kb + e / 4) + 4 g + e % 4 of
// sample col) feature-major into the rows starting at row0
__device__ inline void store_rows(uint16_t *act, int row0, const bf16x8 (&hv)[2], int g, int col) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const s16x8 v = __builtin_bit_cast(s16x8, hv[kb]);
#pragma unroll
        for (int e = 0; e < 8; ++e)
            act[(row0 + (2 * kb + (e >> 2)) * 16 + 4 * g + (e & 3)) * kRS + col] = (uint16_t)v[e];
    }
}

__global__ __launch_bounds__(256) void k_train_step(const float *o, const float *d, const float *tgt,
                                                    int64_t n_pairs, int64_t base, int64_t count,
                                                    int tiles, float inv_batch, const uint16_t *wlane,
                                                    const float *bias, float *part, float *loss_part) {
    extern __shared__ __align__(16) char smem[];
    bf16x8 *sW1 = reinterpret_cast<bf16x8 *>(smem + kTW1);
    bf16x8 *sWh = reinterpret_cast<bf16x8 *>(smem + kTWh);
    bf16x8 *sWt = reinterpret_cast<bf16x8 *>(smem + kTWt);
    bf16x4b *sW5t = reinterpret_cast<bf16x4b *>(smem + kTW5t);
    float *sB = reinterpret_cast<float *>(smem + kTB);
    uint16_t *act = reinterpret_cast<uint16_t *>(smem + kTAct);
    float *sLoss = reinterpret_cast<float *>(smem + kTLoss);

    // ---- stage the lane-ordered weights: contiguous 16-byte copies
    static_assert(kTB % (16 * 256) == 0, "the lane image is copied in whole rounds of the block");
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(wlane);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
#pragma unroll
        for (int k = 0; k < kTB / (16 * 256); ++k) dst[k * 256 + threadIdx.x] = src[k * 256 + threadIdx.x];
    }
    for (int i = threadIdx.x; i < kBiasPad; i += blockDim.x) sB[i] = bias[i];
    __syncthreads();

    const int wave = threadIdx.x >> 6;
    const int lane = __lane_id();
    const int r16 = lane & 15, g = lane >> 4;
    const int col = wave * 16 + r16;     // this lane's sample column in the tile

    f32x4 gacc[21];
#pragma unroll
    for (int j = 0; j < 21; ++j) gacc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float gbias = 0.0f, gb5 = 0.0f, lsum = 0.0f;
    const bf16x8 zero8 = {};

    // the pair of the lane's sample in tile t (false: past the batch)
    auto pair_of = [&](int t, int64_t &ray) {
        const int64_t local = ((int64_t)blockIdx.x * tiles + t) * kTile + col;
        // base < n_pairs: one conditional subtraction unless the batch is
        // larger than the pair set
        int64_t r = base + local;
        if (r >= n_pairs) r -= n_pairs;
        if (r >= n_pairs) r %= n_pairs;
        ray = local < count ? r : 0;
        return local < count;
    };
    // each tile loads the next tile's pair while it computes
    float nx[9];
    {
        int64_t r0;
        pair_of(0, r0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nx[c] = o[3 * r0 + c];
            nx[3 + c] = d[3 * r0 + c];
            nx[6 + c] = tgt[3 * r0 + c];
        }
    }
    for (int tile = 0; tile < tiles; ++tile) {
        // ---- phase A: this wave's 16 samples
        int64_t ray;
        const bool valid = pair_of(tile, ray);
        float oo[3], dd[3], tt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            oo[c] = nx[c];
            dd[c] = nx[3 + c];
            tt[c] = nx[6 + c];
        }
        if (tile + 1 < tiles) {
            int64_t rn;
            pair_of(tile + 1, rn);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                nx[c] = o[3 * rn + c];
                nx[3 + c] = d[3 * rn + c];
                nx[6 + c] = tgt[3 * rn + c];
            }
        }
        float x6[6];
        const bool hit = sphere_x6(oo, dd, x6);
        const bool actv = valid && hit;
        const float e0 = x6[0], e1 = x6[1], e2 = x6[2], e3 = x6[3], e4 = x6[4], e5 = x6[5];
        float f[32];
        const float va = pick6(e0, e1, e2, e3, e4, e5, run_a(g));
        const float vb = pick6(e0, e1, e2, e3, e4, e5, run_b(g));
        sincos_run5(va, f);
        sincos_run5(va * 32.0f, f + 10);
        sincos_run5(run_b0(g) ? vb * 32.0f : vb, f + 20);
        f[30] = g < 3 ? pick6(e0, e1, e2, e3, e4, e5, 2 * g) : 0.0f;
        f[31] = g < 3 ? pick6(e0, e1, e2, e3, e4, e5, 2 * g + 1) : 0.0f;
        bf16x8 x[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const f32x4 lo = {f[kb * 8], f[kb * 8 + 1], f[kb * 8 + 2], f[kb * 8 + 3]};
            const f32x4 hi = {f[kb * 8 + 4], f[kb * 8 + 5], f[kb * 8 + 6], f[kb * 8 + 7]};
            x[kb] = actv ? __builtin_bit_cast(bf16x8, pack8(lo, hi)) : zero8;
            const s16x8 v = __builtin_bit_cast(s16x8, x[kb]);
#pragma unroll
            for (int e = 0; e < 8; ++e) act[(kRowX + slot_feature(g, kb * 8 + e)) * kRS + col] = (uint16_t)v[e];
        }

        // forward
        f32x4 acc[4];
        bf16x8 h[4][2];
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) acc[fb] = *reinterpret_cast<const f32x4 *>(sB + fb * 16 + 4 * g);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int fb = 0; fb < 4; ++fb) acc[fb] = mfma32(sW1[(fb * 4 + kb) * 64 + lane], x[kb], acc[fb]);
        h[0][0] = relu_pack(acc[0], acc[1]);
        h[0][1] = relu_pack(acc[2], acc[3]);
        store_rows(act, kRowH, h[0], g, col);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
                acc[fb] = *reinterpret_cast<const f32x4 *>(sB + (l + 1) * kHidden + fb * 16 + 4 * g);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int fb = 0; fb < 4; ++fb)
                    acc[fb] = mfma32(sWh[((l * 4 + fb) * 2 + kb) * 64 + lane], h[l][kb], acc[fb]);
            h[l + 1][0] = relu_pack(acc[0], acc[1]);
            h[l + 1][1] = relu_pack(acc[2], acc[3]);
            store_rows(act, kRowH + (l + 1) * kHidden, h[l + 1], g, col);
        }
        f32x4 y = *reinterpret_cast<const f32x4 *>(sB + 4 * kHidden + 4 * g);
        y = mfma32(sWh[24 * 64 + lane], h[3][0], y);
        y = mfma32(sWh[25 * 64 + lane], h[3][1], y);

        // loss (Eq. 8, channel-mean luminance held constant) and dL/dy:
        // lanes of group 0 hold outputs 0..3 of their sample
        float gy[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (g == 0 && actv) {
            float ey[3], lh[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ey[c] = expf(y[c]);
                lh[c] = ey[c] - kEpsOut;
            }
            const float den = (lh[0] + lh[1] + lh[2]) * (1.0f / 3.0f) + kLossEps;
            const float id2 = 1.0f / (den * den);
            float lsmp = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float diff = lh[c] - tt[c];
                lsmp += diff * diff * id2;
                gy[c] = 2.0f * diff * ey[c] * id2 * inv_batch;
            }
            lsum += lsmp;
        }
        const bf16x4b dyb = {(__bf16)gy[0], (__bf16)gy[1], (__bf16)gy[2], (__bf16)gy[3]};
        if (g == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) act[(kRowDY + c) * kRS + col] = f2bf(gy[c]);   // = dyb[c]
        }

        // backward data: dZ4 = (W5^T dY) masked by H4 > 0, then down to dZ1
        bf16x8 z[2];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) acc[ib] = mfma16b(sW5t[ib * 64 + lane], dyb, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        z[0] = mask_pack(acc[0], acc[1], h[3][0]);
        z[1] = mask_pack(acc[2], acc[3], h[3][1]);
        store_rows(act, kRowDZ + 3 * kHidden, z, g, col);
#pragma unroll
        for (int l = 2; l >= 0; --l) {    // dZ_{l+1} from dZ_{l+2} through W_{l+2}
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) acc[ib] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int ib = 0; ib < 4; ++ib)
                    acc[ib] = mfma32(sWt[((l * 4 + ib) * 2 + kb) * 64 + lane], z[kb], acc[ib]);
            z[0] = mask_pack(acc[0], acc[1], h[l][0]);
            z[1] = mask_pack(acc[2], acc[3], h[l][1]);
            store_rows(act, kRowDZ + l * kHidden, z, g, col);
        }
        __syncthreads();

        // ---- phase B: weight-gradient blocks over the tile's 64 samples
#pragma unroll
        for (int slot = 0; slot < 21; ++slot) {
            const int j = slot * kWaves + wave;   // block 0..83
            int arow, brow;
            bool arow_ok = true;
            if (j < 32) {
                arow = kRowDZ + (j >> 3) * 16;
                brow = kRowX + (j & 7) * 16;
            } else if (j < 80) {
                const int l = 2 + (j - 32) / 16, jj = (j - 32) % 16;
                arow = kRowDZ + (l - 1) * kHidden + (jj >> 2) * 16;
                brow = kRowH + (l - 2) * kHidden + (jj & 3) * 16;
            } else {
                arow = kRowDY;
                arow_ok = r16 < 4;                 // output rows 4..15 are padding
                brow = kRowH + 3 * kHidden + (j - 80) * 16;
            }
            f32x4 a_acc = gacc[slot];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const int c0 = kb * 32 + 8 * g;
                const bf16x8 ar = *reinterpret_cast<const bf16x8 *>(act + (arow + (arow_ok ? r16 : 0)) * kRS + c0);
                const bf16x8 av = arow_ok ? ar : zero8;
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(act + (brow + r16) * kRS + c0);
                a_acc = mfma32(av, bv, a_acc);
            }
            gacc[slot] = a_acc;
        }
        // bias gradients: thread t owns b_{t/64 + 1}[t % 64]; threads 0..2 b_5
        {
            const int t = threadIdx.x;
            const uint16_t *rowp = act + (kRowDZ + t) * kRS;     // dZ rows of the four hidden layers
            float sacc = 0.0f;
#pragma unroll
            for (int c = 0; c < kTile; c += 8) {
                const s16x8 v = *reinterpret_cast<const s16x8 *>(rowp + c);
#pragma unroll
                for (int e = 0; e < 8; ++e) sacc += bf2f((uint16_t)v[e]);
            }
            gbias += sacc;
            if (t < kOut) {
                const uint16_t *r5 = act + (kRowDY + t) * kRS;
                float s5 = 0.0f;
#pragma unroll
                for (int c = 0; c < kTile; c += 8) {
                    const s16x8 v = *reinterpret_cast<const s16x8 *>(r5 + c);
#pragma unroll
                    for (int e = 0; e < 8; ++e) s5 += bf2f((uint16_t)v[e]);
                }
                gb5 += s5;
            }
        }
        __syncthreads();
    }

    // ---- write this workgroup's partial gradient row
    float *P = part + (size_t)blockIdx.x * kParams;
#pragma unroll
    for (int slot = 0; slot < 21; ++slot) {
        const int j = slot * kWaves + wave;
        int woff, in_dim, out_dim, ob, ib;
        if (j < 32) { woff = kW1; in_dim = kFeat; out_dim = kHidden; ob = j >> 3; ib = j & 7; }
        else if (j < 80) {
            const int l = 2 + (j - 32) / 16, jj = (j - 32) % 16;
            woff = l == 2 ? kW2 : (l == 3 ? kW3 : kW4);
            in_dim = kHidden; out_dim = kHidden; ob = jj >> 2; ib = jj & 3;
        } else { woff = kW5; in_dim = kHidden; out_dim = kOut; ob = 0; ib = j - 80; }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int out = ob * 16 + 4 * g + i;
            const int in = ib * 16 + r16;
            if (out < out_dim) P[woff + out * in_dim + in] = gacc[slot][i];
        }
    }
    {
        const int t = threadIdx.x;
        const int boff = t < 64 ? kB1 : (t < 128 ? kB2 : (t < 192 ? kB3 : kB4));
        P[boff + (t & 63)] = gbias;
        if (t < kOut) P[kB5 + t] = gb5;
    }
    // loss partial: lanes 0..15 of each wave hold per-sample sums
    float l = lsum;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == 0) sLoss[wave] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        float sl = 0.0f;
        for (int w = 0; w < kWaves; ++w) sl += sLoss[w];
        loss_part[blockIdx.x] = sl * inv_batch;
    }
}

__device__ inline int bias_index(int p) {
    if (p >= kB1 && p < kW2) return p - kB1;
    if (p >= kB2 && p < kW3) return 64 + p - kB2;
    if (p >= kB3 && p < kW4) return 128 + p - kB3;
    if (p >= kB4 && p < kW5) return 192 + p - kB4;
    if (p >= kB5) return 256 + p - kB5;
    return -1;
}

// Sum of the partial gradient rows and the Adam update.  A block takes
// kRedParams consecutive parameters; its kRedWaves waves sum fixed slices of
// the rows with all of a slice's loads in flight, and wave 0 adds the slices
// in a fixed order: the result does not depend on scheduling, so a resumed
// run repeats an uninterrupted one bit for bit.  Block 0 also sums the
// per-workgroup losses with a fixed LDS tree.
constexpr int kRedParams = 64;
constexpr int kRedWaves = 16;
constexpr int kRedRows = 16;      // rows per slice loaded at once

__global__ __launch_bounds__(64 * kRedWaves) void k_reduce_adam(const float *part, int rows, float *theta, float *m,
                                                                float *v, uint16_t *wlane, float *bias,
                                                                const float *loss_part, float *loss_out,
                                                                float *grad_out, int update, float lr, float b1,
                                                                float b2, float eps, float c1, float c2) {
    __shared__ float s_part[kRedWaves][kRedParams];
    __shared__ float s_loss[256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * kRedParams + lane;
    float g = 0.0f;
    if (p < kParams) {
        const int r0 = rows * w / kRedWaves, r1 = rows * (w + 1) / kRedWaves;
        for (int r = r0; r < r1; r += kRedRows) {
            float a[kRedRows];
#pragma unroll
            for (int j = 0; j < kRedRows; ++j) a[j] = r + j < r1 ? part[(size_t)(r + j) * kParams + p] : 0.0f;
#pragma unroll
            for (int st = kRedRows / 2; st > 0; st >>= 1)
#pragma unroll
                for (int j = 0; j < st; ++j) a[j] += a[j + st];
            g += a[0];
        }
    }
    s_part[w][lane] = g;
    if (blockIdx.x == 0 && threadIdx.x < 256) {
        float l = 0.0f;
        for (int r = threadIdx.x; r < rows; r += 256) l += loss_part[r];
        s_loss[threadIdx.x] = l;
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) s_loss[threadIdx.x] += s_loss[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) *loss_out = s_loss[0];
    }
    if (w != 0 || p >= kParams) return;
    float sl[kRedWaves];
#pragma unroll
    for (int j = 0; j < kRedWaves; ++j) sl[j] = s_part[j][lane];
#pragma unroll
    for (int st = kRedWaves / 2; st > 0; st >>= 1)
#pragma unroll
        for (int j = 0; j < st; ++j) sl[j] += sl[j + st];
    g = sl[0];
    if (grad_out) grad_out[p] = g;
    if (!update) return;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float th = theta[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    theta[p] = th;
    int u0 = -1, u1 = -1;
    lane_positions(p, u0, u1);
    const uint16_t hb = f2bf(th);
    if (u0 >= 0) wlane[u0] = hb;
    if (u1 >= 0) wlane[u1] = hb;
    const int bi = bias_index(p);
    if (bi >= 0) bias[bi] = th;
}

// parameter that a bias slot holds (-1: padding, stays zero)
__device__ inline int param_of_bias(int i) {
    if (i < 64) return kB1 + i;
    if (i < 128) return kB2 + i - 64;
    if (i < 192) return kB3 + i - 128;
    if (i < 256) return kB4 + i - 192;
    return i - 256 < kOut ? kB5 + i - 256 : -1;
}

__global__ void k_pack(const float *theta, uint16_t *wlane, float *bias) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kLaneElems) {
        const int p = lane_param(i);
        wlane[i] = p >= 0 ? f2bf(theta[p]) : (uint16_t)0;
    }
    if (i < kBiasPad) {
        const int p = param_of_bias(i);
        bias[i] = p >= 0 ? theta[p] : 0.0f;
    }
}

// ------------------------------------------------------------ inference
// The weights live in LDS as MFMA operands in lane order ([block][lane],
// 16 bytes per lane: one conflict-free ds_read_b128 per MFMA), shared by the
// eight waves of a block and read again for every tile (a fence per tile
// keeps the compiler from hoisting them into registers, which would leave
// room for one wave per SIMD instead of four).  Tiles of 16 rays go through MFMA 16x16x32 (bf16
// in, f32 accumulate) with the activations in registers.  Lane l = 16 g + r
// (g = lane group, r = sample of the tile).  The weights are the A operand,
// so output block fb of a layer leaves lane l holding features 16 fb + 4 g + i
// (i < 4) of sample r; a 32-wide K block kb of the next layer takes, in lane
// group g, the four rows of block 2 kb followed by the four of block 2 kb + 1
// -- the weights are staged in that same K order, so no value moves between
// lanes.  The first layer's K order is chosen for the features
// (slot_feature below): lane group g evaluates 10 + 5 consecutive
// frequencies of two input variables: the hardware sine and cosine at the
// first frequency of each run of five, then angle doubling.
// (lanes past the end load ray 0: their results are discarded)
__device__ inline void load_ray(const float *o, const float *d, int64_t ray, float *oo, float *dd) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        oo[c] = o[3 * ray + c];
        dd[c] = d[3 * ray + c];
    }
}

__device__ inline int64_t ray_of(const int64_t *index, int64_t pos) { return index ? index[pos] : pos; }

// mode 0: radiance; mode 2: trust statistics against the reference radiance
// (per bin: pairs, and pairs whose squared error exceeds max_rel2 times the
// squared reference plus abs_floor2).  With an index list the kernel answers rays
// index[0 .. *n_dev) (the count read on the device), else rays 0 .. n.
constexpr int kInfBlock = 512;               // inference block: eight waves share one copy of the weights
constexpr int kInfWaves = kInfBlock / 64;

__global__ __launch_bounds__(kInfBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_infer(
    const float *o, const float *d, int64_t n, const int64_t *index, const unsigned long long *n_dev,
    const uint16_t *wlane, const float *bias, int mode, float *rgb, const float *ref, unsigned *tcnt,
    unsigned *tbad, float max_rel2, float abs_floor2) {
    __shared__ __align__(16) float sB[kBiasPad];
    for (int i = threadIdx.x; i < kBiasPad; i += blockDim.x) sB[i] = bias[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int lane = __lane_id();
    const int r16 = lane & 15, g = lane >> 4;

    // first layer [fb][kb][lane] (K in the feature-slot order), then the
    // hidden and output layers [l][fb][kb][lane] (l = 3: the output layer,
    // fb = 0 only): the leading part of the lane-ordered weight image
    __shared__ __align__(16) bf16x8 sW[(16 + 26) * 64];
    const bf16x8 *sW1 = sW;
    const bf16x8 *sWh = sW + 16 * 64;
    static_assert(kTWh == 16 * 64 * 16 && kTWt == (16 + 26) * 64 * 16, "inference stages W1 and W2..W5");
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(wlane);
        uint4 *dst = reinterpret_cast<uint4 *>(sW);
        for (int i = threadIdx.x; i < kTWt / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    if (n_dev) n = (int64_t)*n_dev;
    const int64_t nblk = (n + 15) / 16;
    const int64_t wstride = (int64_t)gridDim.x * kInfWaves;
    int64_t blk = (int64_t)blockIdx.x * kInfWaves + wave;
    // the next tile's rays are loaded while the current one computes
    bool nvalid = blk * 16 + r16 < n;
    int64_t nray = nvalid ? ray_of(index, blk * 16 + r16) : 0;
    float no[3], nd[3];
    load_ray(o, d, nray, no, nd);
    for (; blk < nblk; blk += wstride) {
        // a fence per tile keeps the weight reads inside the loop (hoisted,
        // the operands would need the register file of a single wave)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t ray = nray;
        const bool valid = nvalid;
        float oo[3] = {no[0], no[1], no[2]}, dd[3] = {nd[0], nd[1], nd[2]};
        const int64_t nxt = blk + wstride;
        nvalid = nxt < nblk && nxt * 16 + r16 < n;
        nray = nvalid ? ray_of(index, nxt * 16 + r16) : 0;
        load_ray(o, d, nray, no, nd);

        float x6[6];
        const bool hit = sphere_x6(oo, dd, x6);
        const bool act = valid && hit;
        const float e0 = x6[0], e1 = x6[1], e2 = x6[2], e3 = x6[3], e4 = x6[4], e5 = x6[5];
        float f[32];
        const float va = pick6(e0, e1, e2, e3, e4, e5, run_a(g));
        const float vb = pick6(e0, e1, e2, e3, e4, e5, run_b(g));
        sincos_run5(va, f);
        sincos_run5(va * 32.0f, f + 10);
        sincos_run5(run_b0(g) ? vb * 32.0f : vb, f + 20);
        f[30] = g < 3 ? pick6(e0, e1, e2, e3, e4, e5, 2 * g) : 0.0f;
        f[31] = g < 3 ? pick6(e0, e1, e2, e3, e4, e5, 2 * g + 1) : 0.0f;
        // (the features of rays that miss the sphere are finite and their
        // outputs are discarded)
        bf16x8 x[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const f32x4 lo = {f[kb * 8], f[kb * 8 + 1], f[kb * 8 + 2], f[kb * 8 + 3]};
            const f32x4 hi = {f[kb * 8 + 4], f[kb * 8 + 5], f[kb * 8 + 6], f[kb * 8 + 7]};
            x[kb] = __builtin_bit_cast(bf16x8, pack8(lo, hi));
        }

        f32x4 acc[4];
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) acc[fb] = *reinterpret_cast<const f32x4 *>(sB + fb * 16 + 4 * g);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int fb = 0; fb < 4; ++fb) acc[fb] = mfma32(sW1[(fb * 4 + kb) * 64 + lane], x[kb], acc[fb]);
        bf16x8 h[2] = {relu_pack(acc[0], acc[1]), relu_pack(acc[2], acc[3])};
#pragma unroll
        for (int l = 0; l < 3; ++l) {
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
                acc[fb] = *reinterpret_cast<const f32x4 *>(sB + (l + 1) * kHidden + fb * 16 + 4 * g);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int fb = 0; fb < 4; ++fb) acc[fb] = mfma32(sWh[((l * 4 + fb) * 2 + kb) * 64 + lane], h[kb], acc[fb]);
            h[0] = relu_pack(acc[0], acc[1]);
            h[1] = relu_pack(acc[2], acc[3]);
        }
        f32x4 y = *reinterpret_cast<const f32x4 *>(sB + 4 * kHidden + 4 * g);
        y = mfma32(sWh[24 * 64 + lane], h[0], y);
        y = mfma32(sWh[25 * 64 + lane], h[1], y);

        if (g == 0 && valid) {
            float L[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) L[c] = act ? fmaxf(expf(y[c]) - kEpsOut, 0.0f) : 0.0f;
            if (mode == 2) {
                if (act) {
                    const float p6[6] = {e0, e1, e2, e3, e4, e5};
                    const int bin = trust_bin(p6);
                    // float32 sums of three squares (relative error under
                    // 8 u each); the error side is inflated by 2^-20 = 16 u,
                    // so a pair at the bound counts as outside (conservative)
                    float se = 0.0f, sr = 0.0f;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float rc = ref[3 * ray + c];
                        const float ec = L[c] - rc;
                        se = fmaf(ec, ec, se);
                        sr = fmaf(rc, rc, sr);
                    }
                    atomicAdd(tcnt + bin, 1u);
                    if (se * (1.0f + 0x1p-20f) > fmaf(max_rel2, sr, abs_floor2)) atomicAdd(tbad + bin, 1u);
                }
            } else {
                rgb[3 * ray] = L[0];
                rgb[3 * ray + 1] = L[1];
                rgb[3 * ray + 2] = L[2];
            }
        }
    }
}

// Split a batch for the hybrid query (sphere_route): rays whose line misses
// the bounding sphere, or whose sphere lies behind them, get radiance 0
// here; rays starting inside the sphere go to the octree list; the others go
// to the surrogate list if their trust bin is trusted, else to the octree
// list.  A block classifies
// kClassRays rays (16 per thread, strided by the block size so that loads
// coalesce), places them with wave ballots and LDS counters, and reserves
// its slots in each global list with one atomic per list.
constexpr int kClassPer = 16;
constexpr int kClassRays = 256 * kClassPer;

__global__ __launch_bounds__(256) void k_classify(const float *o, const float *d, int64_t n, const uint8_t *trust,
                                                  float *rgb, uint8_t *used_fb, int64_t *mlp_list,
                                                  unsigned long long *mlp_cnt, int64_t *oct_list,
                                                  unsigned long long *oct_cnt) {
    __shared__ unsigned s_cnt[2];
    __shared__ unsigned long long s_base[2];
    if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kClassRays;
    uint32_t slot[kClassPer];   // list (bit 31: octree) and position in the block's share, or ~0u: none
#pragma unroll
    for (int k = 0; k < kClassPer; ++k) {
        const int64_t ray = base + k * 256 + threadIdx.x;
        int cls = -1;   // -1 nothing to do, 0 surrogate, 1 octree, 2 miss
        if (ray < n) {
            float oo[3] = {o[3 * ray], o[3 * ray + 1], o[3 * ray + 2]};
            float dd[3] = {d[3 * ray], d[3 * ray + 1], d[3 * ray + 2]};
            float x6[6];
            const int route = sphere_route(oo, dd, x6);
            cls = route == kRouteNet ? (trust[trust_bin(x6)] ? 0 : 1) : (route == kRouteOctree ? 1 : 2);
        }
        slot[k] = ~0u;
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const uint64_t mask = __ballot(cls == l);
            if (!mask) continue;
            const int leader = __ffsll((unsigned long long)mask) - 1;
            unsigned wb = 0;
            if (lane == leader) wb = atomicAdd(&s_cnt[l], (unsigned)__popcll(mask));
            wb = __builtin_amdgcn_readlane(wb, leader);
            if (cls == l) slot[k] = ((unsigned)l << 31) | (wb + (unsigned)__popcll(mask & below));
        }
        if (cls == 2) {
            rgb[3 * ray] = 0.0f;
            rgb[3 * ray + 1] = 0.0f;
            rgb[3 * ray + 2] = 0.0f;
        }
        if (used_fb && cls >= 0) used_fb[ray] = cls == 1 ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_base[0] = atomicAdd(mlp_cnt, (unsigned long long)s_cnt[0]);
    if (threadIdx.x == 1) s_base[1] = atomicAdd(oct_cnt, (unsigned long long)s_cnt[1]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kClassPer; ++k) {
        if (slot[k] == ~0u) continue;
        const int64_t ray = base + k * 256 + threadIdx.x;
        const unsigned l = slot[k] >> 31, pos = slot[k] & 0x7FFFFFFFu;
        (l ? oct_list : mlp_list)[s_base[l] + pos] = ray;
    }
}

// Trust map: a bin is trusted when it holds at least kTrustMinPairs held-out
// pairs and every one of them is within the bound.
constexpr unsigned kTrustMinPairs = 32;
constexpr float kTrustAbsFloor = 1e-2f;   // radiance units: dark rays pass with errors below this

__global__ void k_trust_finalize(const unsigned *tcnt, const unsigned *tbad, uint8_t *trust) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= kTrustBins) return;
    trust[b] = tcnt[b] >= kTrustMinPairs && tbad[b] == 0 ? 1 : 0;
}

__global__ void k_zero_bytes(unsigned char *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace
}  // namespace lq

// ====================================================================== host
struct lq_mlp {
    int device;
    float *theta, *m, *v;
    uint16_t *wlane;   // bfloat16 weights in LDS staging order
    float *bias;
    float *part;
    int part_rows;
    float *loss_part;
    float *loss_dev;   // one float per step of the current training call
    int64_t loss_cap;
    uint8_t *trust;
    bool has_trust;
    int64_t step;
    uint64_t seed;
    int max_wg_train;
};

namespace lq {

static lq_status mfail(lq_status s, const std::string &msg) {
    set_error(msg);
    return s;
}
static lq_status mhip(hipError_t e, const char *what) {
    return mfail(LQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// SplitMix64: a counter-based generator, one draw per parameter index
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static void he_uniform_init(uint64_t seed, std::vector<float> &th) {
    th.assign(kParams, 0.0f);
    const int ins[5] = {kFeat, kHidden, kHidden, kHidden, kHidden};
    const int outs[5] = {kHidden, kHidden, kHidden, kHidden, kOut};
    const int woff[5] = {kW1, kW2, kW3, kW4, kW5};
    for (int l = 0; l < 5; ++l) {
        const double lim = sqrt(6.0 / ins[l]);
        for (int i = 0; i < ins[l] * outs[l]; ++i) {
            const uint64_t r = splitmix64(seed * 0x100000001B3ull + (uint64_t)(woff[l] + i));
            const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
            th[woff[l] + i] = (float)((2.0 * u - 1.0) * lim);
        }
    }
}

static void free_mlp(lq_mlp *p) {
    if (!p) return;
    (void)hipFree(p->theta);
    (void)hipFree(p->m);
    (void)hipFree(p->v);
    (void)hipFree(p->wlane);
    (void)hipFree(p->bias);
    (void)hipFree(p->part);
    (void)hipFree(p->loss_part);
    (void)hipFree(p->loss_dev);
    (void)hipFree(p->trust);
    delete p;
}

static lq_status alloc_mlp(int device, lq_mlp **out) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return mfail(LQ_ERR_HIP, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return mfail(LQ_ERR_INVALID_ARG, "device index out of range");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return mhip(e, "hipSetDevice");
    lq_mlp *p = new (std::nothrow) lq_mlp();
    if (!p) return mfail(LQ_ERR_OOM, "host allocation failed");
    memset(p, 0, sizeof(*p));
    p->device = device;
    int cus = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    p->max_wg_train = cus > 0 ? cus : 1;
    p->part_rows = p->max_wg_train;
    bool ok = hipMalloc((void **)&p->theta, kParams * 4) == hipSuccess &&
              hipMalloc((void **)&p->m, kParams * 4) == hipSuccess &&
              hipMalloc((void **)&p->v, kParams * 4) == hipSuccess &&
              hipMalloc((void **)&p->wlane, kLaneElems * 2) == hipSuccess &&
              hipMalloc((void **)&p->bias, kBiasPad * 4) == hipSuccess &&
              hipMalloc((void **)&p->part, (size_t)p->part_rows * kParams * 4) == hipSuccess &&
              hipMalloc((void **)&p->loss_part, (size_t)p->part_rows * 4) == hipSuccess &&
              hipMalloc((void **)&p->trust, kTrustBins) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_mlp(p);
        return mfail(LQ_ERR_OOM, "device allocation for the surrogate failed");
    }
    if (hipFuncSetAttribute((const void *)k_train_step, hipFuncAttributeMaxDynamicSharedMemorySize, kTrainLds) !=
        hipSuccess) {
        (void)hipGetLastError();
        free_mlp(p);
        return mfail(LQ_ERR_UNSUPPORTED, "the device cannot give the kernels their LDS");
    }
    *out = p;
    return LQ_OK;
}

static lq_status upload_params(lq_mlp *p, const float *host_theta, bool reset_moments) {
    hipError_t e = hipMemcpy(p->theta, host_theta, kParams * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && reset_moments) e = hipMemset(p->m, 0, kParams * 4);
    if (e == hipSuccess && reset_moments) e = hipMemset(p->v, 0, kParams * 4);
    if (e != hipSuccess) return mhip(e, "uploading parameters");
    hipLaunchKernelGGL(k_pack, dim3((kLaneElems + 255) / 256), dim3(256), 0, 0, p->theta, p->wlane, p->bias);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return mhip(e, "packing parameters");
    return LQ_OK;
}

static lq_status check_dev_ptr(const void *ptr, size_t bytes, int device, const char *name) {
    if (!ptr) return mfail(LQ_ERR_INVALID_ARG, std::string(name) + " is NULL");
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(LQ_ERR_INVALID_ARG, std::string(name) + " is not a device pointer");
    }
    if ((at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) || at.device != device)
        return mfail(LQ_ERR_INVALID_ARG, std::string(name) + " is not a device pointer on the surrogate's device");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(LQ_ERR_INVALID_ARG, std::string(name) + ": allocation range unknown");
    }
    if ((const char *)ptr + bytes > (const char *)base + size)
        return mfail(LQ_ERR_INVALID_ARG, std::string(name) + " is smaller than the batch needs");
    if ((uintptr_t)ptr % 4) return mfail(LQ_ERR_INVALID_ARG, std::string(name) + " is not 4-byte aligned");
    return LQ_OK;
}

// one forward/backward over samples [base, base + count) of the pair set
static hipError_t launch_step(lq_mlp *p, const float *o, const float *d, const float *t, int64_t n_pairs,
                              int64_t base, int64_t count, int &rows, hipStream_t s) {
    const int64_t tiles_total = (count + kTile - 1) / kTile;
    int64_t wg = std::min<int64_t>(tiles_total, p->max_wg_train);
    const int tiles = (int)((tiles_total + wg - 1) / wg);
    wg = (tiles_total + tiles - 1) / tiles;
    rows = (int)wg;
    hipLaunchKernelGGL(k_train_step, dim3((unsigned)wg), dim3(256), kTrainLds, s, o, d, t, n_pairs, base, count,
                       tiles, 1.0f / (float)count, p->wlane, p->bias, p->part, p->loss_part);
    return hipGetLastError();
}

}  // namespace lq

using namespace lq;

extern "C" {

lq_status lq_mlp_create(const lq_mlp_config *cfg, uint64_t seed, int device, lq_mlp **out) {
    if (!out) return mfail(LQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (cfg && (cfg->n_freq != kFreq || cfg->hidden != kHidden || cfg->n_hidden_layers != 4))
        return mfail(LQ_ERR_UNSUPPORTED, "the surrogate is built for 10 frequencies and 4 x 64 hidden units");
    lq_mlp *p = nullptr;
    lq_status st = alloc_mlp(device, &p);
    if (st != LQ_OK) return st;
    p->seed = seed;
    std::vector<float> th;
    he_uniform_init(seed, th);
    st = upload_params(p, th.data(), true);
    if (st != LQ_OK) {
        free_mlp(p);
        return st;
    }
    *out = p;
    return LQ_OK;
}

void lq_mlp_free(lq_mlp *p) {
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    free_mlp(p);
    (void)hipSetDevice(cur);
}

int32_t lq_mlp_num_params(void) { return kParams; }

lq_status lq_mlp_get_params(const lq_mlp *p, float *host_theta) {
    if (!p || !host_theta) return mfail(LQ_ERR_INVALID_ARG, "NULL argument");
    (void)hipSetDevice(p->device);
    hipError_t e = hipMemcpy(host_theta, p->theta, kParams * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? LQ_OK : mhip(e, "reading parameters");
}

lq_status lq_mlp_set_params(lq_mlp *p, const float *host_theta) {
    if (!p || !host_theta) return mfail(LQ_ERR_INVALID_ARG, "NULL argument");
    (void)hipSetDevice(p->device);
    p->step = 0;
    return upload_params(p, host_theta, true);
}

lq_status lq_mlp_grad(lq_mlp *p, const float *o, const float *d, const float *rgb, int64_t n, float *grad,
                      float *loss_host, void *stream) {
    if (!p) return mfail(LQ_ERR_INVALID_ARG, "surrogate is NULL");
    if (n <= 0) return mfail(LQ_ERR_INVALID_ARG, "n must be > 0");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return mhip(e, "hipSetDevice");
    lq_status st;
    if ((st = check_dev_ptr(o, n * 12, p->device, "origins")) != LQ_OK) return st;
    if ((st = check_dev_ptr(d, n * 12, p->device, "dirs")) != LQ_OK) return st;
    if ((st = check_dev_ptr(rgb, n * 12, p->device, "rgb")) != LQ_OK) return st;
    if ((st = check_dev_ptr(grad, kParams * 4, p->device, "grad")) != LQ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    float *loss_dev = nullptr;
    if ((e = hipMallocAsync((void **)&loss_dev, 4, s)) != hipSuccess) return mhip(e, "hipMallocAsync");
    int rows = 0;
    e = launch_step(p, o, d, rgb, n, 0, n, rows, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_reduce_adam, dim3((kParams + kRedParams - 1) / kRedParams), dim3(64 * kRedWaves), 0, s, p->part, rows, p->theta,
                           p->m, p->v, p->wlane, p->bias, p->loss_part, loss_dev, grad, 0, 0.0f, 0.0f, 0.0f, 0.0f,
                           0.0f, 0.0f);
        e = hipGetLastError();
    }
    float lh = 0.0f;
    if (e == hipSuccess && loss_host) e = hipMemcpyAsync(&lh, loss_dev, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(loss_dev, s);
    if (e != hipSuccess) return mhip(e, "surrogate gradient");
    if (loss_host) *loss_host = lh;
    return LQ_OK;
}

lq_status lq_mlp_train(lq_mlp *p, const float *o, const float *d, const float *rgb, int64_t n_pairs,
                       const lq_train_config *cfg, float *loss_log_host, void *stream) {
    if (!p || !cfg) return mfail(LQ_ERR_INVALID_ARG, "NULL argument");
    if (n_pairs <= 0) return mfail(LQ_ERR_INVALID_ARG, "n_pairs must be > 0");
    if (cfg->steps < 0 || cfg->batch <= 0 || cfg->batch % kTile || cfg->total_steps <= 0)
        return mfail(LQ_ERR_INVALID_ARG, "steps >= 0, batch a positive multiple of 64, total_steps > 0");
    if (!(cfg->lr0 > 0.0f) || !(cfg->lr1 > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f))
        return mfail(LQ_ERR_INVALID_ARG, "bad optimiser settings");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return mhip(e, "hipSetDevice");
    lq_status st;
    if ((st = check_dev_ptr(o, n_pairs * 12, p->device, "origins")) != LQ_OK) return st;
    if ((st = check_dev_ptr(d, n_pairs * 12, p->device, "dirs")) != LQ_OK) return st;
    if ((st = check_dev_ptr(rgb, n_pairs * 12, p->device, "rgb")) != LQ_OK) return st;
    if (cfg->steps == 0) return LQ_OK;
    hipStream_t s = (hipStream_t)stream;
    float *loss_dev = nullptr;
    if ((e = hipMallocAsync((void **)&loss_dev, (size_t)cfg->steps * 4, s)) != hipSuccess)
        return mhip(e, "hipMallocAsync");
    for (int k = 0; k < cfg->steps && e == hipSuccess; ++k) {
        const int64_t gstep = p->step;   // global step index (0-based)
        const int64_t base = (int64_t)((gstep * (int64_t)cfg->batch) % n_pairs);
        int rows = 0;
        e = launch_step(p, o, d, rgb, n_pairs, base, cfg->batch, rows, s);
        if (e != hipSuccess) break;
        const double frac = (double)gstep / (double)cfg->total_steps;
        const float lr = (float)(cfg->lr0 * pow((double)cfg->lr1 / cfg->lr0, frac));
        const double t = (double)(gstep + 1);
        const float c1 = (float)(1.0 / (1.0 - pow((double)cfg->beta1, t)));
        const float c2 = (float)(1.0 / (1.0 - pow((double)cfg->beta2, t)));
        hipLaunchKernelGGL(k_reduce_adam, dim3((kParams + kRedParams - 1) / kRedParams), dim3(64 * kRedWaves), 0, s, p->part, rows, p->theta,
                           p->m, p->v, p->wlane, p->bias, p->loss_part, loss_dev + k, (float *)nullptr, 1, lr,
                           cfg->beta1, cfg->beta2, cfg->eps, c1, c2);
        e = hipGetLastError();
        p->step++;
    }
    if (e == hipSuccess && loss_log_host)
        e = hipMemcpyAsync(loss_log_host, loss_dev, (size_t)cfg->steps * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && loss_log_host) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(loss_dev, s);
    if (e != hipSuccess) return mhip(e, "surrogate training");
    return LQ_OK;
}

}  // extern "C"

namespace lq {

// one persistent block per resident slot (the occupancy the kernel's
// register and LDS budget allows)
static int infer_grid(int device) {
    int cus = 1, per_cu = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_infer, kInfBlock, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return (cus > 0 ? cus : 1) * per_cu;
}

}  // namespace lq

extern "C" {

lq_status lq_mlp_forward(const lq_mlp *p, const float *o, const float *d, int64_t n, float *rgb, void *stream) {
    if (!p) return mfail(LQ_ERR_INVALID_ARG, "surrogate is NULL");
    if (n < 0) return mfail(LQ_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return LQ_OK;
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return mhip(e, "hipSetDevice");
    lq_status st;
    if ((st = check_dev_ptr(o, n * 12, p->device, "origins")) != LQ_OK) return st;
    if ((st = check_dev_ptr(d, n * 12, p->device, "dirs")) != LQ_OK) return st;
    if ((st = check_dev_ptr(rgb, n * 12, p->device, "rgb")) != LQ_OK) return st;
    hipLaunchKernelGGL(k_infer, dim3(infer_grid(p->device)), dim3(kInfBlock), 0, (hipStream_t)stream, o, d, n,
                       (const int64_t *)nullptr, (const unsigned long long *)nullptr, p->wlane, p->bias, 0, rgb,
                       (const float *)nullptr, (unsigned *)nullptr, (unsigned *)nullptr, 0.0f, 0.0f);
    e = hipGetLastError();
    return e == hipSuccess ? LQ_OK : mhip(e, "surrogate forward");
}

lq_status lq_mlp_build_trust(lq_mlp *p, const float *o, const float *d, const float *rgb_ref, int64_t n,
                             float max_rel_err, void *stream) {
    if (!p) return mfail(LQ_ERR_INVALID_ARG, "surrogate is NULL");
    if (n <= 0 || !(max_rel_err > 0.0f)) return mfail(LQ_ERR_INVALID_ARG, "n > 0 and max_rel_err > 0 required");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return mhip(e, "hipSetDevice");
    lq_status st;
    if ((st = check_dev_ptr(o, n * 12, p->device, "origins")) != LQ_OK) return st;
    if ((st = check_dev_ptr(d, n * 12, p->device, "dirs")) != LQ_OK) return st;
    if ((st = check_dev_ptr(rgb_ref, n * 12, p->device, "rgb_ref")) != LQ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)kTrustBins * 8;   // pair count and out-of-bound count per bin
    unsigned char *acc = nullptr;
    if ((e = hipMallocAsync((void **)&acc, bytes, s)) != hipSuccess) return mhip(e, "hipMallocAsync");
    unsigned *tcnt = reinterpret_cast<unsigned *>(acc);
    unsigned *tbad = tcnt + kTrustBins;
    hipLaunchKernelGGL(k_zero_bytes, dim3(1024), dim3(256), 0, s, acc, bytes);
    hipLaunchKernelGGL(k_infer, dim3(infer_grid(p->device)), dim3(kInfBlock), 0, s, o, d, n, (const int64_t *)nullptr,
                       (const unsigned long long *)nullptr, p->wlane, p->bias, 2, (float *)nullptr, rgb_ref, tcnt, tbad,
                       max_rel_err * max_rel_err, kTrustAbsFloor * kTrustAbsFloor);
    hipLaunchKernelGGL(k_trust_finalize, dim3((kTrustBins + 255) / 256), dim3(256), 0, s, tcnt, tbad, p->trust);
    e = hipGetLastError();
    (void)hipFreeAsync(acc, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return mhip(e, "building the trust map");
    p->has_trust = true;
    return LQ_OK;
}

lq_status lq_mlp_trust_map(const lq_mlp *p, uint8_t *host_map, int32_t *n_bins) {
    if (!p) return mfail(LQ_ERR_INVALID_ARG, "surrogate is NULL");
    if (n_bins) *n_bins = p->has_trust ? kTrustBins : 0;
    if (!host_map || !p->has_trust) return LQ_OK;
    (void)hipSetDevice(p->device);
    hipError_t e = hipMemcpy(host_map, p->trust, kTrustBins, hipMemcpyDeviceToHost);
    return e == hipSuccess ? LQ_OK : mhip(e, "reading the trust map");
}

lq_status lq_mlp_infer(const lq_mlp *p, const lq_octree *fallback, const float *o, const float *d, int64_t n,
                       float *rgb, uint8_t *used_fallback, void *stream) {
    if (!p) return mfail(LQ_ERR_INVALID_ARG, "surrogate is NULL");
    if (n < 0) return mfail(LQ_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return LQ_OK;
    if (!p->has_trust || !fallback) {
        if (used_fallback) return mfail(LQ_ERR_STATE, "no trust map or fallback tree: nothing falls back");
        return lq_mlp_forward(p, o, d, n, rgb, stream);
    }
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return mhip(e, "hipSetDevice");
    lq_status st;
    if ((st = check_dev_ptr(o, n * 12, p->device, "origins")) != LQ_OK) return st;
    if ((st = check_dev_ptr(d, n * 12, p->device, "dirs")) != LQ_OK) return st;
    if ((st = check_dev_ptr(rgb, n * 12, p->device, "rgb")) != LQ_OK) return st;
    if (used_fallback && (st = check_dev_ptr(used_fallback, n, p->device, "used_fallback")) != LQ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // two counters, then the surrogate list and the octree list (n each)
    unsigned char *scratch = nullptr;
    const size_t bytes = 16 + (size_t)n * 16;
    if ((e = hipMallocAsync((void **)&scratch, bytes, s)) != hipSuccess) return mhip(e, "hipMallocAsync");
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(scratch);
    int64_t *mlp_list = reinterpret_cast<int64_t *>(scratch + 16);
    int64_t *oct_list = mlp_list + n;
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, s, scratch, (size_t)16);
    const int64_t cblocks = (n + kClassRays - 1) / kClassRays;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)cblocks), dim3(256), 0, s, o, d, n, p->trust, rgb, used_fallback,
                       mlp_list, cnt, oct_list, cnt + 1);
    hipLaunchKernelGGL(k_infer, dim3(infer_grid(p->device)), dim3(kInfBlock), 0, s, o, d, n, mlp_list,
                       (const unsigned long long *)cnt, p->wlane, p->bias, 0, rgb, (const float *)nullptr,
                       (unsigned *)nullptr, (unsigned *)nullptr, 0.0f, 0.0f);
    e = hipGetLastError();
    if (e == hipSuccess) {
        lq_status q = query_indexed(fallback, o, d, n, oct_list, cnt + 1, rgb, s);
        if (q != LQ_OK) {
            (void)hipFreeAsync(scratch, s);
            return q;
        }
    }
    (void)hipFreeAsync(scratch, s);
    return e == hipSuccess ? LQ_OK : mhip(e, "surrogate inference");
}

lq_status lq_mlp_save(const lq_mlp *p, const char *path) {
    if (!p || !path) return mfail(LQ_ERR_INVALID_ARG, "NULL argument");
    (void)hipSetDevice(p->device);
    std::vector<float> buf((size_t)3 * kParams);
    std::vector<uint8_t> trust(kTrustBins, 0);
    hipError_t e = hipMemcpy(buf.data(), p->theta, kParams * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + kParams, p->m, kParams * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * kParams, p->v, kParams * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && p->has_trust) e = hipMemcpy(trust.data(), p->trust, kTrustBins, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return mhip(e, "reading the surrogate");
    FILE *f = fopen(path, "wb");
    if (!f) return mfail(LQ_ERR_IO, std::string("cannot write ") + path);
    const uint32_t hdr[4] = {0x504D514Cu /* "LQMP" */, 2u, (uint32_t)kParams, p->has_trust ? 1u : 0u};
    const int64_t meta[2] = {p->step, (int64_t)p->seed};
    bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(meta, sizeof(meta), 1, f) == 1 &&
              fwrite(buf.data(), 4, buf.size(), f) == buf.size() &&
              fwrite(trust.data(), 1, trust.size(), f) == trust.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? LQ_OK : mfail(LQ_ERR_IO, std::string("short write to ") + path);
}

lq_status lq_mlp_load(const char *path, int device, lq_mlp **out) {
    if (!out || !path) return mfail(LQ_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return mfail(LQ_ERR_IO, std::string("cannot open ") + path);
    uint32_t hdr[4];
    int64_t meta[2];
    std::vector<float> buf((size_t)3 * kParams);
    std::vector<uint8_t> trust(kTrustBins);
    bool ok = fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 0x504D514Cu && hdr[1] == 2u &&
              hdr[2] == (uint32_t)kParams && fread(meta, sizeof(meta), 1, f) == 1 &&
              fread(buf.data(), 4, buf.size(), f) == buf.size() &&
              fread(trust.data(), 1, trust.size(), f) == trust.size();
    fclose(f);
    if (!ok) return mfail(LQ_ERR_FORMAT, std::string("not a surrogate file: ") + path);
    lq_mlp *p = nullptr;
    lq_status st = alloc_mlp(device, &p);
    if (st != LQ_OK) return st;
    p->step = meta[0];
    p->seed = (uint64_t)meta[1];
    hipError_t e = hipMemcpy(p->m, buf.data() + kParams, kParams * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->v, buf.data() + 2 * kParams, kParams * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->trust, trust.data(), kTrustBins, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_mlp(p);
        return mhip(e, "uploading the surrogate");
    }
    st = upload_params(p, buf.data(), false);
    if (st != LQ_OK) {
        free_mlp(p);
        return st;
    }
    p->has_trust = hdr[3] != 0;
    *out = p;
    return LQ_OK;
}

}  // extern "C"
