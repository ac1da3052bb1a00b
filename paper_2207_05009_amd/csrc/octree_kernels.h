// octree_kernels.h -- the emission-query kernels and their launchers,
// instantiated per storage type by octree_query_{f32,f16,bf16}.hip.
//
// Persistent waves: the grid holds as many 256-lane blocks as fit on the
// chip at once.  Every lane marches one ray at a time (Marcher in march.h),
// one octree node per step.  Every kStepsPerCheck steps the wave counts its
// busy lanes; when fewer than kRefillBelow still hold a ray, the idle lanes
// are refilled from a ray counter with one atomic per wave: a 64-bit ballot
// of the idle lanes, one atomicAdd of its popcount by the lowest idle lane,
// and each idle lane takes base + (number of idle lanes below it).  Rays of very different lengths
// then do not leave most of a wave idle until its longest ray is done,
// while the atomic's latency and the per-ray set-up are paid for many lanes
// at once.
//
// XCD-aware work split: the batch is cut into kXcds groups of kRangesPerXcd
// contiguous ranges, with a counter each.  Workgroups are dispatched to the
// accelerator dies round robin, so a wave of block b starts on a range of
// group b % kXcds: the rays one die's L2 sees are neighbours in the batch
// (for a camera, a band of image rows), not every kXcds-th chunk.  Two
// counters per die rather than one halve the same-address atomics of the
// refills, which bound batches of short or dead rays; more counters spread a
// die's waves over too many places of the batch for its L2.  A wave whose
// range is used up continues on the next ranges, so the tail stays balanced.
//
// Camera batches are split by position in their tile order instead
// (tile_order_pixel): the 64 rays one refill hands a wave then form an 8 x 8
// pixel tile rather than a 1 x 64 strip of a row, so the lanes of a wave
// descend through mostly the same nodes and read mostly the same leaf rows.
#include <mutex>
#include <unordered_map>

#pragma once

#include <algorithm>

#include "march.h"

namespace lq {
namespace {

constexpr int kBlock = 256;
constexpr int kRefillBelow = 40;     // refill when fewer lanes of a wave are busy
constexpr int kStepsPerCheck = 10;   // steps between refill checks
// the same for camera batches in tile order, whose rays in a wave (one
// pixel tile) end at similar steps: fewer checks pay more than early refills
constexpr int kTileRefillBelow = 16;
constexpr int kTileStepsPerCheck = 32;
constexpr int kXcds = 8;             // accelerator dies (XCDs) of an MI355X
constexpr int kRangesPerXcd = 2;     // ray counters (contiguous ranges) per die
constexpr int kRanges = kXcds * kRangesPerXcd;
static_assert(kRanges == kQueryCounters, "one counter per range");
static_assert(kRanges >= 1 && kRanges <= 64, "one bit per range in a 64-bit mask");
constexpr uint64_t kAllRanges = kRanges == 64 ? ~0ull : (1ull << kRanges) - 1ull;   // every range used up
constexpr int kMaxTries = 8;         // refill attempts per check

__device__ inline uint64_t lanemask_lt() {
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// The radiance and opacity of a finished ray go out as non-temporal stores:
// lanes finish at different steps, so each store fills only part of a line,
// and without the hint those partial lines occupy L2 until evicted
// (incoherent batches: room f32 5.81 -> 5.74 ms, f16 5.37 -> 5.28 ms).
template <class M>
__device__ inline void write_ray(const QueryArgs &a, int64_t i, const M &m, bool trace) {
    RayOut r;
    m.result(r);
    if (a.rgb) {
        __builtin_nontemporal_store(r.rgb[0], a.rgb + 3 * i);
        __builtin_nontemporal_store(r.rgb[1], a.rgb + 3 * i + 1);
        __builtin_nontemporal_store(r.rgb[2], a.rgb + 3 * i + 2);
    }
    if (a.alpha) __builtin_nontemporal_store(r.alpha, a.alpha + i);
    if (trace) {
        a.count[i] = r.count;
        a.hash[i] = r.hash;
        a.term_idx[i] = r.term_idx;
        a.n_comp[i] = r.n_comp;
        if (a.n_steps) a.n_steps[i] = r.n_steps;
    }
}

__device__ inline int64_t range_begin(int x, int64_t n) { return n * x / kRanges; }

// the persistent loop shared by the single- and multi-tree kernels;
// tree_index(ray) finds the tree a ray queries (once, when a lane takes the
// ray) and tree_at(k) returns tree k.  With TOP_LDS (one tree)
// the block copies the tree's top grid into LDS; otherwise each ray reads
// its tree's grid from global memory.  ORDER maps a position of the split
// to a ray: kOrderAny takes a.index, then the image tile order, then the
// position itself, whichever the arguments set; kOrderBatch only a.index or
// the position; kOrderTiles only the tile order.
enum { kOrderAny = 0, kOrderBatch = 1, kOrderTiles = 2 };

template <int ST, int DEG, bool ACC64, bool TRACE, bool SKIP, bool TOP_LDS, int MODEL, int ORDER, class TreeIndex,
          class TreeAt>
__device__ inline void persistent_query(const QueryArgs &a, unsigned long long *queue, TreeIndex tree_index,
                                        TreeAt tree_at) {
    __shared__ int32_t s_path[10 * kBlock];   // per-lane node path, [level][lane]
    int32_t *path = s_path + threadIdx.x;
    const int32_t *top_lds = nullptr;
    if constexpr (TOP_LDS) {
        __shared__ int32_t s_top[kTopCells];
        const DevTree &t0 = tree_at(0);
        const int32_t *src = SKIP ? t0.top_skip : t0.top;
        if (src) {
            for (int i = threadIdx.x; i < kTopCells; i += kBlock) s_top[i] = src[i];
            top_lds = s_top;
        }
        __syncthreads();
    }
    auto top_of = [&](const DevTree &t) -> const int32_t * {
        if constexpr (TOP_LDS) return top_lds;
        return SKIP ? t.top_skip : t.top;
    };
    constexpr int refill_below = ORDER == kOrderTiles ? kTileRefillBelow : kRefillBelow;
    constexpr int steps_per_check = ORDER == kOrderTiles ? kTileStepsPerCheck : kStepsPerCheck;
    Marcher<ST, DEG, ACC64, TRACE, SKIP, MODEL> m;
    int64_t ray = -1;            // ray held by this lane, -1 when idle
    int tk = 0;                  // tree of that ray
    uint32_t *ids = nullptr;
    // range this wave draws from (wave-uniform): one of its die's ranges
    int cur = (int)(blockIdx.x % kXcds) * kRangesPerXcd + (int)((blockIdx.x / kXcds) % kRangesPerXcd);
    uint64_t used_up = 0;           // ranges known to be exhausted (wave-uniform)
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n;
    for (;;) {
        bool want = ray < 0 && used_up != kAllRanges;
        uint64_t need = __ballot(want);
        const int busy = __popcll(__ballot(ray >= 0));
        if (__builtin_expect(need && busy < refill_below, 0)) {
            for (int tries = 0; need && tries < kMaxTries; ++tries) {
                const int cnt = __popcll(need);
                const int leader = __ffsll((unsigned long long)need) - 1;
                unsigned long long base = 0;
                if ((int)__lane_id() == leader) base = atomicAdd(queue + cur, (unsigned long long)cnt);
                const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)base, leader);
                const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
                base = ((unsigned long long)hi << 32) | lo;
                const int64_t start = range_begin(cur, n);
                const int64_t len = range_begin(cur + 1, n) - start;
                if (want) {
                    const int64_t slot = (int64_t)base + __popcll(need & lanemask_lt());
                    if (slot < len) {
                        const int64_t pos = start + slot;
                        int64_t idx = pos;
                        if constexpr (ORDER == kOrderTiles) {
                            idx = tile_order_pixel((uint32_t)pos, a.img_w, a.img_h);
                        } else {
                            if (a.index) idx = a.index[pos];
                            else if (ORDER == kOrderAny && a.img_w) idx = tile_order_pixel((uint32_t)pos, a.img_w, a.img_h);
                        }
                        ids = TRACE && a.max_ids > 0 ? a.leaf_ids + (size_t)idx * a.max_ids : nullptr;
                        tk = tree_index(idx);
                        if (m.init(tree_at(tk), a.o + 3 * idx, a.d + 3 * idx)) {
                            ray = idx;
                            want = false;
                        } else {
                            write_ray(a, idx, m, TRACE);   // no positive-length overlap: done
                        }
                    }
                }
                if ((int64_t)base + cnt >= len) {   // this range is used up: move on
                    used_up |= 1ull << cur;
                    for (int j = 1; j <= kRanges; ++j) {
                        const int c = (cur + j) % kRanges;
                        if (!(used_up & (1ull << c))) { cur = c; break; }
                    }
                }
                want = want && used_up != kAllRanges;
                need = __ballot(want);
            }
        }
        if (__all(ray < 0 && used_up == kAllRanges)) break;
        for (int k = 0; k < steps_per_check && ray >= 0; ++k) {
            const DevTree &tr = tree_at(tk);
            if (__builtin_expect(m.step(tr, a.model, a.flags, ids, TRACE ? a.max_ids : 0, path, kBlock, top_of(tr)), 0)) {
                write_ray(a, ray, m, TRACE);
                ray = -1;
            }
        }
    }
}

// MODEL >= 0 fixes the transmittance model at compile time (the plain
// queries), -1 takes it from the arguments.
template <int ST, int DEG, bool ACC64, bool TRACE, bool SKIP, int MODEL>
__global__ __launch_bounds__(kBlock) void k_query(const DevTree t, const QueryArgs a,
                                                  unsigned long long *queue) {
    persistent_query<ST, DEG, ACC64, TRACE, SKIP, true, MODEL, kOrderAny>(
        a, queue, [](int64_t) { return 0; }, [&](int) -> const DevTree & { return t; });
}

// The plain query (float32 accumulation, no trace) with a register budget
// for five waves per SIMD: it waits on dependent loads, and a fifth wave
// hides more of that than the few values the budget moves out of registers
// (spilled only on the path of rays that miss the box) cost.  Larger leaf
// rows (SH degree 3 and 4) hold more values per lane -- the row and the
// (l+1)^2 basis values -- and get a budget for fewer waves instead of
// spilling them.  The validation variants keep the default budget, which
// they need.  The kernels for one transmittance model take rays in batch
// order or, with TILES, in the tile order of a camera batch; the
// model-generic one (the validation flags) in whichever the arguments give.
template <int ST, int DEG>
constexpr int plain_waves_per_simd() {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int row_regs = ((1 + 3 * K) * Storage<ST>::bytes + 15) / 16 * 4;
    return row_regs + K <= 40 ? 5 : (row_regs + K <= 70 ? 4 : 3);
}

template <int ST, int DEG, bool SKIP, int MODEL, bool TILES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(plain_waves_per_simd<ST, DEG>())))
void k_query_plain(
    const DevTree t, const QueryArgs a, unsigned long long *queue) {
    constexpr int order = TILES ? kOrderTiles : (MODEL < 0 ? kOrderAny : kOrderBatch);
    persistent_query<ST, DEG, false, false, SKIP, true, MODEL, order>(
        a, queue, [](int64_t) { return 0; }, [&](int) -> const DevTree & { return t; });
}

template <int ST, int DEG, bool ACC64, bool TRACE, bool SKIP, int MODEL, bool TILES>
constexpr auto query_kernel() {
    if constexpr (!ACC64 && !TRACE) return k_query_plain<ST, DEG, SKIP, MODEL, TILES>;
    else return k_query<ST, DEG, ACC64, TRACE, SKIP, MODEL>;
}

// several trees: rays [offsets[k], offsets[k+1]) query trees[k]; the tree of
// a ray is found by binary search when a lane takes it.  The float32 kernels
// are specialised on the model like the plain ones, but keep the default
// register budget: a lane's tree fields come from memory and need registers
// (with the five-wave budget they spill, 10.7 vs 7.9 ms on the uneven batch).
template <int ST, int DEG, bool ACC64, bool SKIP, int MODEL>
__device__ inline void multi_query(const DevTree *trees, const int64_t *offsets, int n_trees, const QueryArgs &a,
                                   unsigned long long *queue) {
    auto tree_index = [&](int64_t ray) {
        int lo = 0, hi = n_trees;            // offsets[lo] <= ray < offsets[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offsets[mid] <= ray) lo = mid;
            else hi = mid;
        }
        return lo;
    };
    persistent_query<ST, DEG, ACC64, false, SKIP, false, MODEL, kOrderBatch>(
        a, queue, tree_index, [&](int k) -> const DevTree & { return trees[k]; });
}

template <int ST, int DEG, bool ACC64, bool SKIP>
__global__ __launch_bounds__(kBlock) void k_query_multi(const DevTree *trees, const int64_t *offsets,
                                                        int n_trees, const QueryArgs a,
                                                        unsigned long long *queue) {
    multi_query<ST, DEG, ACC64, SKIP, -1>(trees, offsets, n_trees, a, queue);
}

template <int ST, int DEG, bool SKIP, int MODEL>
__global__ __launch_bounds__(kBlock) void k_query_multi_plain(
    const DevTree *trees, const int64_t *offsets, int n_trees, const QueryArgs a, unsigned long long *queue) {
    multi_query<ST, DEG, false, SKIP, MODEL>(trees, offsets, n_trees, a, queue);
}

__global__ void k_zero_u64(unsigned long long *p) { p[threadIdx.x] = 0ull; }

// resident blocks of a kernel on the current device (cached)
template <class Kern>
int resident_blocks(Kern kern) {
    static std::mutex mu;
    static std::unordered_map<int, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 1;
    (void)hipGetLastError();
    int nb = per_cu * cus;
    cache[dev] = nb;
    return nb;
}

template <int ST, int DEG, bool ACC64, bool TRACE, bool SKIP, int MODEL = -1, bool TILES = false>
hipError_t launch_one(const DevTree &t, const QueryArgs &a, hipStream_t s) {
    auto kern = query_kernel<ST, DEG, ACC64, TRACE, SKIP, MODEL, TILES>();
    const int64_t need_blocks = (a.n + kBlock - 1) / kBlock;
    const int64_t nb = std::min<int64_t>(need_blocks, resident_blocks(kern));
    unsigned long long *queue = a.counters;
    hipError_t e = hipSuccess;
    if (!queue && (e = hipMallocAsync((void **)&queue, kRanges * sizeof(unsigned long long), s)) != hipSuccess)
        return e;
    // cleared by a kernel (not a memset node), so the launch can be captured
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(kRanges), 0, s, queue);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kBlock), 0, s, t, a, queue);
    e = hipGetLastError();
    hipError_t f = a.counters ? hipSuccess : hipFreeAsync(queue, s);
    return e != hipSuccess ? e : f;
}

template <int ST, int DEG>
hipError_t launch_deg(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    // traces record every data leaf, so they march the full table; so do
    // queries that composite every leaf
    const bool acc64 = (a.flags & LQ_FP64_ACCUM) != 0;
    const bool full = trace || (a.flags & LQ_NO_SIGMA_SKIP) != 0;
    // a trace of the pruned table (the production query's work)
    if (trace && (a.flags & LQ_TRACE_PRUNED)) return launch_one<ST, DEG, false, true, true>(t, a, s);
    if (trace) return acc64 ? launch_one<ST, DEG, true, true, false>(t, a, s)
                            : launch_one<ST, DEG, false, true, false>(t, a, s);
    if (full) return acc64 ? launch_one<ST, DEG, true, false, false>(t, a, s)
                           : launch_one<ST, DEG, false, false, false>(t, a, s);
    if (acc64) return launch_one<ST, DEG, true, false, true>(t, a, s);
    // the plain kernels of camera batches have the tile order built in
    if (a.img_w)
        return a.model == LQ_EXP ? launch_one<ST, DEG, false, false, true, LQ_EXP, true>(t, a, s)
                                 : launch_one<ST, DEG, false, false, true, LQ_LINEAR, true>(t, a, s);
    return a.model == LQ_EXP ? launch_one<ST, DEG, false, false, true, LQ_EXP>(t, a, s)
                             : launch_one<ST, DEG, false, false, true, LQ_LINEAR>(t, a, s);
}

template <int ST>
hipError_t launch_st(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    switch (t.sh_degree) {
        case 0: return launch_deg<ST, 0>(t, a, trace, s);
        case 1: return launch_deg<ST, 1>(t, a, trace, s);
        case 2: return launch_deg<ST, 2>(t, a, trace, s);
        case 3: return launch_deg<ST, 3>(t, a, trace, s);
        case 4: return launch_deg<ST, 4>(t, a, trace, s);
    }
    return hipErrorInvalidValue;
}

template <int ST, int DEG, bool ACC64, bool SKIP, int MODEL = -1>
hipError_t launch_multi_one(const DevTree *trees, const int64_t *offsets, int n_trees, const QueryArgs &a,
                            hipStream_t s) {
    auto kern = [] {
        if constexpr (!ACC64 && MODEL >= 0) return k_query_multi_plain<ST, DEG, SKIP, MODEL>;
        else return k_query_multi<ST, DEG, ACC64, SKIP>;
    }();
    const int64_t need_blocks = (a.n + kBlock - 1) / kBlock;
    const int64_t nb = std::min<int64_t>(need_blocks, resident_blocks(kern));
    unsigned long long *queue = nullptr;
    hipError_t e = hipMallocAsync((void **)&queue, kRanges * sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(kRanges), 0, s, queue);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kBlock), 0, s, trees, offsets, n_trees, a, queue);
    e = hipGetLastError();
    hipError_t f = hipFreeAsync(queue, s);
    return e != hipSuccess ? e : f;
}

template <int ST, int DEG>
hipError_t launch_multi_deg(const DevTree *trees, const int64_t *offsets, int n_trees, const QueryArgs &a,
                            hipStream_t s) {
    const bool acc64 = (a.flags & LQ_FP64_ACCUM) != 0;
    const bool full = (a.flags & LQ_NO_SIGMA_SKIP) != 0;
    if (full) return acc64 ? launch_multi_one<ST, DEG, true, false>(trees, offsets, n_trees, a, s)
                           : launch_multi_one<ST, DEG, false, false>(trees, offsets, n_trees, a, s);
    if (acc64) return launch_multi_one<ST, DEG, true, true>(trees, offsets, n_trees, a, s);
    return a.model == LQ_EXP ? launch_multi_one<ST, DEG, false, true, LQ_EXP>(trees, offsets, n_trees, a, s)
                             : launch_multi_one<ST, DEG, false, true, LQ_LINEAR>(trees, offsets, n_trees, a, s);
}

template <int ST>
hipError_t launch_multi_st(int deg, const DevTree *trees, const int64_t *offsets, int n_trees, const QueryArgs &a,
                           hipStream_t s) {
    switch (deg) {
        case 2: return launch_multi_deg<ST, 2>(trees, offsets, n_trees, a, s);
        case 3: return launch_multi_deg<ST, 3>(trees, offsets, n_trees, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace lq
