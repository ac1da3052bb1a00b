// api.hip -- host side of the C ABI declared in include/lumiq.h: argument
// checks, plenoctree validation and upload, SH constants, error reporting.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "lq_internal.h"

struct lq_octree {
    int device;
    lq::DevTree t;
    int32_t *d_child;
    int32_t *d_child_skip;
    int32_t *d_top;   // grids of child and child_skip, or null (depth <= kTopLevel)
    void *d_rows;
    int64_t bytes;
};

namespace lq {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

static lq_status fail(lq_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

static lq_status hip_fail(hipError_t e, const char *what) {
    return fail(LQ_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------ conversions
uint16_t f32_to_f16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    uint32_t sign = (u >> 16) & 0x8000u;
    uint32_t ex = (u >> 23) & 0xFFu;
    uint32_t man = u & 0x7FFFFFu;
    if (ex == 0xFFu) return (uint16_t)(sign | 0x7C00u | (man ? 0x200u : 0u));
    int e = (int)ex - 127 + 15;
    if (e >= 31) return (uint16_t)(sign | 0x7C00u);          // overflow -> inf
    if (e <= 0) {                                             // subnormal or zero
        if (e < -10) return (uint16_t)sign;
        man |= 0x800000u;
        int shift = 14 - e;                                   // 1 - e + 13
        uint32_t half = man >> shift;
        uint32_t rem = man & ((1u << shift) - 1u);
        uint32_t mid = 1u << (shift - 1);
        if (rem > mid || (rem == mid && (half & 1u))) ++half;
        return (uint16_t)(sign | half);
    }
    uint32_t half = ((uint32_t)e << 10) | (man >> 13);
    uint32_t rem = man & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (half & 1u))) ++half;   // may carry into inf
    return (uint16_t)(sign | half);
}

uint16_t f32_to_bf16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

int row_bytes(int storage, int K);   // octree_query.hip

// ------------------------------------------------------------ validation
// On success, *bfs (if given) receives the nodes in breadth-first order.
static lq_status validate_desc(const lq_octree_desc *d, std::vector<int32_t> *bfs = nullptr) {
    if (!d) return fail(LQ_ERR_INVALID_ARG, "descriptor is NULL");
    if (d->max_depth < 1 || d->max_depth > 10) return fail(LQ_ERR_FORMAT, "max_depth must be in [1, 10]");
    if (d->sh_degree < 0 || d->sh_degree > 4) return fail(LQ_ERR_FORMAT, "sh_degree must be in [0, 4]");
    if (d->n_nodes < 1) return fail(LQ_ERR_FORMAT, "n_nodes must be >= 1 (the root)");
    // the kernels address child slots with 32-bit offsets (node * 8 + octant)
    if (d->n_nodes >= (1 << 29)) return fail(LQ_ERR_UNSUPPORTED, "n_nodes must be below 2^29");
    if (d->n_leaves < 0) return fail(LQ_ERR_FORMAT, "n_leaves must be >= 0");
    if (!d->child) return fail(LQ_ERR_INVALID_ARG, "child table is NULL");
    if (d->n_leaves > 0 && (!d->sigma || !d->sh)) return fail(LQ_ERR_INVALID_ARG, "sigma/sh is NULL");
    if (!(d->l_max > 0.0f) || !isfinite(d->l_max)) return fail(LQ_ERR_FORMAT, "l_max must be finite and > 0");
    if (!isfinite(d->sigma_min) || !(d->alpha_max > 0.0f) || !(d->alpha_max <= 1.0f))
        return fail(LQ_ERR_FORMAT, "sigma_min must be finite and alpha_max in (0, 1]");
    // the child table must be a tree with leaves exactly one level above max depth
    const int D = d->max_depth;
    std::vector<uint8_t> seen_node(d->n_nodes, 0);
    std::vector<uint8_t> seen_leaf(d->n_leaves, 0);
    std::vector<int32_t> cur{0}, nxt;
    seen_node[0] = 1;
    int64_t nodes_reached = 1;
    if (bfs) bfs->assign(1, 0);
    for (int level = 0; level < D && !cur.empty(); ++level) {
        nxt.clear();
        for (int32_t node : cur) {
            for (int oct = 0; oct < 8; ++oct) {
                int32_t c = d->child[(size_t)node * 8 + oct];
                if (c == 0) continue;
                if (c > 0) {
                    if (level + 1 >= D) return fail(LQ_ERR_FORMAT, "internal node below max_depth - 1");
                    if (c >= d->n_nodes || seen_node[c]) return fail(LQ_ERR_FORMAT, "bad or repeated node index");
                    seen_node[c] = 1;
                    ++nodes_reached;
                    nxt.push_back(c);
                } else {
                    int64_t leaf = -(int64_t)c - 1;
                    if (level + 1 != D) return fail(LQ_ERR_FORMAT, "data leaf above max_depth");
                    if (leaf >= d->n_leaves || seen_leaf[leaf]) return fail(LQ_ERR_FORMAT, "bad or repeated leaf index");
                    seen_leaf[leaf] = 1;
                }
            }
        }
        if (bfs) bfs->insert(bfs->end(), nxt.begin(), nxt.end());
        cur.swap(nxt);
    }
    if (nodes_reached != d->n_nodes) return fail(LQ_ERR_FORMAT, "unreachable nodes in the child table");
    return LQ_OK;
}

// Dense top grid of a child table (see DevTree::top): the descent from the
// root along every cell of level kTopLevel; cells are indexed z, y, x.
static std::vector<int32_t> top_grid(const int32_t *table, int depth) {
    std::vector<int32_t> g;
    if (depth <= kTopLevel) return g;
    const int R = 1 << kTopLevel;
    g.resize(kTopCells);
    for (int z = 0; z < R; ++z)
        for (int y = 0; y < R; ++y)
            for (int x = 0; x < R; ++x) {
                int32_t node = 0, e = 0;
                for (int level = 0; level < kTopLevel; ++level) {
                    const int b = kTopLevel - 1 - level;
                    const int oct = ((x >> b) & 1) | (((y >> b) & 1) << 1) | (((z >> b) & 1) << 2);
                    const int32_t c = table[(size_t)node * 8 + oct];
                    if (c <= 0) {   // leaves sit at max depth > kTopLevel: c is empty
                        e = -(level + 1);
                        break;
                    }
                    node = c;
                    e = c;
                }
                g[((size_t)z * R + y) * R + x] = e;
            }
    return g;
}

// Child table without the leaves for which keep_leaf() is false and without
// the nodes that are left empty; the root stays node 0, order breadth-first.
template <class Keep>
static std::vector<int32_t> prune_tree(const lq_octree_desc *d, const std::vector<int32_t> &bfs,
                                       Keep keep_leaf) {
    const size_t nn = (size_t)d->n_nodes;
    std::vector<uint8_t> alive(nn, 0);
    for (size_t j = bfs.size(); j-- > 0;) {          // children before parents
        const int32_t node = bfs[j];
        uint8_t any = 0;
        for (int oct = 0; oct < 8; ++oct) {
            const int32_t c = d->child[(size_t)node * 8 + oct];
            if (c > 0) any |= alive[c];
            else if (c < 0) any |= keep_leaf(-(int64_t)c - 1) ? 1 : 0;
        }
        alive[node] = any;
    }
    std::vector<int32_t> new_index(nn, 0);
    int32_t next = 0;
    for (int32_t node : bfs)
        if (node == 0 || alive[node]) new_index[node] = next++;
    std::vector<int32_t> out((size_t)next * 8, 0);
    for (int32_t node : bfs) {
        if (node != 0 && !alive[node]) continue;
        int32_t *row = out.data() + (size_t)new_index[node] * 8;
        for (int oct = 0; oct < 8; ++oct) {
            const int32_t c = d->child[(size_t)node * 8 + oct];
            if (c > 0 && alive[c]) row[oct] = new_index[c];
            else if (c < 0 && keep_leaf(-(int64_t)c - 1)) row[oct] = c;
        }
    }
    return out;
}

}  // namespace lq

using namespace lq;

extern "C" {

const char *lq_last_error(void) { return g_err.c_str(); }
const char *lq_version(void) { return "lumiq 0.1 (gfx950)"; }

lq_status lq_load_octree_desc(const lq_octree_desc *desc, int storage, int device, lq_octree **out) {
    if (!out) return fail(LQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (storage != LQ_F32 && storage != LQ_F16 && storage != LQ_BF16)
        return fail(LQ_ERR_INVALID_ARG, "storage must be LQ_F32, LQ_F16 or LQ_BF16");
    std::vector<int32_t> bfs;
    lq_status st = validate_desc(desc, &bfs);
    if (st != LQ_OK) return st;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(LQ_ERR_HIP, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return fail(LQ_ERR_INVALID_ARG, "device index out of range");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");

    const int K = (desc->sh_degree + 1) * (desc->sh_degree + 1);
    const int esz = storage == LQ_F32 ? 4 : 2;
    const int rb = row_bytes(storage, K);
    const int64_t nl = desc->n_leaves;
    std::vector<uint8_t> rows((size_t)nl * rb, 0);
    for (int64_t i = 0; i < nl; ++i) {
        uint8_t *row = rows.data() + (size_t)i * rb;
        for (int j = 0; j < 1 + 3 * K; ++j) {
            float v = j == 0 ? desc->sigma[i] : desc->sh[(size_t)i * 3 * K + (j - 1)];
            if (storage == LQ_F32) {
                memcpy(row + 4 * j, &v, 4);
            } else {
                uint16_t b = storage == LQ_F16 ? f32_to_f16_rne(v) : f32_to_bf16_rne(v);
                memcpy(row + esz * j, &b, 2);
            }
        }
    }
    // density as stored (after rounding), compared like the kernel does
    auto stored_sigma = [&](int64_t leaf) -> float {
        if (storage == LQ_F32) return desc->sigma[leaf];
        uint16_t b;
        memcpy(&b, rows.data() + (size_t)leaf * rb, 2);
        if (storage == LQ_BF16) {
            uint32_t u = (uint32_t)b << 16;
            float f;
            memcpy(&f, &u, 4);
            return f;
        }
        return (float)__builtin_bit_cast(_Float16, b);
    };
    const float smin = desc->sigma_min;
    std::vector<int32_t> skip = prune_tree(desc, bfs, [&](int64_t leaf) { return stored_sigma(leaf) >= smin; });

    lq_octree *t = new (std::nothrow) lq_octree();
    if (!t) return fail(LQ_ERR_OOM, "host allocation failed");
    t->device = device;
    const size_t child_bytes = (size_t)desc->n_nodes * 32;
    const size_t skip_bytes = skip.size() * 4;
    const size_t row_total = rows.size() ? rows.size() : 64;
    std::vector<int32_t> tops = top_grid(desc->child, desc->max_depth);
    const std::vector<int32_t> top_skip = top_grid(skip.data(), desc->max_depth);
    tops.insert(tops.end(), top_skip.begin(), top_skip.end());
    const size_t top_bytes = tops.size() * 4;
    t->d_child = nullptr;
    t->d_child_skip = nullptr;
    t->d_top = nullptr;
    t->d_rows = nullptr;
    auto release = [&]() {
        (void)hipFree(t->d_child);
        (void)hipFree(t->d_child_skip);
        (void)hipFree(t->d_top);
        (void)hipFree(t->d_rows);
        delete t;
    };
    if (hipMalloc((void **)&t->d_child, child_bytes) != hipSuccess ||
        hipMalloc((void **)&t->d_child_skip, skip_bytes) != hipSuccess ||
        (top_bytes && hipMalloc((void **)&t->d_top, top_bytes) != hipSuccess) ||
        hipMalloc(&t->d_rows, row_total) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(LQ_ERR_OOM, "device allocation of the tree tables failed");
    }
    e = hipMemcpy(t->d_child, desc->child, child_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t->d_child_skip, skip.data(), skip_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && top_bytes) e = hipMemcpy(t->d_top, tops.data(), top_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && rows.size()) e = hipMemcpy(t->d_rows, rows.data(), rows.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "uploading the tree");
    }
    t->bytes = (int64_t)(child_bytes + skip_bytes + top_bytes + row_total);
    DevTree &dt = t->t;
    dt.child = t->d_child;
    dt.child_skip = t->d_child_skip;
    dt.top = top_bytes ? t->d_top : nullptr;
    dt.top_skip = top_bytes ? t->d_top + kTopCells : nullptr;
    dt.rows = t->d_rows;
    dt.depth = desc->max_depth;
    dt.sh_degree = desc->sh_degree;
    dt.K = K;
    dt.storage = storage;
    dt.n_nodes = desc->n_nodes;
    dt.n_leaves = desc->n_leaves;
    dt.row_elems = rb / esz;
    dt.l_max = desc->l_max;
    dt.sigma_min = desc->sigma_min;
    dt.alpha_max = desc->alpha_max;
    *out = t;
    return LQ_OK;
}

lq_status lq_load_octree(const char *path, int storage, int device, lq_octree **out) {
    if (!out) return fail(LQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!path) return fail(LQ_ERR_INVALID_ARG, "path is NULL");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(LQ_ERR_IO, std::string("cannot open ") + path);
    struct {
        char magic[4];
        uint32_t version;
        int32_t depth, deg, n_nodes, n_leaves;
        float l_max, sigma_min, alpha_max;
        uint32_t reserved;
    } hdr;
    static_assert(sizeof(hdr) == 40, "header layout");
    lq_status st = LQ_OK;
    std::vector<int32_t> child;
    std::vector<float> sigma, sh;
    if (fread(&hdr, sizeof(hdr), 1, f) != 1 || memcmp(hdr.magic, "LQOT", 4) != 0 || hdr.version != 1) {
        st = fail(LQ_ERR_FORMAT, "not a version-1 LQOT plenoctree file");
    } else if (hdr.depth < 1 || hdr.depth > 10 || hdr.deg < 0 || hdr.deg > 4 || hdr.n_nodes < 1 ||
               hdr.n_leaves < 0 || hdr.n_nodes > (1 << 30) || hdr.n_leaves > (1 << 30)) {
        st = fail(LQ_ERR_FORMAT, "header out of range");
    } else {
        const size_t K = (size_t)(hdr.deg + 1) * (hdr.deg + 1);
        child.resize((size_t)hdr.n_nodes * 8);
        sigma.resize((size_t)hdr.n_leaves);
        sh.resize((size_t)hdr.n_leaves * 3 * K);
        if (fread(child.data(), 4, child.size(), f) != child.size() ||
            fread(sigma.data(), 4, sigma.size(), f) != sigma.size() ||
            fread(sh.data(), 4, sh.size(), f) != sh.size())
            st = fail(LQ_ERR_FORMAT, "truncated plenoctree file");
    }
    fclose(f);
    if (st != LQ_OK) return st;
    lq_octree_desc d;
    d.max_depth = hdr.depth;
    d.sh_degree = hdr.deg;
    d.n_nodes = hdr.n_nodes;
    d.n_leaves = hdr.n_leaves;
    d.l_max = hdr.l_max;
    d.sigma_min = hdr.sigma_min;
    d.alpha_max = hdr.alpha_max;
    d.child = child.data();
    d.sigma = sigma.data();
    d.sh = sh.data();
    return lq_load_octree_desc(&d, storage, device, out);
}

void lq_free_octree(lq_octree *t) {
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    (void)hipFree(t->d_child);
    (void)hipFree(t->d_child_skip);
    (void)hipFree(t->d_top);
    (void)hipFree(t->d_rows);
    (void)hipSetDevice(cur);
    delete t;
}

lq_status lq_octree_download(const lq_octree *t, int32_t *child, float *sigma, float *sh) {
    if (!t) return fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    hipError_t e = hipSetDevice(t->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const DevTree &dt = t->t;
    if (child && (e = hipMemcpy(child, t->d_child, (size_t)dt.n_nodes * 32, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "reading the child table");
    if (!sigma && !sh) return LQ_OK;
    const int esz = dt.storage == LQ_F32 ? 4 : 2;
    const size_t rb = (size_t)dt.row_elems * esz;
    std::vector<uint8_t> rows((size_t)dt.n_leaves * rb);
    if (!rows.empty() && (e = hipMemcpy(rows.data(), t->d_rows, rows.size(), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "reading the leaf rows");
    auto value = [&](const uint8_t *row, int j) -> float {
        if (dt.storage == LQ_F32) {
            float f;
            memcpy(&f, row + 4 * j, 4);
            return f;
        }
        uint16_t b;
        memcpy(&b, row + 2 * j, 2);
        if (dt.storage == LQ_BF16) {
            const uint32_t u = (uint32_t)b << 16;
            float f;
            memcpy(&f, &u, 4);
            return f;
        }
        return (float)__builtin_bit_cast(_Float16, b);
    };
    for (int64_t i = 0; i < dt.n_leaves; ++i) {
        const uint8_t *row = rows.data() + (size_t)i * rb;
        if (sigma) sigma[i] = value(row, 0);
        if (sh)
            for (int j = 0; j < 3 * dt.K; ++j) sh[(size_t)i * 3 * dt.K + j] = value(row, 1 + j);
    }
    return LQ_OK;
}

lq_status lq_octree_info(const lq_octree *t, int64_t *device_bytes, int32_t *n_nodes, int32_t *n_leaves,
                         int32_t *max_depth, int32_t *sh_degree, int32_t *storage) {
    if (!t) return fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    if (device_bytes) *device_bytes = t->bytes;
    if (n_nodes) *n_nodes = t->t.n_nodes;
    if (n_leaves) *n_leaves = t->t.n_leaves;
    if (max_depth) *max_depth = t->t.depth;
    if (sh_degree) *sh_degree = t->t.sh_degree;
    if (storage) *storage = t->t.storage;
    return LQ_OK;
}

}  // extern "C"

namespace lq {

// A device pointer on `device` whose allocation holds `bytes` from ptr on.
static lq_status check_dev(const void *ptr, size_t bytes, int device, const char *name) {
    if (!ptr) return fail(LQ_ERR_INVALID_ARG, std::string(name) + " is NULL");
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LQ_ERR_INVALID_ARG, std::string(name) + " is not a device pointer");
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(LQ_ERR_INVALID_ARG, std::string(name) + " is not a device pointer");
    if (at.device != device) return fail(LQ_ERR_INVALID_ARG, std::string(name) + " is on another device");
    if ((uintptr_t)ptr % 4 != 0) return fail(LQ_ERR_INVALID_ARG, std::string(name) + " is not 4-byte aligned");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LQ_ERR_INVALID_ARG, std::string(name) + ": allocation range unknown");
    }
    if ((const char *)ptr + bytes > (const char *)base + size)
        return fail(LQ_ERR_INVALID_ARG, std::string(name) + " is smaller than the batch needs");
    return LQ_OK;
}

lq_status check_device_array(const void *ptr, size_t bytes, int device, const char *name) {
    return check_dev(ptr, bytes, device, name);
}

int octree_device(const lq_octree *t) { return t->device; }

static lq_status query_common(const lq_octree *t, const QueryArgs &a, bool trace, void *stream) {
    if (!t) return fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    if (a.n < 0) return fail(LQ_ERR_INVALID_ARG, "n must be >= 0");
    if (a.model != LQ_LINEAR && a.model != LQ_EXP) return fail(LQ_ERR_INVALID_ARG, "model must be LQ_LINEAR or LQ_EXP");
    const uint32_t known = LQ_NO_EARLY_TERM | LQ_FP64_ACCUM | LQ_NO_SIGMA_SKIP | (trace ? LQ_TRACE_PRUNED : 0u);
    if (a.flags & ~known) return fail(LQ_ERR_INVALID_ARG, "unknown flag bits");
    if ((a.flags & LQ_TRACE_PRUNED) && (a.flags & (LQ_FP64_ACCUM | LQ_NO_SIGMA_SKIP)))
        return fail(LQ_ERR_INVALID_ARG, "LQ_TRACE_PRUNED combines with LQ_NO_EARLY_TERM only");
    if (a.n > ((int64_t)1 << 40)) return fail(LQ_ERR_INVALID_ARG, "n too large");
    if (a.n == 0) return LQ_OK;
    hipError_t e = hipSetDevice(t->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t n = (size_t)a.n;
    lq_status st;
    if ((st = check_dev(a.o, n * 12, t->device, "origins")) != LQ_OK) return st;
    if ((st = check_dev(a.d, n * 12, t->device, "dirs")) != LQ_OK) return st;
    if (!trace && !a.rgb) return fail(LQ_ERR_INVALID_ARG, "rgb is NULL");
    if (a.rgb && (st = check_dev(a.rgb, n * 12, t->device, "rgb")) != LQ_OK) return st;
    if (a.alpha && (st = check_dev(a.alpha, n * 4, t->device, "alpha")) != LQ_OK) return st;
    if (trace) {
        if ((st = check_dev(a.count, n * 4, t->device, "count")) != LQ_OK) return st;
        if ((st = check_dev(a.hash, n * 8, t->device, "hash")) != LQ_OK) return st;
        if ((uintptr_t)a.hash % 8) return fail(LQ_ERR_INVALID_ARG, "hash is not 8-byte aligned");
        if ((st = check_dev(a.term_idx, n * 4, t->device, "term_idx")) != LQ_OK) return st;
        if ((st = check_dev(a.n_comp, n * 4, t->device, "n_comp")) != LQ_OK) return st;
        if (a.n_steps && (st = check_dev(a.n_steps, n * 4, t->device, "n_steps")) != LQ_OK) return st;
        if (a.max_ids < 0) return fail(LQ_ERR_INVALID_ARG, "max_ids must be >= 0");
        if (a.max_ids > 0 && (st = check_dev(a.leaf_ids, n * (size_t)a.max_ids * 4, t->device, "leaf_ids")) != LQ_OK)
            return st;
    }
    e = launch_query(t->t, a, trace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launching the emission query");
    return LQ_OK;
}

lq_status query_scratch(const lq_octree *t, const float *o, const float *d, int64_t n_max, const int64_t *index,
                        const unsigned long long *n_dev, float *rgb, float *alpha, int model, hipStream_t s) {
    QueryArgs a{};
    a.o = o;
    a.d = d;
    a.n = n_max;
    a.rgb = rgb;
    a.alpha = alpha;
    a.model = model;
    a.index = index;
    a.n_dev = n_dev;
    hipError_t e = launch_query(t->t, a, false, s);
    if (e != hipSuccess) return hip_fail(e, "launching the emission query");
    return LQ_OK;
}

lq_status query_indexed(const lq_octree *t, const float *o, const float *d, int64_t n_max, const int64_t *index,
                        const unsigned long long *n_dev, float *rgb, hipStream_t s) {
    if (!t) return fail(LQ_ERR_INVALID_ARG, "fallback tree is NULL");
    QueryArgs a{};
    a.o = o;
    a.d = d;
    a.n = n_max;
    a.rgb = rgb;
    a.model = LQ_LINEAR;
    a.index = index;
    a.n_dev = n_dev;
    hipError_t e = launch_query(t->t, a, false, s);
    if (e != hipSuccess) return hip_fail(e, "launching the fallback query");
    return LQ_OK;
}

}  // namespace lq

extern "C" {

lq_status lq_query_radiance(const lq_octree *tree, const float *origins, const float *dirs, int64_t n,
                            float *rgb, float *alpha, int model, uint32_t flags, void *hip_stream) {
    QueryArgs a{};
    a.o = origins;
    a.d = dirs;
    a.n = n;
    a.rgb = rgb;
    a.alpha = alpha;
    a.model = model;
    a.flags = flags;
    return query_common(tree, a, false, hip_stream);
}

}  // extern "C"

namespace lq {

// Ray counters of lq_query_radiance_noalloc: a file-scope device array (one
// copy on every GPU the library runs on, held until the process ends).  In
// host code its name is not a device address; the address is looked up once
// per device, with that device current, and only that pointer is used.
static __device__ __align__(256) unsigned long long scratch[kQueryCounters];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned long long *g_scratch_ptr[kMaxDevices] = {};

static lq_status scratch_counters(int device, unsigned long long **out) {
    if (device < 0 || device >= kMaxDevices) return fail(LQ_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress of the counter array");
        g_scratch_ptr[device] = static_cast<unsigned long long *>(p);
    }
    *out = g_scratch_ptr[device];
    return LQ_OK;
}

}  // namespace lq

extern "C" {

lq_status lq_query_radiance_noalloc(const lq_octree *tree, const float *origins, const float *dirs, int64_t n,
                                    float *rgb, float *alpha, int model, uint32_t flags, void *hip_stream) {
    if (!tree) return fail(LQ_ERR_INVALID_ARG, "tree is NULL");
    QueryArgs a{};
    a.o = origins;
    a.d = dirs;
    a.n = n;
    a.rgb = rgb;
    a.alpha = alpha;
    a.model = model;
    a.flags = flags;
    lq_status st = scratch_counters(tree->device, &a.counters);
    if (st != LQ_OK) return st;
    return query_common(tree, a, false, hip_stream);
}

lq_status lq_query_radiance_image(const lq_octree *tree, const float *origins, const float *dirs, int32_t width,
                                  int32_t height, float *rgb, float *alpha, int model, uint32_t flags,
                                  void *hip_stream) {
    if (width < 0 || height < 0) return fail(LQ_ERR_INVALID_ARG, "width and height must be >= 0");
    const int64_t n = (int64_t)width * height;
    if (n > INT32_MAX) return fail(LQ_ERR_INVALID_ARG, "width * height must be < 2^31");
    QueryArgs a{};
    a.o = origins;
    a.d = dirs;
    a.n = n;
    a.rgb = rgb;
    a.alpha = alpha;
    a.model = model;
    a.flags = flags;
    a.img_w = (uint32_t)width;
    a.img_h = (uint32_t)height;
    return query_common(tree, a, false, hip_stream);
}

lq_status lq_query_radiance_multi(const lq_octree *const *trees, int32_t n_trees, const int64_t *ray_offsets,
                                  const float *origins, const float *dirs, float *rgb, float *alpha, int model,
                                  uint32_t flags, void *hip_stream) {
    if (!trees || n_trees <= 0 || !ray_offsets) return fail(LQ_ERR_INVALID_ARG, "trees/ray_offsets missing");
    if (n_trees > 65536) return fail(LQ_ERR_INVALID_ARG, "too many trees");
    if (ray_offsets[0] != 0) return fail(LQ_ERR_INVALID_ARG, "ray_offsets[0] must be 0");
    for (int k = 0; k < n_trees; ++k) {
        if (!trees[k]) return fail(LQ_ERR_INVALID_ARG, "a tree is NULL");
        if (ray_offsets[k + 1] < ray_offsets[k]) return fail(LQ_ERR_INVALID_ARG, "ray_offsets must not decrease");
        if (trees[k]->device != trees[0]->device || trees[k]->t.storage != trees[0]->t.storage ||
            trees[k]->t.sh_degree != trees[0]->t.sh_degree)
            return fail(LQ_ERR_UNSUPPORTED, "all trees must share device, storage and SH degree");
    }
    if (trees[0]->t.sh_degree != 2 && trees[0]->t.sh_degree != 3)
        return fail(LQ_ERR_UNSUPPORTED, "the multi-tree query is built for SH degrees 2 and 3");
    const int64_t n = ray_offsets[n_trees];
    if (n > ((int64_t)1 << 40)) return fail(LQ_ERR_INVALID_ARG, "ray_offsets[n_trees] too large");
    QueryArgs a{};
    a.o = origins;
    a.d = dirs;
    a.n = n;
    a.rgb = rgb;
    a.alpha = alpha;
    a.model = model;
    a.flags = flags;
    if (a.model != LQ_LINEAR && a.model != LQ_EXP) return fail(LQ_ERR_INVALID_ARG, "bad model");
    if (a.flags & ~(uint32_t)(LQ_NO_EARLY_TERM | LQ_FP64_ACCUM | LQ_NO_SIGMA_SKIP))
        return fail(LQ_ERR_INVALID_ARG, "unknown flag bits");
    if (n == 0) return LQ_OK;
    const int dev = trees[0]->device;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    lq_status st;
    if ((st = check_dev(origins, n * 12, dev, "origins")) != LQ_OK) return st;
    if ((st = check_dev(dirs, n * 12, dev, "dirs")) != LQ_OK) return st;
    if ((st = check_dev(rgb, n * 12, dev, "rgb")) != LQ_OK) return st;
    if (alpha && (st = check_dev(alpha, n * 4, dev, "alpha")) != LQ_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<DevTree> host_trees(n_trees);
    for (int k = 0; k < n_trees; ++k) host_trees[k] = trees[k]->t;
    const size_t tb = sizeof(DevTree) * (size_t)n_trees, ob = sizeof(int64_t) * (size_t)(n_trees + 1);
    unsigned char *buf = nullptr;
    if ((e = hipMallocAsync((void **)&buf, tb + ob, s)) != hipSuccess) return hip_fail(e, "hipMallocAsync");
    e = hipMemcpyAsync(buf, host_trees.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(buf + tb, ray_offsets, ob, hipMemcpyHostToDevice, s);
    // the host copies above are staged from pageable memory: keep them alive
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = launch_query_multi(trees[0]->t.storage, trees[0]->t.sh_degree, reinterpret_cast<DevTree *>(buf),
                               reinterpret_cast<int64_t *>(buf + tb), n_trees, a, s);
    (void)hipFreeAsync(buf, s);
    if (e != hipSuccess) return hip_fail(e, "launching the multi-tree query");
    return LQ_OK;
}

lq_status lq_query_trace(const lq_octree *tree, const float *origins, const float *dirs, int64_t n,
                         float *rgb, float *alpha, int model, uint32_t flags, uint32_t *count,
                         uint64_t *hash, int32_t *term_idx, uint32_t *n_comp, uint32_t *n_steps,
                         uint32_t *leaf_ids, int32_t max_ids, void *hip_stream) {
    QueryArgs a{};
    a.o = origins;
    a.d = dirs;
    a.n = n;
    a.rgb = rgb;
    a.alpha = alpha;
    a.model = model;
    a.flags = flags;
    a.count = count;
    a.hash = hash;
    a.term_idx = term_idx;
    a.n_comp = n_comp;
    a.n_steps = n_steps;
    a.leaf_ids = leaf_ids;
    a.max_ids = max_ids;
    return query_common(tree, a, true, hip_stream);
}

}  // extern "C"
