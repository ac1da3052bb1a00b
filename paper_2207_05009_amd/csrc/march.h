// march.h -- the per-ray emission query (traversal + compositing).
//
// One call marches one ray through the plenoctree (Sec. 5) and evaluates
// Eq. 3 exactly over every data leaf it crosses: density and emission are
// constant in a leaf, so the leaf contributes w = T_in - T_out times Phi
// (Sec. 4.2, Eq. 6), with T by the linear model (Sec. 4.1, Eq. 4) or
// Beer-Lambert, alpha = 1 - T (Eq. 5), and the sigma_min skip / alpha_max
// stop of Sec. 6.2.
//
// Geometry.  The marched point is o + t d.  Every traversal decision is the
// sign of a difference of two plane-crossing parameters
//     t_a(P) - t_b(Q) = (P - o_a)/d_a - (Q - o_b)/d_b,
// decided first from float32 approximations with a rigorous error bound and,
// inside the bound, exactly: the numerator (P - o_a) d_b - (Q - o_b) d_a is
// the sum of four products of float32 values, each an integer below 2^48
// times a power of two, whose sign 64-bit integer arithmetic decides.  The
// length of each leaf segment is computed from the same numerator with
// float32 error-free transformations, so it keeps full relative precision
// even for a leaf the ray only grazes.
//
// The march keeps the integer cell q (at max depth) of the point just after
// the current event (the plane crossing, or the origin, that starts the
// current segment).  Each step descends by the bits of q -- from the
// deepest common ancestor of the previous and the new cell, whose path is
// kept per lane, or, when that ancestor lies above the top grid's level,
// from the grid entry of q -- takes the exit of the node found (ties between
// axes are exact), and re-locates q on the other axes inside the node's
// extent.
//
// Everything here is __host__ __device__ so that the same code can be
// compiled for the host when debugging the traversal.
#pragma once

#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lq_internal.h"

namespace lq {

#define LQ_HD __host__ __device__

constexpr float kFilterRel = 0x1p-22f;   // 4 u: bound on |t' - t| / |t| (3.0000002 u) with margin
constexpr float kFilterAbs = 0x1p-120f;  // covers subnormal products
constexpr uint64_t kFnvOffset = 14695981039346656037ull;
constexpr uint64_t kFnvPrime = 1099511628211ull;

// ------------------------------------------------------------ storage
template <int S> struct Storage;
template <> struct Storage<LQ_F32> {
    static constexpr int bytes = 4;
    LQ_HD static float get(const uint32_t *w, int j) { return __builtin_bit_cast(float, w[j]); }
};
template <> struct Storage<LQ_F16> {
    static constexpr int bytes = 2;
    LQ_HD static float get(const uint32_t *w, int j) {
        uint16_t v = (uint16_t)((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu);
        return (float)__builtin_bit_cast(_Float16, v);
    }
};
template <> struct Storage<LQ_BF16> {
    static constexpr int bytes = 2;
    LQ_HD static float get(const uint32_t *w, int j) {
        uint32_t v = (w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu;
        return __builtin_bit_cast(float, v << 16);
    }
};

LQ_HD constexpr int row_bytes_for(int elem_bytes, int K) {
    int need = (1 + 3 * K) * elem_bytes;
    int rb = 64;
    while (rb < need) rb <<= 1;
    return rb;
}

// ------------------------------------------------------------ SH basis
// Y_lm(x, y, z) = c_lm * poly_lm for the real orthonormal basis without the
// Condon-Shortley phase, k = l^2 + l + m.  With K_l^m = sqrt((2l+1)/(4 pi) *
// (l-|m|)!/(l+|m|)!), Y_lm = s_m K_l^|m| P_l^|m|(z) {cos, sin}(|m| phi),
// s_0 = 1, s_m = sqrt(2); a_lm below is the rational factor between
// P_l^|m|(z) {cos, sin}(|m| phi) and the polynomial written in sh_basis, so
// c_lm = s_m K_l^|m| a_lm.  The table is evaluated at compile time.
constexpr double cx_sqrt(double x) {   // Newton's method, to a fixed point
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; ++i) {
        const double nr = 0.5 * (r + x / r);
        if (nr == r) break;
        r = nr;
    }
    return r;
}
struct ShTable {
    float c[25];
};
constexpr ShTable make_sh_table() {
    const double a[25] = {
        1.0,                                      // l = 0
        1.0, 1.0, 1.0,                            // l = 1: y, z, x
        6.0, 3.0, 0.5, 3.0, 3.0,                  // l = 2: xy, yz, 3z^2-1, xz, x^2-y^2
        15.0, 30.0, 1.5, 0.5, 1.5, 15.0, 15.0,    // l = 3
        420.0, 105.0, 15.0, 2.5, 0.125, 2.5, 7.5, 105.0, 105.0,   // l = 4
    };
    ShTable t{};
    for (int l = 0; l <= 4; ++l)
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            double f = 1.0;
            for (int i = l - am + 1; i <= l + am; ++i) f *= (double)i;   // (l+|m|)!/(l-|m|)!
            const double K = cx_sqrt((2.0 * l + 1.0) / (4.0 * 3.14159265358979323846) / f);
            const double sm = am == 0 ? 1.0 : cx_sqrt(2.0);
            t.c[l * l + l + m] = (float)(sm * K * a[l * l + l + m]);
        }
    return t;
}
constexpr ShTable kSh = make_sh_table();

template <int DEG>
LQ_HD inline void sh_basis(float x, float y, float z, float *Y) {
    constexpr const float *c = kSh.c;
    Y[0] = c[0];
    if constexpr (DEG >= 1) {
        Y[1] = c[1] * y;
        Y[2] = c[2] * z;
        Y[3] = c[3] * x;
    }
    if constexpr (DEG >= 2) {
        float x2 = x * x, y2 = y * y, z2 = z * z;
        Y[4] = c[4] * (x * y);
        Y[5] = c[5] * (y * z);
        Y[6] = c[6] * (3.0f * z2 - 1.0f);
        Y[7] = c[7] * (x * z);
        Y[8] = c[8] * (x2 - y2);
        if constexpr (DEG >= 3) {
            Y[9] = c[9] * (y * (3.0f * x2 - y2));
            Y[10] = c[10] * (x * y * z);
            Y[11] = c[11] * (y * (5.0f * z2 - 1.0f));
            Y[12] = c[12] * (z * (5.0f * z2 - 3.0f));
            Y[13] = c[13] * (x * (5.0f * z2 - 1.0f));
            Y[14] = c[14] * (z * (x2 - y2));
            Y[15] = c[15] * (x * (x2 - 3.0f * y2));
        }
        if constexpr (DEG >= 4) {
            Y[16] = c[16] * (x * y * (x2 - y2));
            Y[17] = c[17] * (y * z * (3.0f * x2 - y2));
            Y[18] = c[18] * (x * y * (7.0f * z2 - 1.0f));
            Y[19] = c[19] * (y * z * (7.0f * z2 - 3.0f));
            Y[20] = c[20] * ((35.0f * z2 - 30.0f) * z2 + 3.0f);
            Y[21] = c[21] * (x * z * (7.0f * z2 - 3.0f));
            Y[22] = c[22] * ((x2 - y2) * (7.0f * z2 - 1.0f));
            Y[23] = c[23] * (x * z * (x2 - 3.0f * y2));
            Y[24] = c[24] * (x2 * (x2 - 3.0f * y2) - y2 * (3.0f * x2 - y2));
        }
    }
}

// ------------------------------------------------- exact arithmetic
LQ_HD inline void two_sum_f(float a, float b, float &s, float &e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One product x*y of two finite float32 values as an exact signed term
// m 2^E: x = (-1)^sx mx 2^ex with an integer mx < 2^24 (normal: hidden bit
// and ex = biased exponent - 150; subnormal: ex = -149), so m = mx my < 2^48
// and E = ex + ey.  neg flips the sign.
struct ExactTerm {
    int64_t m;   // signed, |m| < 2^48 (0 for a zero product)
    int E;
};
LQ_HD inline ExactTerm exact_product(float x, float y, bool neg) {
    const uint32_t bx = __builtin_bit_cast(uint32_t, x), by = __builtin_bit_cast(uint32_t, y);
    const uint32_t exb = (bx >> 23) & 0xffu, eyb = (by >> 23) & 0xffu;
    const uint64_t mx = (bx & 0x7fffffu) | (exb ? 0x800000u : 0u);
    const uint64_t my = (by & 0x7fffffu) | (eyb ? 0x800000u : 0u);
    const int ex = exb ? (int)exb - 150 : -149, ey = eyb ? (int)eyb - 150 : -149;
    const int64_t m = (int64_t)(mx * my);
    const bool negative = (((bx ^ by) >> 31) != 0) != neg;
    return ExactTerm{negative ? -m : m, ex + ey};
}
LQ_HD inline void order_terms(ExactTerm &a, ExactTerm &b) {   // larger exponent first
    if (b.E > a.E) {
        const ExactTerm t = a;
        a = b;
        b = t;
    }
}

// P 2^E += t.m 2^t.E (t.E <= E); done once P's sign is the result's or
// the terms left are zero
LQ_HD inline void absorb_term(int64_t &P, int &E, bool &done, const ExactTerm &t) {
    if (done || t.m == 0) {
        done = true;
        return;
    }
    if (P == 0) {
        P = t.m;
        E = t.E;
        return;
    }
    const int g = E - t.E;                    // >= 0: the terms come in order
    const int64_t aP = P < 0 ? -P : P;
    if (g >= 50 || aP >= ((int64_t)1 << (50 - g))) {
        done = true;
        return;
    }
    P = P * ((int64_t)1 << g) + t.m;
    E = t.E;
}

// sign((Pa - oa) db - (Pb - ob) da) for finite float32 operands, exact, in
// 64-bit integer arithmetic: the expression is the sum of four products
// Pa db - oa db - Pb da + ob da, each an integer below 2^48 times a power of
// two.  The terms are added from the largest exponent down into an integer
// P at the scale of the last term added.  Before a term of exponent E joins,
// the terms still to come (at most three, each below 2^48 at scale 2^E) sum
// to less than 2^50 at that scale; when P, shifted to it, reaches 2^50 its
// sign is the result.  Otherwise the shifted P stays below 2^50 and the sum
// below 2^51, so nothing overflows.
LQ_HD inline int exact_cross_sign(float Pa, float oa, float da, float Pb, float ob, float db) {
    ExactTerm t0 = exact_product(Pa, db, false);
    ExactTerm t1 = exact_product(oa, db, true);
    ExactTerm t2 = exact_product(Pb, da, true);
    ExactTerm t3 = exact_product(ob, da, false);
    // zero terms carry no exponent: put them last
    if (t0.m == 0) t0.E = -1000;
    if (t1.m == 0) t1.E = -1000;
    if (t2.m == 0) t2.E = -1000;
    if (t3.m == 0) t3.E = -1000;
    order_terms(t0, t1);
    order_terms(t2, t3);
    order_terms(t0, t2);
    order_terms(t1, t3);
    order_terms(t1, t2);
    int64_t P = t0.m;
    int E = t0.E;
    bool done = false;
    absorb_term(P, E, done, t1);
    absorb_term(P, E, done, t2);
    absorb_term(P, E, done, t3);
    return P > 0 ? 1 : (P < 0 ? -1 : 0);
}

struct Ray {
    float o[3], d[3], inv[3];
    bool filter_ok;
};

// one plane crossing (ax >= 0) or the ray origin (ax < 0, t = 0)
struct Event {
    int ax;
    float P, t;
};

// v[a] for an axis a in 0..2.  sel3 is the form for the rare exact paths
// (the compiler branches on the axis there); sel3v reads the three values
// first and selects among them, which compiles to two v_cndmask per pick
// instead of a branch tree with exec-mask handling -- the form for the
// segment length, computed for every composited leaf.  (Selecting among
// v[0..2] by an index-like condition such as a > 1, or a & 2, makes the
// compiler index the array instead: a stack copy in scratch memory.)
LQ_HD inline float sel3(const float (&v)[3], int a) { return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]); }
LQ_HD inline float sel3v(const float (&v)[3], int a) {
    const float v0 = v[0], v1 = v[1], v2 = v[2];
    return a == 2 ? v2 : (a == 1 ? v1 : v0);
}

LQ_HD inline float tapprox(const Ray &r, int a, float P) { return (P - sel3(r.o, a)) * sel3(r.inv, a); }

// sign((Pa - oa)/da - (Pb - ob)/db), exact, for da, db != 0: the sign of
// (Pa - oa) db - (Pb - ob) da times that of da db
static LQ_HD __noinline__ int cross_cmp_exact(float Pa, float oa, float da, float Pb, float ob, float db) {
    const int s = exact_cross_sign(Pa, oa, da, Pb, ob, db);
    return ((da > 0.0f) == (db > 0.0f)) ? s : -s;
}

// sign(t_a(Pa) - t_b(Pb)); ta/tb are tapprox() of the same planes
LQ_HD inline int cross_cmp(const Ray &r, int a, float Pa, float ta, int b, float Pb, float tb) {
    if (a == b) {
        if (Pa == Pb) return 0;
        return ((Pa > Pb) == (sel3(r.d, a) > 0.0f)) ? 1 : -1;
    }
    if (r.filter_ok) {
        float df = ta - tb;
        float bound = fmaf(kFilterRel, fabsf(ta) + fabsf(tb), kFilterAbs);
        if (__builtin_expect(fabsf(df) > bound, 1)) return df > 0.0f ? 1 : -1;
    }
    return cross_cmp_exact(Pa, sel3(r.o, a), sel3(r.d, a), Pb, sel3(r.o, b), sel3(r.d, b));
}

// sign(t_b(P) - t_event)
LQ_HD inline int cmp_event(const Ray &r, int b, float P, const Event &e) {
    if (e.ax < 0) {   // t_event = 0: the sign of t_b(P) itself
        float ob = sel3(r.o, b);
        if (P == ob) return 0;
        return ((P > ob) == (sel3(r.d, b) > 0.0f)) ? 1 : -1;
    }
    return cross_cmp(r, b, P, tapprox(r, b, P), e.ax, e.P, e.t);
}

LQ_HD inline float plane_of(int k, float h) { return fmaf((float)k, h, -1.0f); }

// true when the filter certifies t_a(P) > t_b(Q) from the approximations
// ta, tb (the same bound as cross_cmp); false means later or undecided
LQ_HD inline bool later(float ta, float tb) {
    return ta - tb > fmaf(kFilterRel, fabsf(ta) + fabsf(tb), kFilterAbs);
}

LQ_HD inline int lo_sel(const int (&lo)[3], int a) { return a == 0 ? lo[0] : (a == 1 ? lo[1] : lo[2]); }

// Cell index along axis b (d_b != 0) of the point just after event e, known
// to lie in [lo, hi).
LQ_HD inline int locate(const Ray &r, int b, int lo, int hi, const Event &e, float h, int N) {
    float db = sel3(r.d, b);
    float p = fmaf(e.t, db, sel3(r.o, b));
    float g = (p + 1.0f) * (0.5f * (float)N);
    g = fminf(fmaxf(g, (float)lo), (float)(hi - 1));
    int k = (int)g;
    for (int it = 0; it <= hi - lo + 1; ++it) {
        if (db > 0.0f) {
            if (k > lo && cmp_event(r, b, plane_of(k, h), e) > 0) { --k; continue; }
            if (k + 1 < hi && cmp_event(r, b, plane_of(k + 1, h), e) <= 0) { ++k; continue; }
        } else {
            if (k + 1 < hi && cmp_event(r, b, plane_of(k + 1, h), e) > 0) { ++k; continue; }
            if (k > lo && cmp_event(r, b, plane_of(k, h), e) <= 0) { --k; continue; }
        }
        break;
    }
    return k;
}

// t(x) - t(e) for the exit crossing x, with full relative precision
LQ_HD inline float seg_dt(const Ray &r, const Event &e, int xa, float xP, float xt) {
    if (e.ax < 0) return xt;
    if (e.ax == xa) return (xP - e.P) * sel3v(r.inv, xa);
    float dx = sel3v(r.d, xa), de = sel3v(r.d, e.ax);
    float X1, X0, V1, V0;
    two_sum_f(xP, -sel3v(r.o, xa), X1, X0);
    two_sum_f(e.P, -sel3v(r.o, e.ax), V1, V0);
    float p1 = X1 * de, p0 = fmaf(X1, de, -p1);
    float q1 = V1 * dx, q0 = fmaf(V1, dx, -q1);
    float num = (p1 - q1) + ((p0 - q0) + (X0 * de - V0 * dx));
    return num * (sel3v(r.inv, xa) * sel3v(r.inv, e.ax));
}

// child octant of cell q at bit sh: bit sh of x, y, z in bits 0, 1, 2
LQ_HD inline int octant_at(const int (&q)[3], int sh) {
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t b0 = __builtin_amdgcn_ubfe((uint32_t)q[0], (uint32_t)sh, 1u);
    const uint32_t b1 = __builtin_amdgcn_ubfe((uint32_t)q[1], (uint32_t)sh, 1u);
    const uint32_t b2 = __builtin_amdgcn_ubfe((uint32_t)q[2], (uint32_t)sh, 1u);
    return (int)(b0 | (b1 << 1) | (b2 << 2));
#else
    return ((q[0] >> sh) & 1) | (((q[1] >> sh) & 1) << 1) | (((q[2] >> sh) & 1) << 2);
#endif
}

LQ_HD inline uint32_t spread3(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// float32 helpers for the emission activation: hardware exp2 and reciprocal
// on the device (relative error ~1e-6 over the logit range of the tables),
// libm on the host build
LQ_HD inline float lq_exp_neg(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_exp2f(x * -1.4426950408889634f);
#else
    return expf(-x);
#endif
}
LQ_HD inline float lq_rcp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

struct RayOut {
    float rgb[3], alpha;
    uint32_t count, n_comp, n_steps;
    int32_t term_idx;
    uint64_t hash;
};

// The query for one ray as a resumable state machine: init() clips the ray
// and locates its first cell, step() visits one octree node (leaf or empty),
// result() reads the outputs.  ids (may be null) receives up to max_ids
// Morton ids of the data leaves in order; path[l * path_stride] (l < depth)
// holds the node indices along the current root-to-node path, so that each
// step re-descends only from the deepest common ancestor of the previous and
// the new cell.  With SKIP the march uses the child table without the
// leaves below sigma_min (DevTree::child_skip): every leaf it meets is
// composited, so its whole row is fetched at once.
// MODEL: LQ_LINEAR or LQ_EXP fixed at compile time, or -1 to take the model
// passed to step().
template <int ST, int DEG, bool ACC64, bool TRACE, bool SKIP = false, int MODEL = -1>
struct Marcher {
    using S = Storage<ST>;
    using Acc = typename std::conditional<ACC64, double, float>::type;
    static constexpr int K = (DEG + 1) * (DEG + 1);
    static constexpr int RB = row_bytes_for(S::bytes, K);
    static constexpr int NE = 1 + 3 * K;
    static constexpr int NCH = (NE * S::bytes + 15) / 16;   // 16-byte chunks holding the row

    Ray r;
    float dlen;
    float Y[K];
    Event ev;
    int q[3];
    uint32_t qdiff;       // OR of the bitwise differences between the current and the previous cell
    int path_top, steps_left;
    Acc L0, L1, L2, T;
    uint32_t count, ncomp, nsteps;
    int32_t term;
    uint64_t hash;

    // returns true when the ray has nodes to visit
    LQ_HD bool init(const DevTree &t, const float *o3, const float *d3) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
#ifdef __HIP_DEVICE_COMPILE__
            // read once: non-temporal, so the rays do not displace tree lines in L2
            r.o[ax] = __builtin_nontemporal_load(o3 + ax);
            r.d[ax] = __builtin_nontemporal_load(d3 + ax);
#else
            r.o[ax] = o3[ax];
            r.d[ax] = d3[ax];
#endif
        }
        L0 = L1 = L2 = 0;
        T = 1;
        count = ncomp = nsteps = 0;
        term = -1;
        hash = kFnvOffset;
        path_top = -1;
        q[0] = q[1] = q[2] = 0;
        qdiff = 0;
        ev = Event{-1, 0.0f, 0.0f};

        const int D = t.depth;
        const int N = 1 << D;
        const float h = 2.0f / (float)N;
        steps_left = 3 * N + 8;

        bool ok = true;
        bool anyd = false;
        r.filter_ok = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            ok = ok && isfinite(r.o[ax]) && isfinite(r.d[ax]);
            anyd = anyd || r.d[ax] != 0.0f;
            float ad = fabsf(r.d[ax]);
            r.filter_ok = r.filter_ok && fabsf(r.o[ax]) <= 0x1p60f &&
                          (ad == 0.0f || (ad >= 0x1p-60f && ad <= 0x1p60f));
            r.inv[ax] = r.d[ax] != 0.0f ? 1.0f / r.d[ax] : 0.0f;
        }
        dlen = sqrtf(r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2]);
        ok = ok && anyd && dlen > 0.0f && isfinite(dlen);
        if (__builtin_expect(!ok, 0)) return false;

        // ---- clip to the proxy box [-1, 1)^3
        int in_ax = -1;
        float in_P = 0.0f, in_t = 0.0f;
        bool origin_start = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            float dx = r.d[ax], ox = r.o[ax];
            if (dx == 0.0f) {
                ok = ok && (ox >= -1.0f && ox < 1.0f);
                continue;
            }
            float Pn = dx > 0.0f ? -1.0f : 1.0f;
            // the far plane must lie after t = 0 (else the box is behind)
            ok = ok && (dx > 0.0f ? ox < 1.0f : ox > -1.0f);
            origin_start = origin_start && (dx > 0.0f ? ox >= -1.0f : ox <= 1.0f);
            float tn = tapprox(r, ax, Pn);
            if (in_ax < 0 || cross_cmp(r, ax, Pn, tn, in_ax, in_P, in_t) > 0) {
                in_ax = ax;
                in_P = Pn;
                in_t = tn;
            }
        }
        if (ok && !origin_start) {
            ev = Event{in_ax, in_P, in_t};
            // the far plane of every axis must come strictly after the entry
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if (r.d[ax] == 0.0f || ax == in_ax) continue;
                float Pf = r.d[ax] > 0.0f ? 1.0f : -1.0f;
                ok = ok && cmp_event(r, ax, Pf, ev) > 0;
            }
        }
        if (__builtin_expect(!ok, 0)) return false;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            float dx = r.d[ax], ox = r.o[ax];
            if (dx == 0.0f || ev.ax < 0) {
                // cell of the origin coordinate (half-open cells; moving
                // down off a plane puts the point in the lower cell)
                float g = fminf(fmaxf((ox + 1.0f) * (0.5f * (float)N), 0.0f), (float)(N - 1));
                int k = (int)g;
                while (k > 0 && plane_of(k, h) > ox) --k;
                while (k + 1 < N && plane_of(k + 1, h) <= ox) ++k;
                if (dx < 0.0f && plane_of(k, h) == ox && k > 0) --k;
                q[ax] = k;
            } else if (ax == ev.ax) {
                q[ax] = dx > 0.0f ? 0 : N - 1;
            } else {
                // the cell coordinate of the entry point, certified like the
                // re-location in step(); else the exact search
                const float pp = fmaf(ev.t, dx, ox);
                const float half_n = 0.5f * (float)N;
                const float g = (pp + 1.0f) * half_n;
                const float eg = (fabsf(ev.t * dx) + fabsf(pp) + 1.0f) * (half_n * 0x1p-21f);
                const float fl = floorf(g);
                const float fr = g - fl;
                const int k = (int)fl;
                q[ax] = r.filter_ok && fr > eg && fr < 1.0f - eg && k >= 0 && k < N ? k
                                                                                  : locate(r, ax, 0, N, ev, h, N);
            }
        }

        // ---- emission direction omega = -d/|d| and its SH values
        float inv_len = 1.0f / dlen;
        sh_basis<DEG>(-r.d[0] * inv_len, -r.d[1] * inv_len, -r.d[2] * inv_len, Y);
        return true;
    }

    // Visit one node; returns true when the march is over.
    // top: the dense top grid of the table marched (DevTree::top or
    // top_skip, possibly a copy in LDS), or null.  path[l] is kept only for
    // the levels the grid does not cover.
    LQ_HD bool step(const DevTree &t, int model, uint32_t flags, uint32_t *ids, int32_t max_ids,
                    int32_t *path, int path_stride, const int32_t *top = nullptr) {
        const int D = t.depth;
        const int N = 1 << D;
        const float h = 2.0f / (float)N;
        const int32_t *child = SKIP ? t.child_skip : t.child;
        if (__builtin_expect(--steps_left < 0, 0)) return true;

        int node = 0, level = 0, c = 0;
        if (path_top >= 0) {
            // the old and new cells share the path down to the level above
            // their highest differing coordinate bit
            int hb = 31 - __builtin_clz(qdiff | 1u);
            level = D - 1 - hb;
            if (level > path_top) level = path_top;
            if (level < 0) level = 0;
        }
        bool descend = true;
        if (top && level < kTopLevel) {
            const int gs = D - kTopLevel;
            const int e = top[((q[2] >> gs) << (2 * kTopLevel)) | ((q[1] >> gs) << kTopLevel) | (q[0] >> gs)];
            if (e > 0) {
                node = e;
                level = kTopLevel;
            } else {   // empty node whose cell is at level -e
                level = -e;
                descend = false;
            }
        } else if (path_top >= 0) {
            node = path[level * path_stride];
        }
        while (descend) {
            path[level * path_stride] = node;
            int sh = D - 1 - level;
            const int oct = octant_at(q, sh);
            c = child[(uint32_t)node * 8u + (uint32_t)oct];   // n_nodes < 2^29 (checked at load)
            ++level;
            if (c <= 0 || level >= D) break;
            node = c;
        }
        if (c > 0) c = 0;   // malformed table guard: never descend below max depth
        path_top = level - 1;
        ++nsteps;
        const int sshift = D - level;
        const int Sz = 1 << sshift;
        int lo[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) lo[ax] = (q[ax] >> sshift) << sshift;

        // Exit crossing of the node and the neighbouring cell.  Fast path:
        // the float32 plane parameters, every decision certified -- the exit
        // axis by the error filter on its margin over the other axes, each
        // re-located coordinate by the distance of its float32 cell
        // coordinate from the nearest cell boundary.  When a margin is too
        // thin (ties, grazing), the exact path below decides everything
        // again.
        int xa = 0;
        float xP = 0.0f, xt = 0.0f;
        unsigned xmask = 0;
        int nq[3] = {q[0], q[1], q[2]};
        bool leave = false;
        bool fast = r.filter_ok;
        {
            float tc[3], Pc[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                Pc[ax] = plane_of(r.d[ax] > 0.0f ? lo[ax] + Sz : lo[ax], h);
                tc[ax] = r.d[ax] != 0.0f ? (Pc[ax] - r.o[ax]) * r.inv[ax] : INFINITY;
            }
            xa = tc[1] < tc[0] ? 1 : 0;
            xa = tc[2] < (xa ? tc[1] : tc[0]) ? 2 : xa;
            xP = xa == 0 ? Pc[0] : (xa == 1 ? Pc[1] : Pc[2]);
            xt = xa == 0 ? tc[0] : (xa == 1 ? tc[1] : tc[2]);
            xmask = 1u << xa;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                if (ax != xa && r.d[ax] != 0.0f) fast = fast && later(tc[ax], xt);
            // the next cell along the exit axis, as selects (written as
            // nested conditionals the compiler branches on the axis)
            const float dxa = xa == 2 ? r.d[2] : (xa == 1 ? r.d[1] : r.d[0]);
            const int loa = xa == 2 ? lo[2] : (xa == 1 ? lo[1] : lo[0]);
            const int nx = loa + (dxa > 0.0f ? Sz : -1);
            leave = nx < 0 || nx >= N;
            nq[0] = xa == 0 ? nx : nq[0];
            nq[1] = xa == 1 ? nx : nq[1];
            nq[2] = xa == 2 ? nx : nq[2];
            if (!leave && Sz > 1) {
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const float db = r.d[ax];
                    if (ax == xa || db == 0.0f) continue;
                    // cell coordinate of the exit point in units of cells: g
                    // and its error bound eg (xt is within 3.0000002u|t| of
                    // the exact exit parameter; the fma and the add round
                    // once each; 8u covers it all with margin).  A g at least
                    // eg away from an integer certifies its cell.
                    const float pp = fmaf(xt, db, r.o[ax]);
                    const float half_n = 0.5f * (float)N;
                    const float g = (pp + 1.0f) * half_n;
                    const float eg = (fabsf(xt * db) + fabsf(pp) + 1.0f) * (half_n * 0x1p-21f);
                    const float fl = floorf(g);
                    const float fr = g - fl;
                    const int k = (int)fl;
                    fast = fast && fr > eg && fr < 1.0f - eg && k >= lo[ax] && k < lo[ax] + Sz;
                    nq[ax] = k;
                }
            }
        }
        if (__builtin_expect(!fast, 0)) {
            xa = -1;
            xmask = 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                float dx = r.d[ax];
                if (dx == 0.0f) continue;
                int k = dx > 0.0f ? lo[ax] + Sz : lo[ax];
                float P = plane_of(k, h);
                float tt = tapprox(r, ax, P);
                int cmpv = xa < 0 ? -1 : cross_cmp(r, ax, P, tt, xa, xP, xt);
                if (cmpv < 0) {
                    xa = ax; xP = P; xt = tt;
                    xmask = 1u << ax;
                } else if (cmpv == 0) {
                    xmask |= 1u << ax;
                }
            }
            leave = false;
            nq[0] = q[0]; nq[1] = q[1]; nq[2] = q[2];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if (!(xmask & (1u << ax))) continue;
                nq[ax] = r.d[ax] > 0.0f ? lo[ax] + Sz : lo[ax] - 1;
                leave = leave || nq[ax] < 0 || nq[ax] >= N;
            }
            if (!leave && Sz > 1) {
                const Event e{xa, xP, xt};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    if ((xmask & (1u << ax)) || r.d[ax] == 0.0f) continue;
                    nq[ax] = locate(r, ax, lo[ax], lo[ax] + Sz, e, h, N);
                }
            }
        }
        const Event nev{xa, xP, xt};
        // the leaf row (fetched after the exit computation: holding it
        // across that code costs more in registers than its latency)
        const bool is_leaf = c < 0;
        const int leaf = is_leaf ? -c - 1 : 0;
        const uint4 *rowp = reinterpret_cast<const uint4 *>(static_cast<const char *>(t.rows) + (size_t)leaf * RB);
        uint32_t w[NCH * 4];
        if (is_leaf) {
            const uint4 c0 = rowp[0];
            w[0] = c0.x; w[1] = c0.y; w[2] = c0.z; w[3] = c0.w;
            if (SKIP) {
#pragma unroll
                for (int ch = 1; ch < NCH; ++ch) {
                    const uint4 cc = rowp[ch];
                    w[4 * ch] = cc.x; w[4 * ch + 1] = cc.y; w[4 * ch + 2] = cc.z; w[4 * ch + 3] = cc.w;
                }
            }
        }


        if (is_leaf) {
            if (TRACE) {
                uint32_t id = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
                if ((int32_t)count < max_ids) ids[count] = id;
                hash = (hash ^ (uint64_t)id) * kFnvPrime;
            }
            ++count;
            const float sig = S::get(w, 0);
            if (SKIP || (flags & LQ_NO_SIGMA_SKIP) || sig >= t.sigma_min) {
#pragma unroll
                for (int ch = 1; ch < NCH && !SKIP; ++ch) {
                    uint4 cc = rowp[ch];
                    w[4 * ch] = cc.x; w[4 * ch + 1] = cc.y; w[4 * ch + 2] = cc.z; w[4 * ch + 3] = cc.w;
                }
                float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    x0 = fmaf(S::get(w, 1 + k), Y[k], x0);
                    x1 = fmaf(S::get(w, 1 + K + k), Y[k], x1);
                    x2 = fmaf(S::get(w, 1 + 2 * K + k), Y[k], x2);
                }
                const float phi0 = t.l_max * lq_rcp(1.0f + lq_exp_neg(x0));
                const float phi1 = t.l_max * lq_rcp(1.0f + lq_exp_neg(x1));
                const float phi2 = t.l_max * lq_rcp(1.0f + lq_exp_neg(x2));
                const float dt = fmaxf(seg_dt(r, ev, xa, xP, xt), 0.0f);
                const Acc delta = (Acc)dt * (Acc)dlen;
                const Acc sd = (Acc)sig * delta;
                Acc wgt;
                if ((MODEL >= 0 ? MODEL : model) == LQ_EXP) wgt = -T * expm1(sd * Acc(-1));
                else wgt = sd < T ? sd : T;
                L0 += wgt * (Acc)phi0;
                L1 += wgt * (Acc)phi1;
                L2 += wgt * (Acc)phi2;
                T -= wgt;
                ++ncomp;
                if (!(flags & LQ_NO_EARLY_TERM) && (Acc(1) - T) >= (Acc)t.alpha_max) {
                    term = (int32_t)count - 1;
                    return true;
                }
            }
        }
        if (__builtin_expect(leave, 0)) return true;
        qdiff = (uint32_t)((q[0] ^ nq[0]) | (q[1] ^ nq[1]) | (q[2] ^ nq[2]));
        q[0] = nq[0]; q[1] = nq[1]; q[2] = nq[2];
        ev = nev;
        return false;
    }

    LQ_HD void result(RayOut &out) const {
        out.rgb[0] = (float)L0;
        out.rgb[1] = (float)L1;
        out.rgb[2] = (float)L2;
        out.alpha = (float)(Acc(1) - T);
        out.count = count;
        out.n_comp = ncomp;
        out.n_steps = nsteps;
        out.term_idx = term;
        out.hash = hash;
    }
};

// The whole query for one ray (init, steps until done, result).
template <int ST, int DEG, bool ACC64, bool TRACE, bool SKIP = false>
LQ_HD inline void march_ray(const DevTree &t, const float *o3, const float *d3, int model,
                            uint32_t flags, RayOut &out, uint32_t *ids, int32_t max_ids,
                            int32_t *path, int path_stride, const int32_t *top = nullptr) {
    Marcher<ST, DEG, ACC64, TRACE, SKIP> m;
    if (m.init(t, o3, d3))
        while (!m.step(t, model, flags, ids, max_ids, path, path_stride, top)) {
        }
    m.result(out);
}

}  // namespace lq
