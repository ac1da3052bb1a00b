/*
 * lq_oracle.c -- plain FP64 CPU oracle for the luminaire emission query.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library (no headers, helpers or tables), and is written to be read
 * against the paper:
 *
 *   Ray:          r(t) = x - omega t (Sec. 4.1, Eq. 3).  A caller passes the
 *                 shading point o and the direction d pointing into the
 *                 luminaire, so omega = -d/|d| and the marched point is o + t d.
 *   Proxy:        the box [-1, 1]^3, which is also the octree's root cube
 *                 (Sec. 5: the emitter plugin is attached to a sphere or box
 *                 proxy).  t_1 (Eq. 3) is the far box hit.
 *   Emission:     Phi_c = L_max * sigmoid(sum_{l,m} c_{c,lm} Y_lm(omega))
 *                 (Sec. 4.2, Eq. 6: the "extended-range sigmoid").
 *   Transmittance linear model T = max(0, 1 - int sigma) (Sec. 4.1, Eq. 4), or
 *                 Beer-Lambert (the exponential model compared in Sec. 6.2,
 *                 Table 4).
 *   Integral:     Eq. 3 over a leaf of constant sigma and Phi.  Reading taken:
 *                 the weight of a leaf is w = T_in - T_out (the derivative
 *                 weight -dT, exact for both models), so the weights sum to
 *                 alpha = 1 - T(t_1) (Sec. 4.1, Eq. 5).
 *   Heuristics:   leaves with stored sigma < sigma_min are skipped; the march
 *                 stops once 1 - T >= alpha_max, tested after each composited
 *                 leaf (Sec. 6.2, "Performance vs Quality": 0.1 and 0.9).
 *
 * Leaf sequence: the octree leaves whose half-open cell [lo, hi)^3 meets the
 * open segment (t_start, t_out) in positive length, in order of t.  The march
 * locates the point just after the current t (descending from the root,
 * choosing each child by comparing the point with the node's mid-planes) and
 * moves to the exit of the node it found.  Every decision compares two
 * FP64-evaluated crossing parameters; when they are within a relative 1e-12
 * the ray is flagged (ORC_NEED_EXACT) and the caller re-runs it in exact
 * rational arithmetic.
 *
 * Spherical harmonics: real, orthonormal, no Condon-Shortley phase, index
 * k = l^2 + l + m, built from the associated Legendre recurrence.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NEED_EXACT 1u   /* a decision fell inside the FP64 filter    */
#define ORC_AMBIGUOUS  2u   /* an alpha_max test was within eta of 0.9f  */
#define ORC_MISS       4u   /* no positive-length overlap with the proxy */
#define ORC_BADRAY     8u   /* non-finite input or zero direction        */

#define ORC_NO_STOP 1u      /* disable the alpha_max stop   */
#define ORC_NO_SKIP 4u      /* disable the sigma_min skip   */

typedef struct {
    int32_t depth, sh_degree, n_nodes, n_leaves;
    double l_max, sigma_min, alpha_max, eta;
    const int32_t *child;   /* [n_nodes][8] */
    const double *sigma;    /* [n_leaves], stored values promoted */
    const double *sh;       /* [n_leaves][3][K], stored values promoted */
} orc_tree;

typedef struct {
    double L[3], alpha;
    int32_t count, term_idx, n_comp, n_nodes_visited;
    uint64_t hash;
    uint32_t flags;
    int32_t first_amb_test;   /* index of the first ambiguous stop test, or -1 */
} orc_result;

static const double REL_FILTER = 1e-12;

/* ------------------------------------------------------------------ SH */
static double factorial(int n) { double r = 1.0; for (int i = 2; i <= n; ++i) r *= i; return r; }

/* P_l^m(x) without the Condon-Shortley phase, 0 <= m <= l */
static double assoc_legendre(int l, int m, double x) {
    double pmm = 1.0;
    double s = sqrt((1.0 - x) * (1.0 + x));
    for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pll;
    }
    return pll;
}

static double sh_norm(int l, int m) {
    return sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
}

/* Real SH values at the unit direction w, k = l^2 + l + m, for l <= deg */
void orc_sh_eval(int deg, const double w[3], double *Y) {
    double z = w[2];
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    double phi = atan2(w[1], w[0]);
    for (int l = 0; l <= deg; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double base = sh_norm(l, am) * assoc_legendre(l, am, z);
            double v;
            if (m == 0) v = base;
            else if (m > 0) v = sqrt(2.0) * base * cos(m * phi);
            else v = sqrt(2.0) * base * sin(am * phi);
            Y[l * l + l + m] = v;
        }
    }
}

/* ---------------------------------------------------------- geometry */
typedef struct {
    double o[3], d[3];
    double dlen;
    int D, N;
    double h;
    uint32_t *flags;
} ray_t;

static double plane_pos(const ray_t *r, int k) { return -1.0 + k * r->h; }

/* crossing parameter of the plane x_a = P */
static double tcross(const ray_t *r, int a, double P) { return (P - r->o[a]) / r->d[a]; }

static int near_tie(double x, double y) {
    return fabs(x - y) <= REL_FILTER * (fabs(x) + fabs(y)) + 1e-300;
}

/* The current parameter t is an event: the crossing of plane index ev_k on
 * axis ev_a, or the ray origin (ev_a = -1, t = 0). */
typedef struct { double t; int ev_a, ev_k; } event_t;

/* Is the point o + t d, just after the event, at or above plane index k of
 * axis a?  Against the event's own axis, or at the origin, the answer is
 * exact without any crossing parameter. */
static int above_after(const ray_t *r, const event_t *e, int a, int k) {
    double P = plane_pos(r, k);
    if (r->d[a] == 0.0) return r->o[a] >= P;
    if (e->ev_a == a) return r->d[a] > 0.0 ? e->ev_k >= k : e->ev_k > k;
    if (e->ev_a < 0) return r->o[a] > P || (r->o[a] == P && r->d[a] > 0.0);
    double tp = tcross(r, a, P);
    if (near_tie(e->t, tp)) *r->flags |= ORC_NEED_EXACT;
    if (r->d[a] > 0.0) return e->t >= tp;   /* already crossed (or crossing now) */
    return e->t < tp;                       /* not yet crossed downward */
}

static uint64_t fnv_step(uint64_t h, uint32_t id) { return (h ^ (uint64_t)id) * 1099511628211ull; }

static uint32_t morton(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t m = 0;
    for (int b = 0; b < 10; ++b) {
        m |= ((x >> b) & 1u) << (3 * b);
        m |= ((y >> b) & 1u) << (3 * b + 1);
        m |= ((z >> b) & 1u) << (3 * b + 2);
    }
    return m;
}

/* ------------------------------------------------------------ march */
/* force_stop values besides a test index */
#define ORC_FORCE_NONE (-1)          /* every stop test decided in FP64          */
#define ORC_FORCE_CONTINUE 0x7fffffff /* continue at every ambiguous test       */

/*
 * One ray.  flip_test >= 0 inverts the outcome of that (0-based) alpha_max
 * test: the second candidate for rays whose test is within eta of the
 * threshold.  force_stop (when not ORC_FORCE_NONE) takes another valid
 * outcome of a threshold-ambiguous ray: continue at every ambiguous test
 * before test force_stop and stop at that test (ORC_FORCE_CONTINUE: continue
 * at every ambiguous test); tests that are not ambiguous keep their FP64
 * decision.  *forced_ok (if given) is cleared when that outcome is not a
 * valid one: the march ended or stopped (at a test that is not ambiguous)
 * before test force_stop, or 1 - T at that test is below alpha_max - eta.
 * leaf_out/max_ids optionally receive the Morton ids in order.
 */
static void march_forced(const orc_tree *T, const float *of, const float *df, int model, uint32_t opts,
                         int flip_test, int force_stop, int *forced_ok, int *amb_list, int amb_cap,
                         int *n_amb, orc_result *res, uint32_t *leaf_out, int max_ids);

static void march(const orc_tree *T, const float *of, const float *df, int model, uint32_t opts,
                  int flip_test, orc_result *res, uint32_t *leaf_out, int max_ids) {
    march_forced(T, of, df, model, opts, flip_test, ORC_FORCE_NONE, NULL, NULL, 0, NULL, res, leaf_out, max_ids);
}

static void march_forced(const orc_tree *T, const float *of, const float *df, int model, uint32_t opts,
                         int flip_test, int force_stop, int *forced_ok, int *amb_list, int amb_cap,
                         int *n_amb, orc_result *res, uint32_t *leaf_out, int max_ids) {
    if (forced_ok) *forced_ok = 1;
    if (n_amb) *n_amb = 0;
    memset(res, 0, sizeof(*res));
    res->term_idx = -1;
    res->first_amb_test = -1;
    res->hash = 14695981039346656037ull;
    ray_t r;
    r.flags = &res->flags;
    r.D = T->depth;
    r.N = 1 << T->depth;
    r.h = 2.0 / r.N;
    for (int a = 0; a < 3; ++a) { r.o[a] = of[a]; r.d[a] = df[a]; }
    for (int a = 0; a < 3; ++a)
        if (!isfinite(r.o[a]) || !isfinite(r.d[a])) { res->flags |= ORC_BADRAY; return; }
    r.dlen = sqrt(r.d[0] * r.d[0] + r.d[1] * r.d[1] + r.d[2] * r.d[2]);
    if (!(r.dlen > 0.0)) { res->flags |= ORC_BADRAY; return; }

    /* slab clip against the box [-1,1)^3 (half-open on axes with d = 0) */
    double t_in = -INFINITY, t_out = INFINITY;
    int in_a = -1;
    for (int a = 0; a < 3; ++a) {
        if (r.d[a] == 0.0) {
            if (!(r.o[a] >= -1.0 && r.o[a] < 1.0)) { res->flags |= ORC_MISS; return; }
            continue;
        }
        double t0 = tcross(&r, a, -1.0), t1 = tcross(&r, a, 1.0);
        double tn = t0 < t1 ? t0 : t1, tf = t0 < t1 ? t1 : t0;
        if (in_a >= 0 && near_tie(tn, t_in)) res->flags |= ORC_NEED_EXACT;
        if (tn > t_in) { t_in = tn; in_a = a; }
        if (tf < t_out) t_out = tf;
    }
    event_t ev;
    if (t_in > 0.0) {
        ev.t = t_in; ev.ev_a = in_a; ev.ev_k = r.d[in_a] > 0.0 ? 0 : r.N;
    } else {
        ev.t = 0.0; ev.ev_a = -1; ev.ev_k = 0;
    }
    double t = ev.t;
    if (t_in > 0.0 && near_tie(t, t_out)) res->flags |= ORC_NEED_EXACT;
    if (!(t_out > t)) { res->flags |= ORC_MISS; return; }

    /* emission direction and its SH values */
    int K = (T->sh_degree + 1) * (T->sh_degree + 1);
    double w[3] = {-r.d[0] / r.dlen, -r.d[1] / r.dlen, -r.d[2] / r.dlen};
    double Y[25];
    orc_sh_eval(T->sh_degree, w, Y);

    double Tr = 1.0;
    double L[3] = {0.0, 0.0, 0.0};
    int tests = 0;
    int guard = 0;
    while (t < t_out) {
        if (++guard > 8 * r.N + 64) { res->flags |= ORC_NEED_EXACT; break; }
        /* locate the node containing the point just after t */
        int node = 0, level = 0;
        int lo[3] = {0, 0, 0};
        int c = 0;
        for (;;) {
            int half = r.N >> (level + 1);
            int oct = 0;
            for (int a = 0; a < 3; ++a) {
                int up = above_after(&r, &ev, a, lo[a] + half);
                if (up) { oct |= 1 << a; lo[a] += half; }
            }
            c = T->child[(size_t)node * 8 + oct];
            ++level;
            if (c > 0) { node = c; continue; }
            break;
        }
        res->n_nodes_visited++;
        int size = r.N >> level;
        /* exit of this node's cube */
        double t_next = INFINITY;
        int nx_a = -1, nx_k = 0;
        for (int a = 0; a < 3; ++a) {
            if (r.d[a] == 0.0) continue;
            int k = r.d[a] > 0.0 ? lo[a] + size : lo[a];
            double ta = tcross(&r, a, plane_pos(&r, k));
            /* an interior plane crossed (almost) where the ray leaves the box */
            if (k != 0 && k != r.N && near_tie(ta, t_out)) res->flags |= ORC_NEED_EXACT;
            if (ta < t_next) { t_next = ta; nx_a = a; nx_k = k; }
        }
        if (t_next > t_out) t_next = t_out;
        if (!(t_next > t)) { res->flags |= ORC_NEED_EXACT; break; }
        if (c < 0) {
            int leaf = -c - 1;
            uint32_t id = morton((uint32_t)lo[0], (uint32_t)lo[1], (uint32_t)lo[2]);
            if (leaf_out && res->count < max_ids) leaf_out[res->count] = id;
            res->hash = fnv_step(res->hash, id);
            res->count++;
            double sig = T->sigma[leaf];
            if ((opts & ORC_NO_SKIP) || sig >= T->sigma_min) {
                double delta = (t_next - t) * r.dlen;
                double wgt;
                if (model == 0) {             /* linear: T' = max(0, T - sigma delta) */
                    double tau = sig * delta;
                    wgt = tau < Tr ? tau : Tr;
                } else {                      /* exponential: T' = T exp(-sigma delta) */
                    wgt = -Tr * expm1(-sig * delta);
                }
                const double *row = T->sh + (size_t)leaf * 3 * K;
                for (int ch = 0; ch < 3; ++ch) {
                    double x = 0.0;
                    for (int k = 0; k < K; ++k) x += row[ch * K + k] * Y[k];
                    double phi = T->l_max / (1.0 + exp(-x));
                    L[ch] += wgt * phi;
                }
                Tr -= wgt;
                res->n_comp++;
                if (!(opts & ORC_NO_STOP)) {
                    double alpha = 1.0 - Tr;
                    int stop = alpha >= T->alpha_max;
                    int amb = fabs(alpha - T->alpha_max) <= T->eta;
                    if (amb) {
                        res->flags |= ORC_AMBIGUOUS;
                        if (res->first_amb_test < 0) res->first_amb_test = tests;
                        if (n_amb) {
                            if (*n_amb < amb_cap) amb_list[*n_amb] = tests;
                            ++*n_amb;
                        }
                    }
                    if (tests == flip_test) stop = !stop;
                    if (force_stop != ORC_FORCE_NONE) {
                        if (tests == force_stop) {
                            if (!(stop || amb) && forced_ok) *forced_ok = 0;
                            stop = 1;
                        } else if (amb) {
                            stop = 0;
                        } else if (stop && tests < force_stop && force_stop != ORC_FORCE_CONTINUE && forced_ok) {
                            *forced_ok = 0;   /* a clear stop before the forced test */
                        }
                    }
                    ++tests;
                    if (stop) { res->term_idx = res->count - 1; break; }
                }
            }
        }
        t = t_next;
        ev.t = t_next; ev.ev_a = nx_a; ev.ev_k = nx_k;
    }
    /* the march ended before the forced stop test */
    if (force_stop != ORC_FORCE_NONE && force_stop != ORC_FORCE_CONTINUE && res->term_idx < 0 && forced_ok)
        *forced_ok = 0;
    res->L[0] = L[0]; res->L[1] = L[1]; res->L[2] = L[2];
    res->alpha = 1.0 - Tr;
}

/*
 * Batch entry point.  Outputs (any may be NULL):
 *   L[n][3], alpha[n], count[n], hash[n], term_idx[n], n_comp[n], n_nodes[n], flags[n],
 *   alt_* : the second candidate (first ambiguous stop test flipped), filled
 *           only where flags has ORC_AMBIGUOUS; alt_valid[n] marks them.
 *   leaf_ids[n][max_ids] Morton ids of the first max_ids data leaves.
 */
int orc_query(const orc_tree *T, const float *o, const float *d, int64_t n, int model, uint32_t opts,
              double *L, double *alpha, int32_t *count, uint64_t *hash, int32_t *term_idx,
              int32_t *n_comp, int32_t *n_nodes, uint32_t *flags,
              double *alt_L, double *alt_alpha, int32_t *alt_count, uint64_t *alt_hash,
              int32_t *alt_term, uint8_t *alt_valid,
              uint32_t *leaf_ids, int32_t max_ids, int n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        orc_result R;
        march(T, o + 3 * i, d + 3 * i, model, opts, -1, &R,
              leaf_ids ? leaf_ids + (size_t)i * max_ids : NULL, max_ids);
        if (L) { L[3 * i] = R.L[0]; L[3 * i + 1] = R.L[1]; L[3 * i + 2] = R.L[2]; }
        if (alpha) alpha[i] = R.alpha;
        if (count) count[i] = R.count;
        if (hash) hash[i] = R.hash;
        if (term_idx) term_idx[i] = R.term_idx;
        if (n_comp) n_comp[i] = R.n_comp;
        if (n_nodes) n_nodes[i] = R.n_nodes_visited;
        if (flags) flags[i] = R.flags;
        if (alt_valid) alt_valid[i] = 0;
        if ((R.flags & ORC_AMBIGUOUS) && R.first_amb_test >= 0) {
            orc_result A;
            march(T, o + 3 * i, d + 3 * i, model, opts, R.first_amb_test, &A, NULL, 0);
            if (alt_L) { alt_L[3 * i] = A.L[0]; alt_L[3 * i + 1] = A.L[1]; alt_L[3 * i + 2] = A.L[2]; }
            if (alt_alpha) alt_alpha[i] = A.alpha;
            if (alt_count) alt_count[i] = A.count;
            if (alt_hash) alt_hash[i] = A.hash;
            if (alt_term) alt_term[i] = A.term_idx;
            if (alt_valid) alt_valid[i] = 1;
        }
    }
    return 0;
}

/*
 * Every valid outcome of a ray's alpha_max stop (the reading for rays with
 * several stop tests within eta of the threshold: each of them may go
 * either way, so the march may stop at any of them, or continue through all
 * of them; tests outside eta keep their FP64 decision).  Since 1 - T never
 * decreases, the ambiguous tests all come before the first clear stop, and
 * the outcomes are: candidate 0, continue at every ambiguous test; candidate
 * c = 1, 2, ..., stop at the c-th ambiguous test.  Outputs [n][max_cand]
 * (any may be NULL except valid): L [..][3], alpha, count, hash, term_idx,
 * n_comp, n_nodes, valid (1 for a candidate, 0 for unused slots).  A ray
 * with no ambiguous test has one candidate, the canonical outcome; a ray
 * with more than max_cand - 1 ambiguous tests gets the first ones.
 */
int orc_candidates(const orc_tree *T, const float *o, const float *d, int64_t n, int model, uint32_t opts,
                   int max_cand, double *L, double *alpha, int32_t *count, uint64_t *hash,
                   int32_t *term_idx, int32_t *n_comp, int32_t *n_nodes, uint8_t *valid, int n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int amb[64];
        int n_amb = 0;
        for (int c = 0; c < max_cand; ++c) valid[(size_t)i * max_cand + c] = 0;
        for (int c = 0; c < max_cand; ++c) {
            if (c > 0 && c > (n_amb < 64 ? n_amb : 64)) break;
            orc_result A;
            int ok = 1;
            const int force = c == 0 ? ORC_FORCE_CONTINUE : amb[c - 1];
            march_forced(T, o + 3 * i, d + 3 * i, model, opts, -1, force, &ok, c == 0 ? amb : NULL,
                         c == 0 ? 64 : 0, c == 0 ? &n_amb : NULL, &A, NULL, 0);
            const size_t j = (size_t)i * max_cand + c;
            if (L) { L[3 * j] = A.L[0]; L[3 * j + 1] = A.L[1]; L[3 * j + 2] = A.L[2]; }
            if (alpha) alpha[j] = A.alpha;
            if (count) count[j] = A.count;
            if (hash) hash[j] = A.hash;
            if (term_idx) term_idx[j] = A.term_idx;
            if (n_comp) n_comp[j] = A.n_comp;
            if (n_nodes) n_nodes[j] = A.n_nodes_visited;
            valid[j] = (uint8_t)ok;
        }
    }
    return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
