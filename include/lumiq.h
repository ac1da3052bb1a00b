/*
 * lumiq.h -- C ABI of the MI355X luminaire emission-query library.
 *
 * The library answers the render-time query of a learned radiance-field
 * luminaire (Condor & Jarabo, "A Learned Radiance-Field Representation for
 * Complex Luminaires", EGSR 2022): for rays leaving a shading point toward
 * the luminaire's proxy box it returns the emitted radiance L_e (Sec. 4.1,
 * Eq. 3) and the opacity alpha (Sec. 4.1, Eq. 5) by marching the distilled
 * plenoctree (Sec. 5).  It also trains and runs a small Fourier-feature MLP
 * that stands in for the octree march, with the octree as its fallback.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: every call returns lq_status; on failure lq_last_error()
 *    returns a message for the calling thread (valid until its next call).
 *    Argument errors are reported synchronously, before any launch.
 *  - Device pointers: ray and output arrays are *device* pointers on the
 *    handle's device, owned by the caller, contiguous, 4-byte aligned, and
 *    must not alias.  Host pointers are rejected with LQ_ERR_INVALID_ARG.
 *  - Streams: hip_stream is a hipStream_t (NULL = the default stream).  Calls
 *    are stream-ordered and asynchronous; device faults surface as LQ_ERR_HIP
 *    on a later call.
 *  - Rays: origins[n][3] and dirs[n][3] are float32.  dirs points from the
 *    shading point INTO the luminaire; it need not be unit length.  The
 *    paper's ray is x - omega t (Sec. 4.1, Eq. 3), so the emission direction
 *    at which the SH are evaluated is omega = -dirs/|dirs|.
 *  - Per-ray outcomes that are not errors: n = 0 is a no-op; a ray with a
 *    non-finite component or a zero direction, or that meets the proxy box
 *    [-1,1]^3 in no positive length, returns RGB 0 and alpha 0; an origin
 *    inside the box marches from t = 0.
 *  - Handles are immutable after creation and safe for concurrent queries
 *    on different streams.
 */
#ifndef LUMIQ_H
#define LUMIQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LQ_OK = 0,
    LQ_ERR_INVALID_ARG = -1,  /* bad pointer, size, enum or flag           */
    LQ_ERR_FORMAT = -2,       /* malformed tree file or descriptor         */
    LQ_ERR_OOM = -3,          /* device or host allocation failed          */
    LQ_ERR_HIP = -4,          /* HIP runtime error (incl. no device)       */
    LQ_ERR_UNSUPPORTED = -5,  /* valid but unsupported combination         */
    LQ_ERR_STATE = -6,        /* call not valid in the handle's state      */
    LQ_ERR_IO = -7            /* file could not be read or written         */
} lq_status;

/* storage precision of density and SH coefficients on the device */
enum { LQ_F32 = 0, LQ_F16 = 1, LQ_BF16 = 2 };
/* transmittance model: linear T = max(0, 1 - int sigma) (Sec. 4.1, Eq. 4),
 * or exponential T = exp(-int sigma) (the model compared in Sec. 6.2, Table 4) */
enum { LQ_LINEAR = 0, LQ_EXP = 1 };
/* query flags */
enum {
    LQ_NO_EARLY_TERM = 1,   /* march to the far proxy hit (no alpha_max stop)    */
    LQ_FP64_ACCUM = 2,      /* validation: accumulate T, weights and L in FP64   */
    LQ_NO_SIGMA_SKIP = 4,   /* composite every data leaf (no sigma_min skip)     */
    LQ_TRACE_PRUNED = 8     /* lq_query_trace only: see there                    */
};

typedef struct lq_octree lq_octree;   /* opaque, library-owned */
typedef struct lq_mlp lq_mlp;         /* opaque, library-owned */

/*
 * Plenoctree descriptor (host memory, read during the call only).
 *   child[n_nodes][8]: > 0 index of an internal node, < 0 -(leaf + 1), 0 empty.
 *     Node 0 is the root cube [-1,1]^3; octant index = bx | by<<1 | bz<<2 where
 *     b_a is 1 for the upper half along axis a.  Data leaves sit at max_depth
 *     (cells of edge 2^(1-max_depth)); the table must be a tree (every node
 *     reached once, leaves only below nodes of depth max_depth-1) of fewer
 *     than 2^29 nodes.
 *   sigma[n_leaves], sh[n_leaves][3][(sh_degree+1)^2] float32: density and
 *     real SH coefficients (orthonormal basis without the Condon-Shortley
 *     phase, index k = l^2 + l + m) per colour channel; emission is
 *     Phi_c = l_max * sigmoid(sum_k sh[c][k] Y_k(omega)) (Sec. 4.2, Eq. 6).
 *   sigma_min, alpha_max: render heuristics (Sec. 6.2: 0.1 and 0.9).
 */
typedef struct {
    int32_t max_depth;        /* 1..10 */
    int32_t sh_degree;        /* 0..4  */
    int32_t n_nodes, n_leaves;
    float l_max, sigma_min, alpha_max;
    const int32_t *child;
    const float *sigma;
    const float *sh;
} lq_octree_desc;

/*
 * Create a device octree from a descriptor (or from a file in the format
 * written by the inputs package: magic "LQOT", version 1, header then child,
 * sigma and sh arrays, little-endian).  storage selects the device precision
 * of sigma and SH (FP32 values are rounded to nearest-even).  The tree is
 * uploaded to `device`, which becomes current for the calling thread.
 * Errors: LQ_ERR_INVALID_ARG, LQ_ERR_FORMAT (structure check failed),
 * LQ_ERR_IO, LQ_ERR_OOM, LQ_ERR_HIP.  *out is NULL on failure.
 */
lq_status lq_load_octree_desc(const lq_octree_desc *desc, int storage, int device,
                              lq_octree **out);
lq_status lq_load_octree(const char *path, int storage, int device, lq_octree **out);
void lq_free_octree(lq_octree *tree);

/* Device bytes held by the tree's tables, and its shape. */
lq_status lq_octree_info(const lq_octree *tree, int64_t *device_bytes, int32_t *n_nodes,
                         int32_t *n_leaves, int32_t *max_depth, int32_t *sh_degree,
                         int32_t *storage);

/*
 * The emission query (Sec. 4.1, Eqs. 3-5; Sec. 5; Sec. 6.2 heuristics).
 * For each ray i: clip to the proxy box, visit in order of t the octree
 * leaves whose half-open cell the ray crosses in positive length, and for
 * each data leaf with stored sigma >= sigma_min composite
 *     w = T_in - T_out  (T by `model`),   L += w * Phi(omega),
 * stopping after the first composited leaf at which 1 - T >= alpha_max.
 * Outputs: rgb[n][3] (L_e) and, if alpha != NULL, alpha[n] = 1 - T.
 * Leaf-segment lengths and every ordering decision of the traversal are
 * exact (robust predicates on the float32 inputs); compositing is float32
 * (FP64 with LQ_FP64_ACCUM).
 */
lq_status lq_query_radiance(const lq_octree *tree, const float *origins, const float *dirs,
                            int64_t n, float *rgb, float *alpha, int model, uint32_t flags,
                            void *hip_stream);

/*
 * lq_query_radiance without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results (bit for bit), flags and
 * errors as lq_query_radiance.  The launch's only scratch -- 16 ray
 * counters, 128 bytes, whatever n -- lives in a static device array of the
 * library (one copy per GPU, held until the process ends), cleared by a
 * kernel at the start of every call.  Every call on one GPU shares that
 * array: calls that overlap in time on one GPU (concurrent streams, or
 * threads) race on it and give wrong results; serialise them.  Its address
 * is looked up on the first call on each device.
 */
lq_status lq_query_radiance_noalloc(const lq_octree *tree, const float *origins, const float *dirs,
                                    int64_t n, float *rgb, float *alpha, int model, uint32_t flags,
                                    void *hip_stream);

/*
 * Camera batch: the query of lq_query_radiance over the width * height rays
 * of an image stored row-major (ray y * width + x belongs to pixel (x, y)),
 * e.g. the primary rays of a rendered frame.  The results are those of
 * lq_query_radiance on the same arrays, ray for ray and bit for bit; only
 * the order in which the device takes the rays up differs: 8 x 8 pixel tiles
 * (the columns and rows beyond the last whole tile after them), so that the
 * 64 lanes of a wave march neighbouring pixels, which cross mostly the same
 * octree nodes.  Arrays hold width * height rays; width * height = 0 is a
 * no-op.  Errors: those of lq_query_radiance, and LQ_ERR_INVALID_ARG for a
 * negative width or height or width * height >= 2^31.
 */
lq_status lq_query_radiance_image(const lq_octree *tree, const float *origins, const float *dirs,
                                  int32_t width, int32_t height, float *rgb, float *alpha,
                                  int model, uint32_t flags, void *hip_stream);

/*
 * Validation variant of lq_query_radiance: same traversal and compositing,
 * plus per-ray records of the visited data leaves.  For each ray:
 *   count[i]     data leaves visited, up to and including the stop leaf;
 *   hash[i]      FNV-1a style hash: h = 14695981039346656037;
 *                h = (h ^ id) * 1099511628211 (mod 2^64) for each leaf id in order,
 *                where id is the Morton code of the leaf cell (x bit b -> bit 3b,
 *                y -> 3b+1, z -> 3b+2);
 *   term_idx[i]  index (in that sequence) of the leaf at which alpha_max
 *                stopped the march, or -1;
 *   n_comp[i]    leaves composited;
 *   n_steps[i]   optional: octree nodes visited (data leaves and empty
 *                nodes, each reached by one descent), up to the stop;
 *   leaf_ids     optional [n][max_ids]: the first max_ids leaf ids.
 * rgb/alpha may be NULL.  All arrays are device pointers.
 * With LQ_TRACE_PRUNED the trace marches the table that lq_query_radiance
 * marches: the tree without the data leaves whose stored density is below
 * sigma_min and without the nodes they leave empty (Sec. 6.2: those leaves
 * are never composited).  Radiance and alpha are those the production
 * query computes; the records then list only the composited leaves (count
 * = n_comp) and n_steps counts the nodes of that table visited -- the work
 * of the production query.  It combines with LQ_NO_EARLY_TERM only.
 */
lq_status lq_query_trace(const lq_octree *tree, const float *origins, const float *dirs,
                         int64_t n, float *rgb, float *alpha, int model, uint32_t flags,
                         uint32_t *count, uint64_t *hash, int32_t *term_idx, uint32_t *n_comp,
                         uint32_t *n_steps, uint32_t *leaf_ids, int32_t max_ids,
                         void *hip_stream);

/*
 * Multi-luminaire batch: rays [ray_offsets[k], ray_offsets[k+1]) query
 * trees[k], all in one persistent launch.  ray_offsets is a HOST array of
 * n_trees + 1 non-decreasing values starting at 0; origins/dirs/rgb/alpha
 * are device arrays of ray_offsets[n_trees] rays.  Every tree must live on
 * the same device and share its storage and SH degree, which must be 2 or 3
 * (else LQ_ERR_UNSUPPORTED); ray_offsets[n_trees] must not exceed 2^40.
 * Same per-ray semantics as lq_query_radiance.  The trees' device
 * descriptors and the offsets are staged from host memory through
 * stream-ordered scratch: the call synchronises hip_stream once, before
 * the launch, so that the host copies are complete when it returns.
 */
lq_status lq_query_radiance_multi(const lq_octree *const *trees, int32_t n_trees,
                                  const int64_t *ray_offsets, const float *origins,
                                  const float *dirs, float *rgb, float *alpha, int model,
                                  uint32_t flags, void *hip_stream);

/*
 * Consumer side: irradiance at shading points from the light leaving the
 * proxy box.  The radiance leaving the proxy along a ray is the emission
 * plus the light behind the luminaire seen through it (Sec. 3, Eq. 2):
 *     L_o = L_e + (1 - alpha) L_b,
 * with L_e and alpha as lq_query_radiance returns them and L_b the constant
 * colour background_rgb (host float[3]; NULL = black).  The proxy is sampled
 * uniformly over its surface (Sec. 6, Sampling): sample s of point i reads
 * u[i][s][0..2] in [0,1) (values outside give unspecified finite results),
 * picks face f = floor(6 u0) (axis f/2; the face at -1 for even f, +1 for
 * odd) and on it the point with coordinates 2 u1 - 1 and 2 u2 - 1 on the
 * next two axes in cyclic order, at area density 1/24.  The ray goes from
 * the point x to that face point y (float32: d = y - x).  A sample whose
 * face x does not see from the front, or that lies below x's tangent plane
 * (normal[i], any nonzero length), weighs 0; otherwise its term is
 *     L_o cos(theta_x) cos(theta_y) / (|y - x|^2 / 24),
 * and irradiance[i][c] is the mean of the terms over the n_samples samples
 * (an unbiased estimate of the integral of L_o cos(theta_x) over the box's
 * solid angle; a Lambertian surface of albedo rho reflects rho / pi of it).
 * Points inside the proxy receive 0.  model: LQ_LINEAR or LQ_EXP, default
 * query flags.  points, normals [n_points][3], u [n_points][n_samples][3],
 * irradiance [n_points][3] and the optional sample_terms
 * [n_points][n_samples][3] (each sample's term) are float32 device arrays.
 * Scratch: 52 bytes per sample, stream-ordered; only samples that weigh
 * more than 0 are marched.  Sums are FP64 in a fixed
 * order (deterministic).  Errors: LQ_ERR_INVALID_ARG for a NULL tree, a bad
 * model, n_samples outside 1..65536, n_points * n_samples >= 2^36, or a bad
 * array; LQ_ERR_OOM; LQ_ERR_HIP.
 */
lq_status lq_proxy_irradiance(const lq_octree *tree, const float *points, const float *normals,
                              int64_t n_points, const float *u, int32_t n_samples,
                              const float *background_rgb, int model, float *irradiance,
                              float *sample_terms, void *hip_stream);

/*
 * Radiance-field-guided sampling of the proxy: the importance sampling that
 * the paper leaves as future work (Sec. 6, Sampling; Sec. 7, Limitations --
 * Sampling), in a form of this library's.  The proxy's surface is cut into
 * 6 grid^2 cells: face f (as in lq_proxy_irradiance), then grid x grid
 * cells on it along the face's next two axes in cyclic order, cell
 * k = (f grid + i) grid + j.
 *
 * Direction bins: with dir_res = D > 1 the guide is directional.  An
 * outward direction w through face f (axis a) falls in bin i1 D + i2,
 * where i1 and i2 are the tangent bins of its components on axes a + 1 and
 * a + 2 (cyclic).  The tangent bin of a component v, with l2 = |w|^2
 * summed in axis order, is the number of thresholds th_j = 2 j / D - 1
 * (j = 1..D-1) that v / sqrt(l2) reaches.  Each test is decided on
 * squares in FP64: for th < 0, v >= 0 or v^2 <= th^2 l2; for th = 0,
 * v >= 0; for th > 0, v >= 0 and v^2 >= th^2 l2.  dir_res in 1..4.
 *
 * lq_proxy_guide: the guide weights, D^2 per cell (cell-major, weight
 * k D^2 + b).  Weight (k, b) is the mean luminance (mean of R, G, B) of
 * the emission that lq_query_radiance returns for those of the cell's
 * n_probes probe rays whose outward direction -d falls in bin b.  A bin
 * that none of them fell in takes the mean over all the cell's probes
 * (D = 1: that mean alone).  Probe r of cell k reads
 * u_probe[k][r][0..4] in [0, 1): it starts at the cell's point with
 * coordinates -1 + (i + u0) 2 / grid and -1 + (j + u1) 2 / grid (float32)
 * and aims at the point 2 (u2, u3, u4) - 1 inside the box.
 * weights [6 grid^2 D^2] float32, u_probe [6 grid^2][n_probes][5]
 * float32: device arrays.  The probe luminances are summed in FP64 in probe
 * order.
 *
 * lq_proxy_irradiance_guided: lq_proxy_irradiance with the sample's cell
 * drawn from the guide, weights [6 grid^2 D^2] as lq_proxy_guide writes
 * them.  Each direction bin b has its own table.  With W_b the sum of the
 * bin's weights (a weight that is negative, NaN or infinite counts as 0),
 * cell k has probability
 *     p_b[k] = (1 - defensive) w_(k,b) / W_b + defensive / (6 grid^2)
 * (1 / (6 grid^2) each when W_b = 0), summed in cell order in FP64 into
 * cdf_b[0] = 0, cdf_b[k + 1] = cdf_b[k] + p_b[k].  A point receives light
 * only through the faces it sees from the front (side * x_axis > 1), so
 * its samples pick among those faces' cells.  On face f it uses the table
 * of b_f, the bin of its direction x - c_f from the face's centre c_f
 * (side on the face's axis, 0 on the others).  The face's guide mass is
 * P_f = cdf_b_f[(f + 1) grid^2] - cdf_b_f[f grid^2], and its geometry
 * weight is
 *     g_f = max(0, n.(c_f - x)) (side x_axis - 1) / |c_f - x|^4,
 * the integrand cos(theta_x) cos(theta_y) / r^2 at c_f up to the constant
 * 1 / |n|.  With P_vis and S the sums of P_f and P_f g_f over the visible
 * faces, face f is chosen with probability
 *     Q_f = 0.5 P_f g_f / S + 0.5 P_f / P_vis   (P_f / P_vis when S = 0).
 * Sample s of point i walks the visible faces in order with
 * t = u[i][s][0].  In the face where t < Q_f (the last visible face takes
 * any remainder) it picks the largest cell k of the face with
 * cdf_b_f[k] <= cdf_b_f[f grid^2] + (t / Q_f) P_f (t / Q_f taken as 0 when
 * Q_f = 0), and the point of that cell at u[i][s][1], u[i][s][2] as above.
 * All of the choice is FP64 from the float32 inputs, sums in axis and face
 * order.  The sample's area density is p_b_f[k] (Q_f / P_f) / (2 / grid)^2,
 * and its term L_o cos(theta_x) cos(theta_y) / (|y - x|^2 p_A) (zero as in
 * lq_proxy_irradiance, for a point that sees no face, and for a cell of
 * p_b_f[k] Q_f = 0).  The estimate stays unbiased for any guide with
 * defensive > 0; defensive in [0, 1], grid in 1..256.  Scratch: as
 * lq_proxy_irradiance plus 8 D^2 (12 grid^2 + 1) bytes.
 */
lq_status lq_proxy_guide(const lq_octree *tree, int32_t grid, int32_t dir_res, int32_t n_probes,
                         const float *u_probe, int model, float *weights, void *hip_stream);
lq_status lq_proxy_irradiance_guided(const lq_octree *tree, const float *points, const float *normals,
                                     int64_t n_points, const float *u, int32_t n_samples,
                                     const float *weights, int32_t grid, int32_t dir_res, float defensive,
                                     const float *background_rgb, int model, float *irradiance,
                                     float *sample_terms, void *hip_stream);

/* ------------------------------------------------------------------------
 * Plenoctree distillation (Sec. 5, "Creating the plenoctree"): a density
 * sample at the centre of every voxel of the finest grid (2^max_depth per
 * axis over [-1,1]^3), pruning of the voxels whose centre density is below
 * prune_sigma (0.01 in the paper), and for every voxel kept the mean density
 * and mean SH coefficients of n_samples uniformly random positions inside
 * it (256 in the paper, against aliasing at discontinuities); the octree
 * over the kept voxels collapses empty octants bottom-up.
 *
 * The continuous field stands in for a trained radiance field:
 *   density(x) = sigma_max inside a shell (| |x - s_j| - R_j | < shell_half_width),
 *              = min(exp(log_density_base + sum_k a_k g_k(x)), sigma_max) elsewhere,
 *   g_k(x) = exp(-|x - c_k|^2 / (2 r_k^2));
 * its emission coefficients are blended by w_k(x) = g_k(x) / sum_j g_j(x):
 *   coefficient 0 of channel c = logit(E_c(x) / l_max) / Y_00, E_c = sum_k w_k e_kc
 *     (so that Eq. 6's l_max sigmoid(...) returns E_c for that band alone),
 *   coefficient j >= 1 of channel c = sum_k w_k h_kcj (index j = l^2 + l + m).
 * The random positions come from Philox4x32-10 (Salmon et al., SC 2011):
 * counter (Morton code of the voxel, sample index, 0, 0), key (low and high
 * 32 bits of seed); the first three output words u give the offsets
 * (u >> 8) 2^-24 along x, y, z in units of the voxel edge.  Decisions (the
 * centre test, shell membership) are taken as in FP64; per sample, the blob
 * exponents are FP64 and the exponentials and sums float32; the sums over
 * samples are FP64 across blocks of 16 samples.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_blobs;          /* 1..32                                           */
    int32_t n_shells;         /* 0..8                                            */
    int32_t sh_degree;        /* 0..4                                            */
    int32_t reserved;
    const double *blobs;      /* host [n_blobs][8]: centre x, y, z (in [-2, 2]),
                                 radius r (in [1e-3, 4]), log-density amplitude a
                                 (|a| <= 12), radiance e_r, e_g, e_b (each in
                                 (0, l_max))                                     */
    const double *blob_sh;    /* host [n_blobs][3][(sh_degree+1)^2 - 1]: h_kcj for
                                 j >= 1 (NULL for degree 0)                      */
    const double *shells;     /* host [n_shells][4]: centre x, y, z, radius (each
                                 in [-2, 2])                                     */
    double shell_half_width, log_density_base, sigma_max, l_max;
} lq_field_desc;

/*
 * Distil the leaves: codes[i] (ascending Morton codes of the kept voxels,
 * x bit b -> bit 3b, y -> 3b+1, z -> 3b+2), sigma[i] and sh[i][3][K] (the
 * means), device arrays of `capacity` entries on `device`.  *n_leaves (host)
 * receives the number of voxels kept.  capacity = 0 only counts them (the
 * arrays may then be NULL); a count above capacity is LQ_ERR_INVALID_ARG
 * with *n_leaves set and nothing written.  The call synchronises hip_stream
 * (the count decides the launch size).  Errors: LQ_ERR_INVALID_ARG,
 * LQ_ERR_UNSUPPORTED (more than 32 blobs or 8 shells), LQ_ERR_OOM,
 * LQ_ERR_HIP.
 */
lq_status lq_distill_leaves(const lq_field_desc *field, int32_t max_depth, float prune_sigma,
                            int32_t n_samples, uint64_t seed, int device, int64_t capacity,
                            uint32_t *codes, float *sigma, float *sh, int64_t *n_leaves,
                            void *hip_stream);

/*
 * An octree from leaves at max depth: codes (device, strictly ascending
 * Morton codes below 8^max_depth, else LQ_ERR_FORMAT), sigma [n] and
 * sh [n][3][K] (device, float32).  The child table is built on the device
 * by collapsing empty octants bottom-up (nodes breadth-first, Morton order
 * within a level; leaf i is codes[i]) and the tree is then loaded as by
 * lq_load_octree_desc (its storage conversion and tables); synchronous.
 */
lq_status lq_octree_from_leaves(int32_t max_depth, int32_t sh_degree, const uint32_t *codes,
                                const float *sigma, const float *sh, int64_t n_leaves, float l_max,
                                float sigma_min, float alpha_max, int storage, int device,
                                lq_octree **out);

/*
 * Copy a tree's tables to host memory: child [n_nodes][8], sigma [n_leaves]
 * and sh [n_leaves][3][K] (any may be NULL), with the sizes lq_octree_info
 * reports; values as stored (float16 / bfloat16 widened exactly to
 * float32).  Synchronous.
 */
lq_status lq_octree_download(const lq_octree *tree, int32_t *child, float *sigma, float *sh);

/* ------------------------------------------------------------------------
 * Learned surrogate.  A ray is reduced to the point where its line enters
 * the sphere of radius sqrt(3) bounding the proxy box and its unit direction
 * (the 5D light-field coordinates of Sec. 3, Eq. 1), encoded with 10
 * frequencies of Fourier features (the positional encoding of Sec. 4.2),
 * and mapped by a 4 x 64 ReLU MLP to y = log(L + 0.01).  Training minimises
 * the HDR relative loss of Sec. 4.3, Eq. 8 (lambda = 1, epsilon = 0.01, the
 * channel mean of the prediction as luminance, held constant in the
 * gradient) with Adam and an exponentially decaying learning rate
 * (Sec. 4.4).  GEMMs run on MFMA in bfloat16 with float32 accumulation;
 * master weights and Adam moments are float32.  A line that misses the
 * sphere has radiance 0.  Parameters are one float32 vector of
 * lq_mlp_num_params() values: per layer W[out][in] row-major then b[out],
 * layers 128->64, 64->64, 64->64, 64->64, 64->3.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_freq;           /* must be 10 */
    int32_t hidden;           /* must be 64 */
    int32_t n_hidden_layers;  /* must be 4  */
} lq_mlp_config;

typedef struct {
    int32_t steps;        /* optimiser steps to run in this call                  */
    int32_t total_steps;  /* length of the learning-rate schedule                 */
    int32_t batch;        /* samples per step, a positive multiple of 64          */
    float lr0, lr1;       /* learning rate decays from lr0 (step 0) to lr1 (total) */
    float beta1, beta2, eps;
} lq_train_config;

/* Create a surrogate on `device` with He-uniform weights drawn from `seed`
 * (cfg may be NULL).  Errors: LQ_ERR_UNSUPPORTED for another shape. */
lq_status lq_mlp_create(const lq_mlp_config *cfg, uint64_t seed, int device, lq_mlp **out);
void lq_mlp_free(lq_mlp *mlp);
int32_t lq_mlp_num_params(void);
/* Copy the float32 master parameters to / from host memory; set also
 * clears the Adam state and the step counter. */
lq_status lq_mlp_get_params(const lq_mlp *mlp, float *host_params);
lq_status lq_mlp_set_params(lq_mlp *mlp, const float *host_params);

/*
 * Train on n_pairs (ray, radiance) pairs (device arrays origins/dirs [n][3],
 * rgb [n][3] float32).  Step k of the run (counted over all calls) uses the
 * `batch` pairs starting at (k * batch) mod n_pairs, so the pair set should
 * be in random order.  Deterministic: the batch-gradient reduction has a
 * fixed order.  loss_log_host (nullable, host) receives one batch loss per
 * step of this call.  Synchronises the stream when loss_log_host is given.
 */
lq_status lq_mlp_train(lq_mlp *mlp, const float *origins, const float *dirs, const float *rgb,
                       int64_t n_pairs, const lq_train_config *cfg, float *loss_log_host,
                       void *hip_stream);

/* Batch loss (host, nullable) and its gradient (device float32 [n_params])
 * at the current parameters over n pairs; no update.  Synchronises. */
lq_status lq_mlp_grad(lq_mlp *mlp, const float *origins, const float *dirs, const float *rgb,
                      int64_t n, float *grad, float *loss_host, void *hip_stream);

/* Surrogate radiance rgb[n][3] = max(exp(y) - 0.01, 0) for every ray. */
lq_status lq_mlp_forward(const lq_mlp *mlp, const float *origins, const float *dirs, int64_t n,
                         float *rgb, void *hip_stream);

/*
 * Trust map: held-out (ray, reference radiance) pairs are binned by the
 * octahedral cells (32 x 32) of the entry direction and of the ray
 * direction (1,048,576 bins).  A bin is trusted when it holds at least 32
 * pairs and every one of them is within the bound: sum_c (L_c - ref_c)^2 <=
 * max_rel_err^2 sum_c ref_c^2 + (0.01)^2 (an absolute floor of 0.01 radiance
 * units for dark rays).  The bins of lines that no held-out pair met, or met
 * fewer than 32 times, fall back.  Synchronises the stream.
 */
lq_status lq_mlp_build_trust(lq_mlp *mlp, const float *origins, const float *dirs,
                             const float *rgb_ref, int64_t n, float max_rel_err, void *hip_stream);
/* Copy the trust map (host, nullable) and report its size (0 if none). */
lq_status lq_mlp_trust_map(const lq_mlp *mlp, uint8_t *host_map, int32_t *n_bins);

/*
 * Surrogate with octree fallback.  A classification pass splits the batch on
 * the device.  The network models the radiance of a whole line, which a ray
 * sees only when the bounding sphere lies wholly ahead of its origin: rays
 * whose line misses the sphere, or whose sphere lies wholly behind them, get
 * radiance 0; rays that start inside the sphere go to the octree list; the
 * others go to a surrogate list when their trust bin is trusted, else to
 * the octree list.
 * The surrogate then answers only its list and lq_query_radiance on
 * `fallback` (linear model, default flags) only the other;
 * used_fallback[n] (device, nullable) marks the rays the octree answered.
 * No host synchronisation; the lists live in stream-ordered scratch
 * (16 n + 16 bytes).  Without a trust map or a fallback tree this is
 * lq_mlp_forward.
 */
lq_status lq_mlp_infer(const lq_mlp *mlp, const lq_octree *fallback, const float *origins,
                       const float *dirs, int64_t n, float *rgb, uint8_t *used_fallback,
                       void *hip_stream);

/* Checkpoint: parameters, Adam moments, step counter and trust map.
 * Resuming from a checkpoint and training N more steps is bit-identical to
 * training without the interruption. */
lq_status lq_mlp_save(const lq_mlp *mlp, const char *path);
lq_status lq_mlp_load(const char *path, int device, lq_mlp **out);

/* Text of the last error on this thread ("" if none). */
const char *lq_last_error(void);
/* Library version string. */
const char *lq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LUMIQ_H */
