/*
 * rvis.h -- C ABI of the MI355X (gfx950) visibility tracer for 3D Gaussians.
 *
 * The library implements the point-based ray tracing of "Relightable 3D
 * Gaussians" (arXiv 2311.16043), Sec. 4: a bounding volume hierarchy built as
 * a binary radix tree over the Gaussians (Sec. 4.1, after Karras 2012), all-hit
 * traversal that attenuates transmittance T by (1 - alpha_j) for every
 * Gaussian a ray crosses (Sec. 4.1, Eq. (15)), with alpha_j the Gaussian's
 * contribution at its equivalent intersection point (Eq. (13)-(14)), early
 * termination below T_min, and per-Gaussian visibility pre-computation over N
 * directions of the hemisphere about each normal (Sec. 4.2; directions from
 * Fibonacci sampling, Sec. 3.3). Around that path: the adjoint of T with
 * respect to opacity, mean and log-scale, and a small MLP visibility
 * surrogate with tracer fallback.
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch-owned)
 *    unless stated otherwise. Arrays are dense, row-major, FP32 unless stated.
 *  - `stream` is a hipStream_t (NULL = the default stream). Every call only
 *    enqueues work on that stream and returns; nothing is synchronised. Inputs
 *    must stay unchanged and alive until the stream has executed the call.
 *  - The library never allocates device memory. Callers size buffers with the
 *    *_bytes() queries and pass them in; the library owns nothing between calls.
 *  - Every call validates its arguments before enqueuing anything and returns
 *    an rv_status. On failure nothing has been enqueued (except RV_ERR_HIP,
 *    reported after a failed launch) and rv_last_error() describes the cause.
 *  - Ray ids: ray r = i * K + k is direction k of Gaussian i (original, not
 *    sorted, order); ids are 64-bit.
 *  - A BVH blob records the number of Gaussians it was built over (header
 *    word 12), and every section offset follows from that number. Entry
 *    points that take a blob and a Gaussian set compare the two on the device
 *    before reading anything else in the blob: with a different g->n the
 *    traversals write NaN to their per-ray, per-Gaussian and gradient
 *    outputs, and rv_refit_bvh leaves the blob unchanged. The host cannot see
 *    device memory without synchronising, so such a call still returns RV_OK.
 */
#ifndef RVIS_H
#define RVIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rv_status;
#define RV_OK 0
#define RV_ERR_INVALID_ARG (-1)
#define RV_ERR_WORKSPACE (-2)
#define RV_ERR_HIP (-3)
#define RV_ERR_UNSUPPORTED (-4)

/* Largest Gaussian count the library accepts (node ids are 32-bit). */
#define RV_MAX_GAUSSIANS (1LL << 30)

/*
 * The geometric part of the Gaussian set (Sec. 3.1: mean mu, unit quaternion
 * q, scale s, opacity o; the normal n is the per-Gaussian attribute added in
 * Sec. 3.3). Covariance Sigma = R(q) S S^T R(q)^T with S = diag(exp(log_scale)).
 *   mean      [n][3]
 *   quat      [n][4]  (w, x, y, z); normalised by the library before use
 *   log_scale [n][3]
 *   opacity   [n]
 *   normal    [n][3]  unit normal (normalised before use); may be NULL when
 *                     only sphere-mode directions are traced
 */
typedef struct rv_gaussians {
    const float *mean;
    const float *quat;
    const float *log_scale;
    const float *opacity;
    const float *normal;
    int64_t n;
} rv_gaussians;

/*
 * Tracing parameters. A Gaussian j contributes to the ray leaving Gaussian i
 * iff j != i, its peak parameter t_j >= t_min(i) = tmin_scale * max scale of i,
 * its squared Mahalanobis distance at the peak q_j <= sigma_cut^2 and
 * alpha_j = o_j exp(-q_j / 2) >= alpha_min; it then multiplies T by
 * 1 - min(alpha_j, alpha_max). A ray stops once T < T_min (0 disables the
 * early exit); the value returned is T at that point.
 * dir_mode 0: directions are world-frame unit vectors (sphere).
 * dir_mode 1: directions are local (x, y, z) with +z along the Gaussian's
 *             normal (hemisphere), rotated by the Duff et al. 2017 basis.
 * Defaults: {1/255, 0.99, 1e-4, 3, 3, 1}.
 */
typedef struct rv_trace_params {
    float alpha_min;
    float alpha_max;
    float T_min;
    float sigma_cut;
    float tmin_scale;
    int32_t dir_mode;
} rv_trace_params;

/* Device pointers into a built BVH blob (see rv_bvh_view). */
typedef struct rv_bvh_arrays {
    int64_t n;
    const float *header;        /* [16]: lo[3], hi[3] of the means, root box lo[3], hi[3], ... */
    const uint64_t *keys;       /* [n]   63-bit Morton keys, sorted ascending */
    const uint32_t *perm;       /* [n]   sorted position -> original index */
    const float *nodes;         /* [n-1][16] internal nodes, see below */
    const int32_t *parent;      /* [2n-1] parent of internal node i at i, of leaf m at n-1+m; root -1 */
    const float *leaf_records;  /* [n][12] per sorted leaf: mu[3], o, W row0[3], s0 s1/s2, W row1[3], src;
                                   W = diag(1/s) R^T, row 2 = (s0 s1/s2) (row0 x row1) */
    const float *leaf_boxes;    /* [n][6]  per sorted leaf: lo[3], hi[3] (3-sigma box, widened outward) */
    const float *origins;       /* [n][4]  per sorted leaf: unit normal[3], t_min */
    const uint32_t *nodes4;     /* [n-1][16] compressed four-wide node per internal node, see rv_build_bvh */
} rv_bvh_arrays;

/* const char* describing the last failure on the calling thread ("" if none). */
const char *rv_last_error(void);

/* Library version string. */
const char *rv_version(void);

/* ------------------------------------------------------------------------ */
/* BVH build (Sec. 4.1)                                                     */
/* ------------------------------------------------------------------------ */

/* Bytes of the BVH blob for n Gaussians (256-byte aligned sections). */
size_t rv_bvh_bytes(int64_t n);

/* Bytes of build scratch for n Gaussians. */
size_t rv_build_workspace_bytes(int64_t n);

/*
 * Build the LBVH of the Gaussian set g into `bvh` (rv_bvh_bytes(g->n) bytes,
 * 256-byte aligned). Steps (all on `stream`): scene bounds of the means;
 * 63-bit Morton keys (21 bits per axis, binary32 quantisation
 * u = (x - lo) / (hi - lo), c = min(floor(u * 2^21), 2^21 - 1), x bits most
 * significant in each triplet); stable LSD radix sort of (key, index);
 * binary radix tree with Karras 2012 node numbering (internal node i has one
 * end of its key range at i; the root is node 0; children are written as the
 * internal id, or ~m for leaf m); per-leaf records in sorted order; refit of
 * the 3-sigma boxes (each child box the union of the leaf boxes under it).
 * Node record (16 floats): left-child box lo[3], hi[3], right-child box lo[3],
 * hi[3], then the left and right child ids, then the first and last sorted
 * leaf under the node, all four as int32 bit patterns. Compressed four-wide record of
 * internal node i (16 words, the one the tracer walks) lists the children of
 * i's two children; a leaf child keeps its own slot and the next slot is
 * empty. Words 0-2: origin O (float); word 3: bytes 0-2 per-axis step
 * exponents (step_a = 2^(byte - 127)), byte 3 the kind of slot j in bits
 * 2j..2j+1 (0 empty, 1 internal node, 3 leaf); words 4-9: lo_x, lo_y, lo_z,
 * hi_x, hi_y, hi_z planes, byte j for slot j, plane = O_a + byte * step_a;
 * words 10-11: index of slot 2s for side s (slot 2s + 1 holds index + 1);
 * words 12-15 zero. Planes lie outside the binary child boxes by at least
 * eta = (largest root-box coordinate + root diagonal + 1) * 2^-20 and by at
 * most eta + one step.
 * The result depends only on the inputs (bit-identical across runs).
 * Errors: RV_ERR_INVALID_ARG (null pointers, n < 1, n > RV_MAX_GAUSSIANS,
 * unaligned bvh), RV_ERR_WORKSPACE (bvh_bytes or ws_bytes too small),
 * RV_ERR_HIP (launch failure).
 */
rv_status rv_build_bvh(const rv_gaussians *g, void *bvh, size_t bvh_bytes, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Refit a built BVH to moved Gaussians (scene edits and compositions,
 * Sec. 4.3): g must be the set the blob was built from (same n, same
 * indices), with any means, rotations, scales, opacities and normals. The
 * build's sorted order, Morton keys and topology are kept; the means' box,
 * leaf records, 3-sigma boxes, origin data, internal boxes and four-wide
 * records are recomputed exactly as rv_build_bvh computes them. Traversal
 * stays exact (boxes are recomputed, so they stay conservative); its cost
 * grows as moved Gaussians drift from their neighbours in the old order, and
 * a rebuild restores it. Same workspace as rv_build_bvh. With unchanged
 * inputs the blob is reproduced bit for bit.
 * Errors: as rv_build_bvh.
 */
rv_status rv_refit_bvh(const rv_gaussians *g, void *bvh, size_t bvh_bytes, void *ws, size_t ws_bytes, void *stream);

/* Host-side decoding of a BVH blob into device pointers (no device access). */
rv_status rv_bvh_view(const void *bvh, int64_t n, rv_bvh_arrays *out);

/* ------------------------------------------------------------------------ */
/* Visibility (Sec. 4.1 traversal, Sec. 4.2 pre-computation)                */
/* ------------------------------------------------------------------------ */

/*
 * Bytes of trace scratch: 256 bytes of work-queue counters, then room for the
 * n*K per-ray values (used when the mean is wanted without per-ray output).
 */
size_t rv_trace_workspace_bytes(int64_t n, int32_t K);

/*
 * Trace all n*K rays: ray (i, k) starts at mean_i with direction k of `dirs`
 * ([K][3], see dir_mode), after `bvh` was built from the same g. Writes
 * vis_ray[i*K + k] = T of that ray (if vis_ray != NULL) and
 * vis_mean[i] = (1/K) sum_k T (if vis_mean != NULL); at least one of them must
 * be given. ws: device scratch, 256-byte aligned, at least
 * rv_trace_workspace_bytes(n, K) bytes, or 256 bytes when vis_ray is given;
 * calls that share a ws must not overlap. Deterministic: each ray's T does
 * not depend on scheduling, and the mean adds the row in FP64 in a fixed
 * order.
 * Errors: RV_ERR_INVALID_ARG (null g/bvh/dirs/params, K < 1, both outputs
 * NULL, dir_mode 1 with NULL normals, out-of-range parameters, missing or
 * unaligned ws), RV_ERR_WORKSPACE (ws_bytes too small), RV_ERR_HIP.
 */
rv_status rv_trace_visibility(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                              const rv_trace_params *p, float *vis_ray, float *vis_mean, void *ws,
                              size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rv_trace_visibility with its scratch (the work-queue counters, and the
 * per-ray values when vis_ray is NULL) taken from a static array that the
 * library holds on each device it runs on until the process ends, of
 * rv_trace_static_scratch_bytes() = 32 MiB. The call allocates nothing; the
 * caller passes the inputs and outputs as for rv_trace_visibility and gets the
 * same bits. Without vis_ray, n*K must be at most (32 MiB - 256) / 4 =
 * 8,388,544 rays, else RV_ERR_WORKSPACE and nothing is enqueued; with vis_ray
 * any size is accepted. Every call on a device shares that device's array:
 * calls that overlap on one device (on different streams, or from several
 * threads) race and give undefined results; calls on one stream are ordered.
 * The counters are cleared by a kernel at the start of every call (never a
 * memset, so the call can be captured in a graph).
 * Errors: as rv_trace_visibility, RV_ERR_WORKSPACE (size beyond the scratch),
 * RV_ERR_HIP (no current device, or the scratch could not be located).
 */
size_t rv_trace_static_scratch_bytes(void);
rv_status rv_trace_visibility_static(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                     const rv_trace_params *p, float *vis_ray, float *vis_mean, void *stream);

/*
 * Trace an explicit list of ray ids (device int64 [n_rays], r = i*K + k) and
 * write out[s] = T of ray ids[s]. Gives the same bits as rv_trace_visibility
 * for the same ray.
 */
rv_status rv_trace_rays(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                        const rv_trace_params *p, const int64_t *ray_ids, int64_t n_rays, float *out,
                        void *stream);

/*
 * Bytes of the workspace of rv_trace_visibility_sh: 256 bytes of queue
 * counters, the K x 9 table of Y_j(d_k), and the per-ray values of one batch
 * of Gaussians (at most 2^28 values, 1 GiB, however large n is).
 */
size_t rv_trace_sh_workspace_bytes(int64_t n, int32_t K);

/*
 * Visibility compressed to spherical harmonics, without per-ray output: the
 * same rays and transmittances as rv_trace_visibility (the same traversal, so
 * the same T for every ray), each Gaussian's K values projected onto the real
 * SH of degree <= 2 (the "3-level SH" of Sec. 3.3) by the quadrature of
 * Eq. (10): vis_sh[i][j] = sum_k T_ik Y_j(d_k) dw, dw = 2 pi / K (hemisphere)
 * or 4 pi / K (sphere), d_k the table's unit directions in the rays' frame
 * (local about the normal in hemisphere mode), basis order (0,0), (1,-1),
 * (1,0), (1,1), (2,-2), (2,-1), (2,0), (2,1), (2,2). vis_mean (optional) is
 * the mean of T over the K directions. Deterministic (fixed summation order).
 * vis_sh: [n][9] FP32 (device); ws: rv_trace_sh_workspace_bytes(n, K) bytes,
 * 256-byte aligned. Errors: as rv_trace_visibility, RV_ERR_WORKSPACE.
 */
rv_status rv_trace_visibility_sh(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                 const rv_trace_params *p, float *vis_sh, float *vis_mean, void *ws, size_t ws_bytes,
                                 void *stream);

/*
 * Traversal statistics of rv_trace_visibility's rays: writes (device)
 * totals[0] = four-wide node visits, totals[1] = leaf records tested,
 * totals[2] = Gaussians included, summed over all n*K rays (int64, overwritten).
 * Used to compute algorithmic bytes; runs a separate instrumented kernel.
 * totals[1] and totals[2] are fixed by the rays; totals[0] can vary by a few
 * visits between runs: a ray keeps walking while the leaves it found wait for
 * its wave's leaf test, and the visits made before the leaf that ends it by
 * T < T_min depend on scheduling (its T does not).
 * ws: at least 256 bytes of device scratch, 256-byte aligned (work-queue
 * counters). Errors: as rv_trace_visibility.
 */
rv_status rv_trace_stats(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                         const rv_trace_params *p, int64_t *totals, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Copy `bytes` (a multiple of 16; 16-byte aligned pointers) from src to dst on
 * `stream` with a grid-stride streaming kernel: the achievable-bandwidth probe
 * for the roofline and the known-size reference for hardware byte counters.
 * Errors: RV_ERR_INVALID_ARG (null or misaligned pointers, bad size), RV_ERR_HIP.
 */
rv_status rv_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/*
 * Read-only streaming probe: reads `bytes` (a positive multiple of 16;
 * 16-byte aligned src) once with non-temporal loads; each thread stores the
 * XOR of what it read to sink (device uint32 [rv_stream_read_sink_words(bytes)]).
 * The achievable read bandwidth: the denominator for kernels whose HBM
 * traffic is reads. Errors: RV_ERR_INVALID_ARG, RV_ERR_HIP.
 */
size_t rv_stream_read_sink_words(size_t bytes);
rv_status rv_stream_read(const void *src, size_t bytes, uint32_t *sink, void *stream);

/*
 * Record-gather probe: the achievable rate of the traversal's memory access
 * pattern, measured rather than assumed. table: device, n_records records of
 * 64 bytes (16-byte aligned); each of blocks x 256 threads reads `rounds`
 * records (a positive multiple of 4), each as three 16-byte loads of its
 * first 48 bytes, at indices hashed independently per thread and round, so
 * the lanes of a wave diverge as traversal lanes do; four records are in
 * flight per thread. sink: device uint32 [blocks * 256], receives the XOR of
 * what each thread read. Bytes gathered = 48 * rounds * blocks * 256.
 * Errors: RV_ERR_INVALID_ARG (null or misaligned pointers, sizes out of
 * range), RV_ERR_HIP.
 */
rv_status rv_gather_probe(const void *table, int64_t n_records, int32_t rounds, int32_t blocks, uint32_t *sink,
                          void *stream);

/* ------------------------------------------------------------------------ */
/* Adjoint                                                                  */
/* ------------------------------------------------------------------------ */

/*
 * Gradient of L with respect to opacity [n], mean [n][3] and log_scale [n][3],
 * given dL/dvis_ray [n*K] (or NULL) and dL/dvis_mean [n] (or NULL, at least one
 * given). Each ray is traced again in the same order with the same early exit
 * (no hit lists are stored): a first pass recovers the ray's final T (skipped
 * when vis_ray_fwd, the forward's vis_ray, is given), a second pass adds, for
 * every included Gaussian j with alpha_j < alpha_max,
 *   dL/dalpha_j = -g * T / (1 - alpha_j),   g = dL/dT of the ray,
 *   dalpha/do_j = alpha/o_j, dalpha/dmu_j = alpha W_j^T e,
 *   dalpha/dlog_scale_{j,a} = alpha e_a^2, dalpha/dmu_i = -alpha W_j^T e,
 * with W_j = diag(1/s_j) R_j^T and e = p + t* v the whitened closest-approach
 * vector (dq/dt = 0 at the peak, so t* is not differentiated). Cuts and the
 * clamp are not differentiated. Gradients are ACCUMULATED (+=) into the
 * caller's buffers with FP32 atomics: zero them first; the summation order,
 * hence the last bits, may vary between runs.
 * The call takes 256 MB of device scratch, stream-ordered on `stream`
 * (hipMallocAsync, released by hipFreeAsync after its launches), for the hits
 * that overflow each block's on-chip accumulation table; if that allocation
 * fails, those hits are added with atomics at once (same result up to the
 * summation order). Calls on different streams take separate scratch.
 */
rv_status rv_trace_visibility_backward(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                       const rv_trace_params *p, const float *grad_vis_ray,
                                       const float *grad_vis_mean, const float *vis_ray_fwd,
                                       float *grad_opacity, float *grad_mean, float *grad_log_scale,
                                       void *stream);

/* ------------------------------------------------------------------------ */
/* MLP visibility surrogate                                                 */
/* ------------------------------------------------------------------------ */

/*
 * A learned stand-in for tracing the visibility term V of Eq. (9), trained on
 * the tracer's own output, with the tracer as fallback.
 *
 * Network: input x (3, mapped to [-1, 1] by the box lo/hi stored in the
 * parameter blob) and unit direction d (3); each of the 6 scalars u is encoded
 * as [u, sin(2^l pi u), cos(2^l pi u)] for l = 0, 1, 2 (42 features,
 * zero-padded to 64); four hidden layers of 256 with ReLU (64->256, then
 * 3 x 256->256); a 256->2 head giving V = sigmoid(z0) and the predicted
 * absolute error U = z1 (linear). Matrix products run on the gfx950 matrix
 * cores in BF16 (weights and layer inputs rounded to nearest even) with FP32
 * accumulation; biases, nonlinearities, the loss, the master weights and Adam
 * are FP32.
 * Loss per sample: BCE(V, T) + (U - |T - V|)^2 with V held constant in the
 * second term, so that U estimates the mean absolute error of V given the
 * query, by which the fallback ranks queries. Parameters: one flat FP32 vector W1, b1, ..., W5, b5, each W
 * stored [in][out] row-major (rv_surrogate_n_params() = 214,530 floats).
 */
typedef struct rv_train_opts {
    int64_t steps;       /* optimiser steps in this call */
    int32_t batch;       /* samples per step (multiple of 128, <= the workspace's batch) */
    float lr;            /* Adam step size at the start of the schedule */
    float beta1, beta2, eps;
    float lr_min;        /* cosine-decay floor at step total_steps */
    uint64_t seed;       /* sample draw: index = hash(seed, global step, slot) mod n_samples */
    int64_t step0;       /* global index of this call's first step (Adam bias correction, schedule) */
    int64_t total_steps; /* schedule length */
} rv_train_opts;

/* Device pointers into a parameter blob (host-side arithmetic only). */
typedef struct rv_surrogate_arrays {
    float *header;   /* [16]: box lo[3], hi[3], ... */
    float *master;   /* [n_params] FP32 weights */
    float *adam_m;   /* [n_params] */
    float *adam_v;   /* [n_params] */
    void *packed;    /* BF16 copies laid out for the matrix cores */
} rv_surrogate_arrays;

/* Number of FP32 parameters (214,530). */
int64_t rv_surrogate_n_params(void);

/* Bytes of the parameter blob. */
size_t rv_surrogate_bytes(void);

/* rv_surrogate_arrays of a blob (no device access). */
rv_status rv_surrogate_view(const void *params, rv_surrogate_arrays *out);

/* Bytes of training scratch for batches of up to `batch` samples. */
size_t rv_surrogate_train_workspace_bytes(int32_t batch);

/* Bytes of inference scratch for q_count grid queries (counters, fallback list and flags). */
size_t rv_surrogate_infer_workspace_bytes(int64_t q_count);

/*
 * Initialise a blob (256-byte aligned, rv_surrogate_bytes()): the box
 * lo[3]/hi[3] (host floats), the FP32 weights from `init_weights` (device,
 * n_params floats, the flat order above) or, when it is NULL, a seeded
 * He-uniform draw from a counter-based hash of (seed, index) with zero biases;
 * Adam state zero; BF16 copies packed.
 * Errors: RV_ERR_INVALID_ARG (null params or box, params not 256-byte
 * aligned), RV_ERR_HIP (a launch failed).
 */
rv_status rv_surrogate_init(void *params, uint64_t seed, const float *box_lo_host, const float *box_hi_host,
                            const float *init_weights, void *stream);

/*
 * Mean loss (loss_out, device float[1]) and its gradient (grad_out, device
 * float[n_params], overwritten) on samples 0..n-1 of (x [n][3], d [n][3],
 * T [n]); n <= the workspace's batch. Deterministic.
 * Errors: RV_ERR_INVALID_ARG (a null pointer, n outside [1, 2^30], ws not
 * 256-byte aligned), RV_ERR_WORKSPACE (ws_bytes below the training scratch of
 * a batch of n), RV_ERR_HIP.
 */
rv_status rv_surrogate_loss_grad(const void *params, const float *x, const float *d, const float *T, int64_t n,
                                 float *grad_out, float *loss_out, void *ws, size_t ws_bytes, void *stream);

/*
 * o->steps Adam steps on batches drawn from n_samples tracer samples (x [n][3],
 * d [n][3], T [n]). loss_log (device, FP32 [steps]; NULL to skip) receives
 * each step's mean loss.
 * Errors: RV_ERR_INVALID_ARG (a null pointer, n_samples < 1, steps < 0, batch
 * not a positive multiple of 128, lr < 0, beta1 or beta2 outside [0, 1),
 * eps <= 0, ws not 256-byte aligned), RV_ERR_WORKSPACE (ws_bytes below
 * rv_surrogate_train_workspace_bytes(batch)), RV_ERR_HIP.
 */
rv_status rv_surrogate_train(void *params, const float *x, const float *d, const float *T, int64_t n_samples,
                             const rv_train_opts *o, float *loss_log, void *ws, size_t ws_bytes, void *stream);

/*
 * Free-form inference: vis[s], unc[s] (unc may be NULL) for n queries
 * (x[s], d[s]; device [n][3]). n = 0 is a no-op.
 * Errors: RV_ERR_INVALID_ARG (null params or vis, null x or d with n > 0,
 * n < 0), RV_ERR_HIP.
 */
rv_status rv_surrogate_infer_xd(const void *params, const float *x, const float *d, int64_t n, float *vis,
                                float *unc, void *stream);

/*
 * Grid inference over queries q in [q_begin, q_begin + q_count), q = i*K + k
 * (x = mean_i, d = direction k of Gaussian i exactly as rv_trace_visibility
 * forms it). vis[s] receives the surrogate's V, or the tracer's T where the
 * predicted error U exceeds tau and `bvh` is not NULL (fallback; the same bits
 * as rv_trace_rays for that ray). unc (may be NULL) receives U; *n_fallback
 * (device int64) the number of traced queries. Queries are flagged, gathered
 * into a list in `ws` in the BVH's leaf (Morton) order of their Gaussians,
 * and traced by a persistent kernel; ws: 256-byte aligned,
 * rv_surrogate_infer_workspace_bytes(q_count) bytes, not shared by
 * overlapping calls. Deterministic (each query's value does not depend on
 * the list order). q_count = 0 is a no-op.
 * Errors: RV_ERR_INVALID_ARG (a null pointer among params, g, dirs, p, vis;
 * null means or log-scales, n outside [1, RV_MAX_GAUSSIANS], K < 1, dir_mode 1
 * without normals, trace parameters out of range, the query range outside
 * [0, n K), ws missing or unaligned), RV_ERR_WORKSPACE (ws_bytes below
 * rv_surrogate_infer_workspace_bytes(q_count)), RV_ERR_HIP. A bvh built for
 * another Gaussian set is not walked: its fallback queries give NaN.
 */
rv_status rv_surrogate_infer(const void *params, const void *bvh, const rv_gaussians *g, const float *dirs,
                             int32_t K, const rv_trace_params *p, int64_t q_begin, int64_t q_count, float tau,
                             float *vis, float *unc, int64_t *n_fallback, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Origin and unit direction of each listed ray (device, out_o/out_d [n][3]),
 * formed exactly as the tracer forms them: the training inputs of the surrogate.
 * ray_ids (device int64 [n]) hold q = i*K + k. n = 0 is a no-op.
 * Errors: RV_ERR_INVALID_ARG (null g, dirs, p or means; n outside
 * [1, RV_MAX_GAUSSIANS] Gaussians, K < 1 or n < 0 rays; dir_mode 1 without
 * normals; null ids or outputs with n > 0), RV_ERR_HIP.
 */
rv_status rv_ray_setup(const rv_gaussians *g, const float *dirs, int32_t K, const rv_trace_params *p,
                       const int64_t *ray_ids, int64_t n, float *out_o, float *out_d, void *stream);

/* ------------------------------------------------------------------------ */
/* Shading with pre-computed visibility (Sec. 3.3, Eq. (7)-(10))            */
/* ------------------------------------------------------------------------ */

/*
 * Material and light of rv_shade_pbr (device arrays, FP32, contiguous).
 * albedo [n][3] in [0, 1]; roughness [n] in (0, 1] (GGX alpha = r^2);
 * sh [n][9][3]: indirect light as real spherical harmonics of degree <= 2 per
 * colour channel, basis order (0,0), (1,-1), (1,0), (1,1), (2,-2), (2,-1),
 * (2,0), (2,1), (2,2) with the usual orthonormal constants (Y_00 = 1/(2
 * sqrt(pi)), Y_1m = sqrt(3/(4 pi)) (y, z, x), ...); env [16][32][3]: direct
 * light, equirectangular in the world frame with +z up, row 0 at the +z pole,
 * column 0 at azimuth -pi, texel centres at half-integer coordinates,
 * sampled bilinearly (wrapping in azimuth, clamped at the poles); camera:
 * view position, w_o = normalize(camera - mu_i); f0: Fresnel reflectance at
 * normal incidence (0.04 for a dielectric).
 */
typedef struct rv_pbr_material {
    const float *albedo;
    const float *roughness;
    const float *sh;
    const float *env;
    float camera[3];
    float f0;
} rv_pbr_material;

/*
 * PBR colour of every Gaussian from its pre-computed visibility (Eq. (10)
 * with the light of Eq. (9)): color[i] = sum_k (albedo_i / pi + f_s(w_o, w_k))
 * (vis_ray[i][k] L_env(w_k) + L_sh_i(w_k)) max(n_i . w_k, 0) dw, where w_k are
 * the visibility rays' directions (dirs, K, p->dir_mode as for
 * rv_trace_visibility), dw = 2 pi / K (hemisphere) or 4 pi / K (sphere), and
 * f_s = D F G / (4 (n . w_k)(n . w_o)) with GGX D (alpha = roughness^2),
 * Schlick F (f0) and separable Smith G (0 when n . w_o <= 0).
 * vis_ray: [n][K] FP32 (device), as written by rv_trace_visibility.
 * color: [n][3] FP32 (device), overwritten. Normals are required.
 * Errors: RV_ERR_INVALID_ARG (null pointers, n or K out of range, bad
 * dir_mode, f0 outside [0, 1], a camera coordinate that is not finite),
 * RV_ERR_HIP.
 */
rv_status rv_shade_pbr(const rv_gaussians *g, const float *dirs, int32_t K, const rv_trace_params *p,
                       const float *vis_ray, const rv_pbr_material *m, float *color, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RVIS_H */
