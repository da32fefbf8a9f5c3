// trace.hip -- visibility pre-computation (Sec. 4.2): for every Gaussian i and
// direction k, the transmittance of the ray leaving mean_i (Sec. 4.1), and the
// per-Gaussian average over the K directions (the "averaged visibility" of the
// ablation study, Sec. 5.4).
//
// Work mapping: one lane per Gaussian in Morton (sorted-leaf) order, so a wave
// holds 64 spatially adjacent origins whose rays share most of the tree. Each
// lane walks its K rays one node per loop iteration and starts its next ray as
// soon as the current one ends, so lanes never wait on each other's rays; the
// per-Gaussian mean is accumulated in a register (FP64) and needs no atomics.
#include "trace_core.h"

namespace rv {
namespace {

constexpr int kTraceBlock = 256;
constexpr int kRing = 16;

struct Origin {
    f3 o, nrm, b1, b2;
    float tmin;
    int32_t src;
};

__device__ __forceinline__ Origin load_origin(const float4 *__restrict__ rec, const float4 *__restrict__ origins,
                                              int64_t m, const Cuts &c) {
    Origin g;
    const float4 r0 = rec[4 * m];
    const float4 og = origins[m];
    g.src = __float_as_int(rec[4 * m + 1].w);
    g.o = mk(r0.x, r0.y, r0.z);
    g.nrm = mk(og.x, og.y, og.z);
    g.tmin = c.tmin_scale * og.w;
    onb_duff(g.nrm, g.b1, g.b2);
    return g;
}

template <bool kCount>
__global__ __launch_bounds__(kTraceBlock) void k_trace_origins(const float4 *__restrict__ nodes,
                                                               const float4 *__restrict__ rec,
                                                               const float4 *__restrict__ origins, int64_t n,
                                                               const float *__restrict__ dirs, int K, Cuts c,
                                                               float *__restrict__ vis_ray,
                                                               float *__restrict__ vis_mean,
                                                               unsigned long long *__restrict__ totals) {
    __shared__ int32_t lds[kRing * kTraceBlock];
    const int64_t m = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
    if (m >= n) return;
    const Origin g = load_origin(rec, origins, m, c);
    RayState<kRing> rs;
    rs.st.lds = lds + threadIdx.x;
    rs.st.stride = kTraceBlock;
    NoHit none;
    int64_t cn = 0, cl = 0, ch = 0;
    double sum = 0.0;
    int k = 0;
    rs.start(g.o, ray_direction(dirs, 0, c.dir_mode, g.nrm, g.b1, g.b2), g.tmin, g.src, n);
    while (true) {
        const bool done = rs.node < 0 || rs.template step<NoHit, kCount>(nodes, rec, c, none, &cn, &cl, &ch);
        if (done) {
            if (vis_ray) vis_ray[(int64_t)g.src * K + k] = rs.T;
            sum += (double)rs.T;
            if (++k == K) break;
            rs.start(g.o, ray_direction(dirs, k, c.dir_mode, g.nrm, g.b1, g.b2), g.tmin, g.src, n);
        }
    }
    if (vis_mean) vis_mean[g.src] = (float)(sum / (double)K);
    if (kCount) {
        atomicAdd(totals + 0, (unsigned long long)cn);
        atomicAdd(totals + 1, (unsigned long long)cl);
        atomicAdd(totals + 2, (unsigned long long)ch);
    }
}

// One lane per listed ray; origin data recomputed from the input arrays with
// the same operations as the leaf preparation, so results match bit for bit.
__global__ __launch_bounds__(kTraceBlock) void k_trace_list(const float4 *__restrict__ nodes,
                                                            const float4 *__restrict__ rec,
                                                            const float *__restrict__ mean,
                                                            const float *__restrict__ normal,
                                                            const float *__restrict__ log_scale, int64_t n,
                                                            const float *__restrict__ dirs, int K, Cuts c,
                                                            const int64_t *__restrict__ ids, int64_t n_rays,
                                                            float *__restrict__ out) {
    __shared__ int32_t lds[kRing * kTraceBlock];
    const int64_t s = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
    if (s >= n_rays) return;
    const int64_t r = ids[s];
    if (r < 0 || r >= n * (int64_t)K) {  // not a ray of this scene
        out[s] = __int_as_float(0x7fc00000);
        return;
    }
    const int64_t i = r / K;
    const int k = (int)(r - i * K);
    float nx = 0.f, ny = 0.f, nz = 1.f;
    if (normal) {
        nx = normal[3 * i]; ny = normal[3 * i + 1]; nz = normal[3 * i + 2];
        const float nl = sqrtf(nx * nx + ny * ny + nz * nz);
        nx /= nl; ny /= nl; nz /= nl;
    }
    const float smax = expf(fmaxf(log_scale[3 * i], fmaxf(log_scale[3 * i + 1], log_scale[3 * i + 2])));
    const f3 nrm = mk(nx, ny, nz);
    f3 b1, b2;
    onb_duff(nrm, b1, b2);
    RayState<kRing> rs;
    rs.st.lds = lds + threadIdx.x;
    rs.st.stride = kTraceBlock;
    NoHit none;
    rs.start(mk(mean[3 * i], mean[3 * i + 1], mean[3 * i + 2]), ray_direction(dirs, k, c.dir_mode, nrm, b1, b2),
             c.tmin_scale * smax, (int32_t)i, n);
    while (rs.node >= 0 && !rs.step(nodes, rec, c, none)) {
    }
    out[s] = rs.T;
}

// ---- adjoint ----------------------------------------------------------------

struct GradScatter {
    float g_over;       // -(dL/dT) * T_final for the current ray
    float *go, *gm, *gl;
    f3 origin;          // accumulated d/d(origin), flushed once per Gaussian

    __device__ __forceinline__ void operator()(const LeafHit &h, float) {
        if (h.clamped) return;
        const float ga = g_over / (1.0f - h.alpha);   // dL/dalpha
        const float a = ga * h.alpha;
        const f3 wte = h.e.x * h.w0 + h.e.y * h.w1 + h.e.z * h.w2;   // W^T e
        const int64_t j = h.src;
        unsafeAtomicAdd(go + j, a / h.opacity);
        unsafeAtomicAdd(gm + 3 * j + 0, a * wte.x);
        unsafeAtomicAdd(gm + 3 * j + 1, a * wte.y);
        unsafeAtomicAdd(gm + 3 * j + 2, a * wte.z);
        unsafeAtomicAdd(gl + 3 * j + 0, a * h.e.x * h.e.x);
        unsafeAtomicAdd(gl + 3 * j + 1, a * h.e.y * h.e.y);
        unsafeAtomicAdd(gl + 3 * j + 2, a * h.e.z * h.e.z);
        origin = origin - a * wte;
    }
};

__global__ __launch_bounds__(kTraceBlock) void k_trace_backward(
    const float4 *__restrict__ nodes, const float4 *__restrict__ rec, const float4 *__restrict__ origins, int64_t n,
    const float *__restrict__ dirs, int K, Cuts c, const float *__restrict__ grad_ray,
    const float *__restrict__ grad_mean_in, const float *__restrict__ vis_fwd, float *go, float *gm, float *gl) {
    __shared__ int32_t lds[kRing * kTraceBlock];
    const int64_t m = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
    if (m >= n) return;
    const Origin g = load_origin(rec, origins, m, c);
    RayState<kRing> rs;
    rs.st.lds = lds + threadIdx.x;
    rs.st.stride = kTraceBlock;
    NoHit none;
    GradScatter gs;
    gs.go = go;
    gs.gm = gm;
    gs.gl = gl;
    gs.origin = mk(0.f, 0.f, 0.f);
    const float gmean = grad_mean_in ? grad_mean_in[g.src] / (float)K : 0.0f;
    int k = 0;
    int phase = 0;
    float gk = 0.0f;
    // find the first ray with a nonzero upstream gradient
    auto begin_ray = [&](int kk) -> bool {
        for (; kk < K; ++kk) {
            gk = gmean + (grad_ray ? grad_ray[(int64_t)g.src * K + kk] : 0.0f);
            if (gk != 0.0f) break;
        }
        k = kk;
        if (k >= K) return false;
        rs.start(g.o, ray_direction(dirs, k, c.dir_mode, g.nrm, g.b1, g.b2), g.tmin, g.src, n);
        if (vis_fwd) {
            phase = 1;
            gs.g_over = -gk * vis_fwd[(int64_t)g.src * K + k];
        } else {
            phase = 0;
        }
        return true;
    };
    bool live = begin_ray(0);
    while (live) {
        bool done;
        if (phase == 0) {
            done = rs.node < 0 || rs.step(nodes, rec, c, none);
            if (done) {
                gs.g_over = -gk * rs.T;
                rs.start(rs.o, rs.d, rs.tmin, rs.self, n);
                phase = 1;
            }
        } else {
            done = rs.node < 0 || rs.step(nodes, rec, c, gs);
            if (done) live = begin_ray(k + 1);
        }
    }
    if (gs.origin.x != 0.f || gs.origin.y != 0.f || gs.origin.z != 0.f) {
        unsafeAtomicAdd(gm + 3 * (int64_t)g.src + 0, gs.origin.x);
        unsafeAtomicAdd(gm + 3 * (int64_t)g.src + 1, gs.origin.y);
        unsafeAtomicAdd(gm + 3 * (int64_t)g.src + 2, gs.origin.z);
    }
}

__global__ __launch_bounds__(64) void k_fill_u32_trace(uint32_t *__restrict__ p, int64_t count, uint32_t v) {
    for (int64_t i = threadIdx.x; i < count; i += 64) p[i] = v;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

rv_status validate_trace(const char *fn, const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                         const rv_trace_params *p) {
    RV_REQUIRE(bvh && g && dirs && p, RV_ERR_INVALID_ARG, "%s: null argument (bvh, g, dirs or params)", fn);
    RV_REQUIRE(g->mean && g->log_scale, RV_ERR_INVALID_ARG, "%s: null Gaussian mean/log_scale", fn);
    RV_REQUIRE(g->n >= 1 && g->n <= RV_MAX_GAUSSIANS, RV_ERR_INVALID_ARG, "%s: n=%lld out of range", fn,
               (long long)g->n);
    RV_REQUIRE(K >= 1, RV_ERR_INVALID_ARG, "%s: K=%d must be >= 1", fn, K);
    RV_REQUIRE(p->dir_mode == 0 || p->dir_mode == 1, RV_ERR_INVALID_ARG, "%s: dir_mode must be 0 or 1", fn);
    RV_REQUIRE(p->dir_mode == 0 || g->normal, RV_ERR_INVALID_ARG, "%s: hemisphere mode needs normals", fn);
    RV_REQUIRE(p->sigma_cut > 0.0f && p->sigma_cut <= kBuildSigma, RV_ERR_INVALID_ARG,
               "%s: sigma_cut must be in (0, %g] (the BVH boxes cover 3 sigma)", fn, (double)kBuildSigma);
    RV_REQUIRE(p->alpha_min > 0.0f && p->alpha_max < 1.0f && p->alpha_min <= p->alpha_max, RV_ERR_INVALID_ARG,
               "%s: need 0 < alpha_min <= alpha_max < 1", fn);
    RV_REQUIRE(p->T_min >= 0.0f && p->T_min < 1.0f && p->tmin_scale >= 0.0f, RV_ERR_INVALID_ARG,
               "%s: need 0 <= T_min < 1 and tmin_scale >= 0", fn);
    return RV_OK;
}

}  // namespace
}  // namespace rv

using namespace rv;

extern "C" size_t rv_trace_workspace_bytes(int64_t n, int32_t K) {
    (void)n;
    (void)K;
    return kAlign;
}

extern "C" rv_status rv_trace_visibility(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                         const rv_trace_params *p, float *vis_ray, float *vis_mean, void *ws,
                                         size_t ws_bytes, void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_visibility", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(vis_ray || vis_mean, RV_ERR_INVALID_ARG, "rv_trace_visibility: both outputs are NULL");
    (void)ws;
    (void)ws_bytes;
    const BvhLayout L = bvh_layout(g->n);
    const Cuts c = make_cuts(*p);
    hipLaunchKernelGGL(k_trace_origins<false>, dim3(grid_for(g->n, kTraceBlock)), dim3(kTraceBlock), 0,
                       (hipStream_t)stream, at<float4>(bvh, L.nodes), at<float4>(bvh, L.leaf_rec),
                       at<float4>(bvh, L.origins), g->n, dirs, K, c, vis_ray, vis_mean,
                       (unsigned long long *)nullptr);
    return check_launch("rv_trace_visibility");
}

extern "C" rv_status rv_trace_stats(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                    const rv_trace_params *p, int64_t *totals, void *ws, size_t ws_bytes,
                                    void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_stats", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(totals, RV_ERR_INVALID_ARG, "rv_trace_stats: null totals");
    (void)ws;
    (void)ws_bytes;
    const BvhLayout L = bvh_layout(g->n);
    const Cuts c = make_cuts(*p);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_u32_trace, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(totals), (int64_t)6,
                       0u);
    hipLaunchKernelGGL(k_trace_origins<true>, dim3(grid_for(g->n, kTraceBlock)), dim3(kTraceBlock), 0, s,
                       at<float4>(bvh, L.nodes), at<float4>(bvh, L.leaf_rec), at<float4>(bvh, L.origins), g->n,
                       dirs, K, c, (float *)nullptr, (float *)nullptr, (unsigned long long *)totals);
    return check_launch("rv_trace_stats");
}

extern "C" rv_status rv_trace_rays(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                   const rv_trace_params *p, const int64_t *ray_ids, int64_t n_rays, float *out,
                                   void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_rays", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(n_rays >= 0, RV_ERR_INVALID_ARG, "rv_trace_rays: n_rays < 0");
    if (n_rays == 0) return RV_OK;
    RV_REQUIRE(ray_ids && out, RV_ERR_INVALID_ARG, "rv_trace_rays: null ray_ids or out");
    const BvhLayout L = bvh_layout(g->n);
    const Cuts c = make_cuts(*p);
    hipLaunchKernelGGL(k_trace_list, dim3(grid_for(n_rays, kTraceBlock)), dim3(kTraceBlock), 0, (hipStream_t)stream,
                       at<float4>(bvh, L.nodes), at<float4>(bvh, L.leaf_rec), g->mean, p->dir_mode ? g->normal : nullptr,
                       g->log_scale, g->n, dirs, K, c, ray_ids, n_rays, out);
    return check_launch("rv_trace_rays");
}

extern "C" rv_status rv_trace_visibility_backward(const void *bvh, const rv_gaussians *g, const float *dirs,
                                                  int32_t K, const rv_trace_params *p, const float *grad_vis_ray,
                                                  const float *grad_vis_mean, const float *vis_ray_fwd,
                                                  float *grad_opacity, float *grad_mean, float *grad_log_scale,
                                                  void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_visibility_backward", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(grad_vis_ray || grad_vis_mean, RV_ERR_INVALID_ARG,
               "rv_trace_visibility_backward: both upstream gradients are NULL");
    RV_REQUIRE(grad_opacity && grad_mean && grad_log_scale, RV_ERR_INVALID_ARG,
               "rv_trace_visibility_backward: null gradient output");
    const BvhLayout L = bvh_layout(g->n);
    const Cuts c = make_cuts(*p);
    hipLaunchKernelGGL(k_trace_backward, dim3(grid_for(g->n, kTraceBlock)), dim3(kTraceBlock), 0,
                       (hipStream_t)stream, at<float4>(bvh, L.nodes), at<float4>(bvh, L.leaf_rec),
                       at<float4>(bvh, L.origins), g->n, dirs, K, c, grad_vis_ray, grad_vis_mean, vis_ray_fwd,
                       grad_opacity, grad_mean, grad_log_scale);
    return check_launch("rv_trace_visibility_backward");
}
