// shade.hip -- per-Gaussian physically based shading with pre-computed
// visibility (Sec. 3.3, Eq. (7)-(10)): for Gaussian i and its K incident
// directions w_k (the visibility rays' directions, Sec. 3.3 and 4.2)
//
//   c_i = sum_k (b / pi + f_s(w_o, w_k)) (V_ik L_env(w_k) + sum_j l_j Y_j(w_k)) max(n . w_k, 0) dw
//
// with f_s = D F G / (4 (n . w_k)(n . w_o)) (GGX D with alpha = r^2, Schlick F,
// separable Smith G), the 16 x 32 environment map sampled bilinearly, the
// indirect light as real SH of degree <= 2, and dw = 2 pi / K (4 pi / K on the
// sphere).
//
// Mapping: one wave per Gaussian, lanes striding over the directions; the
// Gaussian's parameters are wave-uniform, the map sits in LDS, and the three
// colour sums end with a wave reduction.
#include <cmath>

#include "trace_core.h"

namespace rv {
namespace {

constexpr int kEnvRows = 16, kEnvCols = 32;
constexpr int kShadeBlock = 256;
constexpr float kPi = 3.14159265358979323846f;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// atan2(y, x) in binary32: t = min(|x|, |y|) / max(|x|, |y|) in [0, 1] by the
// hardware reciprocal, atan(t) = t P(t^2) with P of degree 7 fitted to atan on
// [0, 1] (least squares on Chebyshev nodes, reweighted toward the largest
// errors; at most 1.3e-7 rad evaluated in binary32 by Horner's rule), then the
// octant and the quadrant from |y| > |x| and the signs.
__device__ __forceinline__ float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float u = t * t;
    float p = -0.004054537042975426f;
    p = fmaf(p, u, 0.021862857043743134f);
    p = fmaf(p, u, -0.05591219663619995f);
    p = fmaf(p, u, 0.09642188996076584f);
    p = fmaf(p, u, -0.1390862613916397f);
    p = fmaf(p, u, 0.19946564733982086f);
    p = fmaf(p, u, -0.33329859375953674f);
    p = fmaf(p, u, 0.9999993443489075f);
    float r = t * p;
    if (ay > ax) r = 1.5707963267948966f - r;
    if (x < 0.0f) r = 3.141592653589793f - r;
    return y < 0.0f ? -r : r;
}

__global__ __launch_bounds__(kShadeBlock) void k_shade(const float *__restrict__ mean, const float *__restrict__ normal,
                                                       int64_t n, const float *__restrict__ dirs, int K, int dir_mode,
                                                       const float *__restrict__ vis, const float *__restrict__ albedo,
                                                       const float *__restrict__ roughness,
                                                       const float *__restrict__ sh, const float *__restrict__ env,
                                                       float cx, float cy, float cz, float f0, int64_t i_off,
                                                       float *__restrict__ color) {
    __shared__ float env_s[kEnvRows * kEnvCols * 3];
    for (int t = threadIdx.x; t < kEnvRows * kEnvCols * 3; t += kShadeBlock) env_s[t] = env[t];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t i = i_off + (int64_t)__builtin_amdgcn_readfirstlane(blockIdx.x) * (kShadeBlock / 64) +
                      __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;  // wave-uniform

    // the Gaussian: normal frame as the visibility rays use it, view direction
    float nx = normal[3 * i], ny = normal[3 * i + 1], nz = normal[3 * i + 2];
    const float nl = sqrtf(nx * nx + ny * ny + nz * nz);
    nx /= nl; ny /= nl; nz /= nl;
    const f3 nrm = mk(nx, ny, nz);
    f3 b1, b2;
    onb_duff(nrm, b1, b2);
    f3 wo = mk(cx - mean[3 * i], cy - mean[3 * i + 1], cz - mean[3 * i + 2]);
    wo = (1.0f / sqrtf(dot(wo, wo))) * wo;
    const float no = dot(nrm, wo);
    const float r = roughness[i];
    const float a2 = (r * r) * (r * r);
    const float g1o = no > 0.0f ? 2.0f * no / (no + sqrtf(a2 + (1.0f - a2) * no * no)) : 0.0f;
    // per-Gaussian factor of the specular term: G1(w_o) / (4 pi (n . w_o)) times alpha^2
    const float spec_k = no > 0.0f ? g1o * a2 / (4.0f * kPi * no) : 0.0f;
    const float kd0 = albedo[3 * i] * (1.0f / kPi), kd1 = albedo[3 * i + 1] * (1.0f / kPi),
                kd2 = albedo[3 * i + 2] * (1.0f / kPi);
    float l[9][3];
#pragma unroll
    for (int j = 0; j < 9; ++j)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) l[j][ch] = sh[(i * 9 + j) * 3 + ch];
    const float dw = (dir_mode ? 2.0f : 4.0f) * kPi / (float)K;

    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    for (int k = lane; k < K; k += 64) {
        const f3 w = ray_direction(dirs, k, dir_mode, nrm, b1, b2);
        const float ci = dot(nrm, w);
        if (!(ci > 0.0f)) continue;
        // environment: bilinear at texel coordinates of (theta, phi)
        const float rho = sqrtf(w.x * w.x + w.y * w.y);
        const float theta = atan2_poly(rho, w.z), phi = atan2_poly(w.y, w.x);
        const float u = (phi + kPi) * ((float)kEnvCols / (2.0f * kPi)) - 0.5f;
        const float v = theta * ((float)kEnvRows / kPi) - 0.5f;
        const float uf = floorf(u), vf = floorf(v);
        const float fu = u - uf, fv = v - vf;
        // u lies in [-0.5, 31.5): the left texel column is -1 (wraps to 31) .. 31
        const int c0 = uf < 0.0f ? kEnvCols - 1 : (int)uf;
        const int c1 = c0 + 1 == kEnvCols ? 0 : c0 + 1;
        const int ra = min(max((int)vf, 0), kEnvRows - 1), rb = min(max((int)vf + 1, 0), kEnvRows - 1);
        float Le[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float top = (1.0f - fu) * env_s[(ra * kEnvCols + c0) * 3 + ch] + fu * env_s[(ra * kEnvCols + c1) * 3 + ch];
            const float bot = (1.0f - fu) * env_s[(rb * kEnvCols + c0) * 3 + ch] + fu * env_s[(rb * kEnvCols + c1) * 3 + ch];
            Le[ch] = (1.0f - fv) * top + fv * bot;
        }
        // indirect light: real SH of degree <= 2
        const float Y[9] = {0.28209479177387814f, 0.4886025119029199f * w.y, 0.4886025119029199f * w.z,
                            0.4886025119029199f * w.x, 1.0925484305920792f * w.x * w.y,
                            1.0925484305920792f * w.y * w.z, 0.31539156525252005f * (3.0f * w.z * w.z - 1.0f),
                            1.0925484305920792f * w.x * w.z, 0.5462742152960396f * (w.x * w.x - w.y * w.y)};
        float Li[3];
        const float V = vis[i * K + k];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < 9; ++j) s = fmaf(l[j][ch], Y[j], s);
            Li[ch] = V * Le[ch] + s;
        }
        // specular times the cosine: D F G / (4 (n . w_o)); the GGX denominator
        // uses 1 - (n.h)^2 = |n x h|^2 to stay accurate for smooth surfaces.
        // Hardware reciprocals (about 1 ulp) for the BRDF's quotients.
        float spec = 0.0f;
        if (no > 0.0f) {
            f3 h = w + wo;
            h = __builtin_amdgcn_rsqf(dot(h, h)) * h;
            const float nh = fmaxf(dot(nrm, h), 0.0f), vh = fmaxf(dot(wo, h), 0.0f);
            const f3 nxh = cross(nrm, h);
            const float t = dot(nxh, nxh) + nh * nh * a2;
            const float m = 1.0f - vh, m2 = m * m;
            const float F = f0 + (1.0f - f0) * (m2 * m2 * m);
            const float g1i_over_2ci = __builtin_amdgcn_rcpf(ci + sqrtf(a2 + (1.0f - a2) * ci * ci));
            // D F G1(w_i) G1(w_o) / (4 n.w_o) with D = alpha^2 / (pi t^2)
            spec = spec_k * F * (2.0f * ci * g1i_over_2ci) * __builtin_amdgcn_rcpf(t * t);
        }
        acc0 = fmaf((kd0 * ci + spec) * Li[0], dw, acc0);
        acc1 = fmaf((kd1 * ci + spec) * Li[1], dw, acc1);
        acc2 = fmaf((kd2 * ci + spec) * Li[2], dw, acc2);
    }
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    acc2 = wave_sum(acc2);
    if (lane == 0) {
        color[3 * i] = acc0;
        color[3 * i + 1] = acc1;
        color[3 * i + 2] = acc2;
    }
}

}  // namespace
}  // namespace rv

using namespace rv;

extern "C" rv_status rv_shade_pbr(const rv_gaussians *g, const float *dirs, int32_t K, const rv_trace_params *p,
                                  const float *vis_ray, const rv_pbr_material *m, float *color, void *stream) {
    clear_error();
    RV_REQUIRE(g && dirs && p && vis_ray && m && color, RV_ERR_INVALID_ARG, "rv_shade_pbr: null argument");
    RV_REQUIRE(g->mean && g->normal, RV_ERR_INVALID_ARG, "rv_shade_pbr: needs means and normals");
    RV_REQUIRE(m->albedo && m->roughness && m->sh && m->env, RV_ERR_INVALID_ARG, "rv_shade_pbr: null material array");
    RV_REQUIRE(g->n >= 1 && g->n <= RV_MAX_GAUSSIANS, RV_ERR_INVALID_ARG, "rv_shade_pbr: n=%lld out of range",
               (long long)g->n);
    RV_REQUIRE(K >= 1, RV_ERR_INVALID_ARG, "rv_shade_pbr: K=%d must be >= 1", K);
    RV_REQUIRE(p->dir_mode == 0 || p->dir_mode == 1, RV_ERR_INVALID_ARG, "rv_shade_pbr: dir_mode must be 0 or 1");
    RV_REQUIRE(m->f0 >= 0.0f && m->f0 <= 1.0f, RV_ERR_INVALID_ARG, "rv_shade_pbr: f0 must lie in [0, 1]");
    RV_REQUIRE(std::isfinite(m->camera[0]) && std::isfinite(m->camera[1]) && std::isfinite(m->camera[2]),
               RV_ERR_INVALID_ARG, "rv_shade_pbr: camera position is not finite");
    // one wave per Gaussian, at most 2^24 waves (2^30 work-items) per grid
    const int64_t waves_per_block = kShadeBlock / 64, per_launch = int64_t(1) << 24;
    for (int64_t i0 = 0; i0 < g->n; i0 += per_launch) {
        const int64_t cnt = std::min(per_launch, g->n - i0);
        hipLaunchKernelGGL(k_shade, dim3((unsigned)((cnt + waves_per_block - 1) / waves_per_block)), dim3(kShadeBlock),
                           0, (hipStream_t)stream, g->mean, g->normal, g->n, dirs, (int)K, (int)p->dir_mode, vis_ray,
                           m->albedo, m->roughness, m->sh, m->env, m->camera[0], m->camera[1], m->camera[2], m->f0, i0,
                           color);
    }
    return check_launch("rv_shade_pbr");
}
