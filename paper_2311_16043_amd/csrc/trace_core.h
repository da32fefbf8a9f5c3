// trace_core.h -- per-lane all-hit BVH traversal of one ray through 3D
// Gaussians (Sec. 4.1): starting at the root, test the children's boxes,
// descend into the hit ones, and at each leaf evaluate the Gaussian at its
// equivalent intersection point (Eq. (13), peak parameter Eq. (14) with
// Sigma^-1) and attenuate T by (1 - alpha) (Eq. (15)); stop early once
// T < T_min. The tree is walked through its compressed four-wide records
// (each internal node lists its grandchildren). The order of hits does not
// change the full product (Sec. 4.1), so children are taken in slot order
// without sorting by distance.
#pragma once

#include "rv_internal.h"

namespace rv {

// Deepest possible root-to-leaf path: each level consumes at least one bit of
// the 95-bit augmented key (63-bit Morton key + 32-bit position).
constexpr int kMaxDepth = 96;
// Stack bound of the four-wide walk: at most 48 wide levels on a path, each
// leaving at most three siblings on the stack.
constexpr int kMaxStack = 3 * (kMaxDepth / 2);

// Idle lanes that trigger the refill of a wave in the pooled traversals
// (unless no lane holds a ray). Waiting for several idle lanes runs the ray
// setup for many lanes at once at the price of a few lanes of traversal; the
// best count grows with the tree: 12 measured best at 300k and 1.2M Gaussians
// (16 equal at 1.2M, 20 slower at both), 20 at 3M (2.5 % faster than 12).
constexpr int kRefillShallow = 12, kRefillDeep = 20;
constexpr int64_t kDeepTreeGaussians = int64_t(2) << 20;
inline int refill_lanes(int64_t n) { return n >= kDeepTreeGaussians ? kRefillDeep : kRefillShallow; }

struct Cuts {
    float alpha_min, alpha_max, T_stop, q_cut, tmin_scale;
    int dir_mode;
    int refill;   // idle lanes before a refill (refill_lanes of the tree's size)
};

inline Cuts make_cuts(const rv_trace_params &p) {
    Cuts c;
    c.alpha_min = p.alpha_min;
    c.alpha_max = p.alpha_max;
    c.T_stop = p.T_min;
    c.q_cut = p.sigma_cut * p.sigma_cut;
    c.tmin_scale = p.tmin_scale;
    c.dir_mode = p.dir_mode;
    c.refill = kRefillShallow;
    return c;
}

// Orthonormal basis (b1, b2) completing the unit normal n: Duff et al.,
// "Building an Orthonormal Basis, Revisited" (JCGT 2017).
__device__ __forceinline__ void onb_duff(f3 n, f3 &b1, f3 &b2) {
    const float sign = copysignf(1.0f, n.z);
    const float a = -__builtin_amdgcn_rcpf(sign + n.z);  // |sign + n.z| in [1, 2]; one ulp
    const float b = n.x * n.y * a;
    b1 = mk(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    b2 = mk(b, sign + n.y * n.y * a, -n.y);
}

// Direction k: world frame (mode 0) or local frame about n (mode 1), unit length.
__device__ __forceinline__ f3 ray_direction(const float *__restrict__ dirs, int k, int mode, f3 n, f3 b1, f3 b2) {
    const float dx = dirs[3 * k], dy = dirs[3 * k + 1], dz = dirs[3 * k + 2];
    f3 d = mode ? (dx * b1 + dy * b2 + dz * n) : mk(dx, dy, dz);
    const float inv = __builtin_amdgcn_rsqf(dot(d, d));  // one ulp; |d| is 1 up to rounding
    return inv * d;
}

// Reciprocal direction (hardware reciprocal, within one ulp) with zero
// components replaced by a tiny signed value, so every component is finite,
// nonzero and carries the sign of d.
__device__ __forceinline__ f3 safe_inv(f3 d) {
    auto r = [](float x) {
        const float tiny = 1e-30f;
        float y = fabsf(x) < tiny ? copysignf(tiny, x) : x;
        return __builtin_amdgcn_rcpf(y);
    };
    return mk(r(d.x), r(d.y), r(d.z));
}

// Children of compressed four-wide node `node` whose boxes the ray segment
// [t0, inf) enters, in slot order; missed and unused slots come out as
// kEmptyChild. A box plane is P = O_a + q step_a (q one byte), so its ray
// distance is fma(q, step_a inv_a, (O_a - o_a) inv_a) with inv_a the
// reciprocal of d_a to within one ulp; step_a inv_a is exact (a power-of-two
// scaling). The roundings of inv_a (2^-23 relative), of O_a - o_a, of the
// product and of the fma (2^-24 each) move a plane by at most
// 2^-23 (1.5 |P - o| + |O - o|) <= 5 2^-23 max|coordinate| in space, which
// is below the outward margin eta >= 2^-20 (max|coordinate| + 1) that the
// builder added to every plane. So a box the exact ray enters beyond t0 is
// never rejected, and no further enlargement of the exit distance is needed.
// The fma is monotone in q, rising for inv_a > 0 and falling for inv_a < 0,
// so the entry plane of each axis is the low one for a positive direction
// component and the high one otherwise: the plane bytes are swapped once per
// node by the direction's signs instead of ordering every pair of distances.
__device__ __forceinline__ void visit4(const float4 *__restrict__ nodes4, int32_t node, f3 o, f3 inv, float t0,
                                       int32_t (&id)[4]) {
    const uint4 *r = reinterpret_cast<const uint4 *>(nodes4) + 4 * (int64_t)node;
    const uint4 w0 = r[0], w1 = r[1], w2 = r[2];
    const uint32_t meta = w0.w;
    const float ax = __uint_as_float((meta & 0xffu) << 23) * inv.x;
    const float ay = __uint_as_float(((meta >> 8) & 0xffu) << 23) * inv.y;
    const float az = __uint_as_float(((meta >> 16) & 0xffu) << 23) * inv.z;
    const float bx = (__uint_as_float(w0.x) - o.x) * inv.x;
    const float by = (__uint_as_float(w0.y) - o.y) * inv.y;
    const float bz = (__uint_as_float(w0.z) - o.z) * inv.z;
    // all ones where the direction component is negative
    const uint32_t mx = (uint32_t)(__float_as_int(inv.x) >> 31), my = (uint32_t)(__float_as_int(inv.y) >> 31),
                   mz = (uint32_t)(__float_as_int(inv.z) >> 31);
    // entry (near) and exit (far) plane bytes of the four slots per axis
    const uint32_t nx = (w1.x & ~mx) | (w1.w & mx), fx = (w1.w & ~mx) | (w1.x & mx);
    const uint32_t ny = (w1.y & ~my) | (w2.x & my), fy = (w2.x & ~my) | (w1.y & my);
    const uint32_t nz = (w1.z & ~mz) | (w2.y & mz), fz = (w2.y & ~mz) | (w1.z & mz);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        auto q = [j](uint32_t w) { return (float)((w >> (8 * j)) & 0xffu); };
        const float tn = fmaxf(fmaxf(fmaf(q(nx), ax, bx), fmaf(q(ny), ay, by)), fmaxf(fmaf(q(nz), az, bz), t0));
        const float tf = fminf(fminf(fmaf(q(fx), ax, bx), fmaf(q(fy), ay, by)), fmaf(q(fz), az, bz));
        // kind bits: bit 0 slot used, bit 1 leaf (~index); slots 0 and 2
        // always hold a child (the first child of each side)
        const bool used = (j & 1) == 0 || ((meta >> (24 + 2 * j)) & 1u);
        const int32_t leaf_mask = -(int32_t)((meta >> (25 + 2 * j)) & 1u);
        const int32_t idx = (int32_t)(j < 2 ? w2.z : w2.w) + (j & 1);
        id[j] = used && tn <= tf ? (idx ^ leaf_mask) : kEmptyChild;
    }
}

__device__ __forceinline__ bool is_leaf(int32_t id) { return id < 0 && id != kEmptyChild; }

// What a leaf test hands to a hit callback.
struct LeafHit {
    float alpha;     // unclamped alpha = o exp(-q/2)
    float one_minus; // the factor applied to T: 1 - min(alpha, alpha_max)
    bool clamped;    // alpha >= alpha_max (contribution used min(alpha, alpha_max))
    float opacity;
    int32_t src;     // original index of the Gaussian
    f3 e;            // whitened closest-approach vector p + t* v (|e|^2 = q)
    f3 w0, w1, w2;   // rows of W
};

struct NoHit {
    __device__ __forceinline__ void operator()(const LeafHit &, float) const {}
};

// e^x - 1 for x in [-1/4, 0] from its Taylor series through x^7 (the
// remainder x^8 / 8! is below 2e-9 of the result there), evaluated in
// Horner form; unlike e^x - 1 it keeps full relative precision as x -> 0.
__device__ __forceinline__ float expm1_small(float x) {
    float r = 1.0f / 5040.0f;
    r = fmaf(r, x, 1.0f / 720.0f);
    r = fmaf(r, x, 1.0f / 120.0f);
    r = fmaf(r, x, 1.0f / 24.0f);
    r = fmaf(r, x, 1.0f / 6.0f);
    r = fmaf(r, x, 0.5f);
    r = fmaf(r, x, 1.0f);
    return r * x;
}

// Evaluate leaf m for the ray (o, d) of source `self`. Returns the factor
// (1 - alpha) to multiply into T (1 when excluded); calls on_hit for included
// Gaussians with the running T before this factor. Branch-free up to the
// final decision, so the record's three rows are fetched together.
template <class OnHit>
__device__ __forceinline__ float leaf_factor(const float4 *__restrict__ rec, int32_t m, f3 o, f3 d, float tmin,
                                             int32_t self, int32_t self_leaf, const Cuts &c, OnHit &on_hit,
                                             float T_before) {
    if (m == self_leaf) return 1.0f;   // the source's own leaf, known by sorted position
    const float4 r0 = rec[kLeafF4 * m + 0];
    const float4 r1 = rec[kLeafF4 * m + 1];
    const float4 r2 = rec[kLeafF4 * m + 2];
    const int32_t src = __float_as_int(r2.w);
    const f3 w0 = mk(r1.x, r1.y, r1.z), w1 = mk(r2.x, r2.y, r2.z);
    const f3 w2 = r1.w * cross(w0, w1);
    const f3 x = o - mk(r0.x, r0.y, r0.z);
    const f3 p = mk(dot(w0, x), dot(w1, x), dot(w2, x));
    const f3 v = mk(dot(w0, d), dot(w1, d), dot(w2, d));
    const float vv = dot(v, v);
    const float pv = dot(p, v);
    const f3 cp = cross(p, v);
    const float cc = dot(cp, cp);
    // peak parameter t* = -pv / vv >= t_min and squared distance at the peak
    // q = |p x v|^2 / vv <= q_cut, both decided without dividing (vv > 0); the
    // source itself (when its sorted position is not known) never counts
    const bool in_support = src != self && -pv >= tmin * vv && cc <= c.q_cut * vv;
    const float inv_vv = __builtin_amdgcn_rcpf(vv);
    const float q = cc * inv_vv;
    // alpha = o e^{-q/2} = o + o m with m = e^{-q/2} - 1. For small q, m comes
    // from the series so that 1 - alpha = (1 - o) - o m keeps full relative
    // precision when alpha approaches 1 (the adjoint divides by it).
    const float ex = -0.5f * q;
    const float m_small = expm1_small(ex), m_large = __expf(ex) - 1.0f;
    const float em1 = q < 0.5f ? m_small : m_large;
    const float op = r0.w;
    const float alpha = op + op * em1;
    if (!(in_support && alpha >= c.alpha_min)) return 1.0f;
    const bool clamped = alpha >= c.alpha_max;
    const float one_minus = clamped ? 1.0f - c.alpha_max : (1.0f - op) - op * em1;
    LeafHit h;
    h.alpha = alpha;
    h.one_minus = one_minus;
    h.clamped = clamped;
    h.opacity = op;
    h.src = src;
    h.e = p + (-pv * inv_vv) * v;
    h.w0 = w0;
    h.w1 = w1;
    h.w2 = w2;
    on_hit(h, T_before);
    return one_minus;
}

// LDS ring holding the top kRing stack entries of each lane (slot-major, so a
// wave's lanes touch consecutive words for equal depths); deeper entries spill
// to a private array owned by the kernel (kept outside this struct so that the
// scalar state stays in registers). Invariant: entries [max(0, sp - kRing), sp)
// live in the ring at slot (index % kRing), entries [0, sp - kRing) in spill[].
template <int kRing>
struct RingStack {
    static constexpr int kSpill = kMaxStack - kRing;
    int32_t *lds;   // this lane's column: lds[slot * stride]
    int32_t *spill; // private array of kSpill entries
    int stride;
    int sp;

    __device__ __forceinline__ void reset() { sp = 0; }
    __device__ __forceinline__ bool empty() const { return sp == 0; }
    __device__ __forceinline__ void push(int32_t x) {
        const int slot = sp & (kRing - 1);
        if (sp >= kRing) spill[sp - kRing] = lds[slot * stride];
        lds[slot * stride] = x;
        ++sp;
    }
    __device__ __forceinline__ int32_t pop() {
        --sp;
        const int slot = sp & (kRing - 1);
        const int32_t x = lds[slot * stride];
        if (sp >= kRing) lds[slot * stride] = spill[sp - kRing];
        return x;
    }
};

// Enqueue the pooled traversal of listed rays on `stream` (defined with the
// traversal kernels): ray j is ids[j] + id_offset = i * K + k; its T goes to
// out[ids[j]] (out_by_value) or out[j]. With count non-null, only the first
// min(n_list, *count) entries (read on the device) are traced. Ids outside
// [0, n K) give NaN. With queues (8 counters of device scratch, cleared here)
// a persistent grid takes the list's pools from per-XCD queues; without, each
// wave takes a fixed run of pools.
void launch_trace_list(const void *bvh, const rv_gaussians *g, const float *dirs, int K, const Cuts &c,
                       const int64_t *ids, int64_t n_list, const unsigned long long *count, int64_t id_offset,
                       bool out_by_value, float *out, unsigned long long *queues, hipStream_t stream);

}  // namespace rv
