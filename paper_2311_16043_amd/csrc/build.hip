// build.hip -- LBVH construction over 3D Gaussians on gfx950 (Sec. 4.1: a
// binary radix tree built after Karras 2012; leaves are the tight boxes of the
// Gaussians, internal nodes the boxes of their two children).
//
// Pipeline on one stream, no host synchronisation:
//   bounds_partial/bounds_final   min/max of the means (exact in any order)
//   morton                        63-bit keys in binary32 arithmetic
//   sort_hist, scan_seg_sum/sort_scan/scan_seg_apply, sort_scatter  x 8
//                                 stable LSD radix sort, 8-bit digits, wave64
//                                 ballot ranking, one wave per tile, two-level
//                                 prefix sum of the digit counts
//   leaf_prep                     per sorted leaf: whitening W, 3-sigma box, origin data
//   karras                        internal nodes and parents, one thread per node
//   block_boxes, refit_lanes + refit_ranges
//                                 each child box the union of the leaf boxes of
//                                 its sorted-leaf range (no ordering between
//                                 nodes): a lane per node for short ranges, a
//                                 wave per node for the rest
//   collapse4                     compressed four-wide records the tracer walks
#include "rv_internal.h"

namespace rv {
namespace {

// Order-preserving float min/max in a block of 256 threads.
__global__ __launch_bounds__(256) void k_bounds_partial(const float *__restrict__ mean, int64_t n,
                                                        float *__restrict__ partial) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float x = mean[3 * i + a];
            lo[a] = fminf(lo[a], x);
            hi[a] = fmaxf(hi[a], x);
        }
    }
    __shared__ float s[6][256];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + w]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// check != 0 (refit): leave the header untouched unless it records n.
__global__ __launch_bounds__(256) void k_bounds_final(const float *__restrict__ partial, int nparts,
                                                      float *__restrict__ header, int64_t n, int check) {
    if (check && !tree_matches(header, n)) return;  // block-uniform
    __shared__ float s[6][256];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nparts; b += 256) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], partial[b * 6 + a]);
            v[3 + a] = fmaxf(v[3 + a], partial[b * 6 + 3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + w]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) header[threadIdx.x] = s[threadIdx.x][0];
    if (threadIdx.x == 6) header[12] = __int_as_float((int)(n & 0x7fffffff));
}

// Spread the low 21 bits of v to every third bit (bit b -> bit 3b).
__device__ __forceinline__ uint64_t part1by2_21(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x001f00000000ffffull;
    v = (v | (v << 16)) & 0x001f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Quantise one coordinate: every operation is a single correctly rounded
// binary32 operation (sub, sub, div, exact scale by 2^21, floor, clamp).
__device__ __forceinline__ uint32_t quantise21(float x, float lo, float hi) {
#pragma clang fp contract(off)
    float den = hi - lo;
    float u = den > 0.0f ? (x - lo) / den : 0.0f;
    float f = floorf(u * 2097152.0f);
    f = fminf(fmaxf(f, 0.0f), 2097151.0f);
    return (uint32_t)f;
}

__global__ __launch_bounds__(256) void k_morton(const float *__restrict__ mean, int64_t n,
                                                const float *__restrict__ header, uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t cx = quantise21(mean[3 * i + 0], header[0], header[3]);
    uint32_t cy = quantise21(mean[3 * i + 1], header[1], header[4]);
    uint32_t cz = quantise21(mean[3 * i + 2], header[2], header[5]);
    keys[i] = (part1by2_21(cx) << 2) | (part1by2_21(cy) << 1) | part1by2_21(cz);
    vals[i] = (uint32_t)i;
}

// ---- radix sort ------------------------------------------------------------

__global__ __launch_bounds__(kSortWave) void k_sort_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                         uint32_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    const int lane = threadIdx.x;
    for (int i = lane; i < 256; i += kSortWave) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j0 = 0; j0 < kSortItems && base + (int64_t)j0 * kSortWave < n; j0 += kSortAhead) {
        // the next kSortAhead keys of this lane are in flight together:
        // unconditional loads (past the end: the last key, discarded) so that
        // none waits behind a branch
        uint64_t kv[kSortAhead];
        bool ok[kSortAhead];
#pragma unroll
        for (int u = 0; u < kSortAhead; ++u) {
            const int64_t idx = base + (int64_t)(j0 + u) * kSortWave + lane;
            ok[u] = idx < n;
            kv[u] = keys[ok[u] ? idx : n - 1];
        }
#pragma unroll
        for (int u = 0; u < kSortAhead; ++u) {
            const uint32_t d = ok[u] ? (uint32_t)(kv[u] >> shift) & 255u : 0u;
            const uint64_t valid = __ballot(ok[u]);
            if (valid == 0) break;
            const uint64_t peers = match_digit8(d, valid);
            // the lowest lane of each group adds the group's size
            if (ok[u] && (peers & ((1ull << lane) - 1ull)) == 0) h[d] += (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    for (int i = lane; i < 256; i += kSortWave) hist[(int64_t)i * nblocks + blockIdx.x] = h[i];
}

// Exclusive prefix sum of the digit-major counts hist[256 * nblocks] in two
// levels: k_scan_seg_sum adds each segment of kScanSeg counts, k_sort_scan
// (one block) turns the segment sums into segment offsets, and
// k_scan_seg_apply scans each segment from its offset. Integer sums: the
// result is the plain prefix sum whatever the grouping.

// seg[b] = sum of hist[b kScanSeg, (b + 1) kScanSeg), clipped to total
// (256 threads, four counts each).
__global__ __launch_bounds__(256) void k_scan_seg_sum(const uint32_t *__restrict__ hist, int64_t total,
                                                      uint32_t *__restrict__ seg) {
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanSeg;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k * 256 + t;
        if (i < total) v += hist[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    if (t == 0) seg[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Exclusive prefix sum of segment b in place, starting from seg[b] (the
// segment's offset). Thread t holds counts 4t .. 4t + 3 of the segment; total
// is a multiple of 256, so a thread's four counts are all in range or none.
__global__ __launch_bounds__(256) void k_scan_seg_apply(uint32_t *__restrict__ hist, int64_t total,
                                                        const uint32_t *__restrict__ seg) {
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t i = (int64_t)blockIdx.x * kScanSeg + 4 * t;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i < total) v = *reinterpret_cast<const uint4 *>(hist + i);
    const uint32_t own = v.x + v.y + v.z + v.w;
    uint32_t x = own;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = seg[blockIdx.x] + x - own;
    for (int k = 0; k < w; ++k) before += wsum[k];
    if (i < total) {
        uint4 o;
        o.x = before;
        o.y = o.x + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        *reinterpret_cast<uint4 *>(hist + i) = o;
    }
}

// Exclusive prefix sum over hist[total] in one block (the top level of the
// two-level sum above).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *__restrict__ hist, int64_t total) {
    // exclusive prefix sum in place, 1024 consecutive counts at a time:
    // coalesced loads, a shuffle scan per wave, the 16 wave totals scanned in
    // LDS, and a running carry between rows
    __shared__ uint32_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < total; base += 1024) {
        const int64_t i = base + t;
        const uint32_t v = i < total ? hist[i] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            uint32_t u = lane < 16 ? wsum[lane] : 0u;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const uint32_t y = __shfl_up(u, off);
                if (lane >= off) u += y;
            }
            if (lane < 16) wsum[lane] = u;
        }
        __syncthreads();
        const uint32_t before = w > 0 ? wsum[w - 1] : 0u;
        if (i < total) hist[i] = carry + before + x - v;
        carry += wsum[15];
        __syncthreads();  // wsum is rewritten by the next row
    }
}

__global__ __launch_bounds__(kSortWave) void k_sort_scatter(const uint64_t *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin, int64_t n, int shift,
                                                            const uint32_t *__restrict__ hist, int64_t nblocks,
                                                            uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    __shared__ uint32_t offs[256];
    const int lane = threadIdx.x;
    for (int i = lane; i < 256; i += kSortWave) offs[i] = hist[(int64_t)i * nblocks + blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int j0 = 0; j0 < kSortItems && base + (int64_t)j0 * kSortWave < n; j0 += kSortAhead) {
        // the next kSortAhead items of this lane are loaded together, then
        // ranked strictly in order (the sort stays stable)
        uint64_t key[kSortAhead];
        uint32_t val[kSortAhead];
        bool ok[kSortAhead];
#pragma unroll
        for (int u = 0; u < kSortAhead; ++u) {
            // unconditional loads (past the end: the last item, discarded)
            const int64_t idx = base + (int64_t)(j0 + u) * kSortWave + lane;
            ok[u] = idx < n;
            const int64_t at_idx = ok[u] ? idx : n - 1;
            key[u] = kin[at_idx];
            val[u] = vin[at_idx];
        }
#pragma unroll
        for (int u = 0; u < kSortAhead; ++u) {
            const uint32_t d = (uint32_t)(key[u] >> shift) & 255u;
            const uint64_t valid = __ballot(ok[u]);
            if (valid == 0) break;
            const uint64_t peers = match_digit8(d, valid);
            const uint32_t rank = (uint32_t)__popcll(peers & lt);
            const uint32_t pos = ok[u] ? offs[d] + rank : 0u;
            __builtin_amdgcn_wave_barrier();
            // every lane has read its group's offset; the group leader advances it
            if (ok[u] && rank == 0) offs[d] = pos + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            if (ok[u]) {
                kout[pos] = key[u];
                vout[pos] = val[u];
            }
        }
    }
}

// ---- leaf records ------------------------------------------------------------

__global__ __launch_bounds__(256) void k_leaf_prep(const float *__restrict__ mean, const float *__restrict__ quat,
                                                   const float *__restrict__ log_scale,
                                                   const float *__restrict__ opacity, const float *__restrict__ normal,
                                                   int64_t n, const uint32_t *__restrict__ perm,
                                                   const float *__restrict__ header,
                                                   float4 *__restrict__ rec, float *__restrict__ box,
                                                   float4 *__restrict__ origins) {
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n || !tree_matches(header, n)) return;
    // scene scale: largest coordinate magnitude plus the diagonal of the means' box
    float scale = 0.0f, diag2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        scale = fmaxf(scale, fmaxf(fabsf(header[a]), fabsf(header[3 + a])));
        diag2 += (header[3 + a] - header[a]) * (header[3 + a] - header[a]);
    }
    const float widen_abs = (scale + sqrtf(diag2) + 1.0f) * 0x1p-20f;
    const int64_t i = perm[m];
    float qw = quat[4 * i], qx = quat[4 * i + 1], qy = quat[4 * i + 2], qz = quat[4 * i + 3];
    float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    // rotation matrix of the unit quaternion (w, x, y, z)
    float R[3][3];
    R[0][0] = 1.f - 2.f * (qy * qy + qz * qz); R[0][1] = 2.f * (qx * qy - qw * qz); R[0][2] = 2.f * (qx * qz + qw * qy);
    R[1][0] = 2.f * (qx * qy + qw * qz); R[1][1] = 1.f - 2.f * (qx * qx + qz * qz); R[1][2] = 2.f * (qy * qz - qw * qx);
    R[2][0] = 2.f * (qx * qz - qw * qy); R[2][1] = 2.f * (qy * qz + qw * qx); R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
    float ls[3] = {log_scale[3 * i], log_scale[3 * i + 1], log_scale[3 * i + 2]};
    float s[3], is[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a] = expf(ls[a]);
        is[a] = expf(-ls[a]);
    }
    float mu[3] = {mean[3 * i], mean[3 * i + 1], mean[3 * i + 2]};
    // whitening W = diag(1/s) R^T: row a is column a of R divided by s_a
    float W[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) W[a][c] = is[a] * R[c][a];
    // row 2 of W is not stored: for a proper rotation, column 2 of R is
    // column 0 x column 1, so W row 2 = (s0 s1 / s2) (W row 0 x W row 1)
    rec[kLeafF4 * m + 0] = make_float4(mu[0], mu[1], mu[2], opacity[i]);
    rec[kLeafF4 * m + 1] = make_float4(W[0][0], W[0][1], W[0][2], s[0] * s[1] * is[2]);
    rec[kLeafF4 * m + 2] = make_float4(W[1][0], W[1][1], W[1][2], __int_as_float((int)i));
    // 3-sigma box: half extent along world axis a is 3 sqrt(sum_m (R_am s_m)^2),
    // widened by a relative 2^-12 (rounding of R, s and the square root) and by
    // 2^-20 of the scene scale (rounding of the box and of the slab test)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float e0 = R[a][0] * s[0], e1 = R[a][1] * s[1], e2 = R[a][2] * s[2];
        float h = kBuildSigma * sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
        h = h * (1.0f + 0x1p-12f) + widen_abs;
        box[6 * m + a] = mu[a] - h;
        box[6 * m + 3 + a] = mu[a] + h;
    }
    float nx = 0.f, ny = 0.f, nz = 1.f;
    if (normal) {
        nx = normal[3 * i]; ny = normal[3 * i + 1]; nz = normal[3 * i + 2];
        float nl = sqrtf(nx * nx + ny * ny + nz * nz);
        nx /= nl; ny /= nl; nz /= nl;
    }
    float smax = expf(fmaxf(ls[0], fmaxf(ls[1], ls[2])));
    origins[m] = make_float4(nx, ny, nz, smax);
}

// ---- Karras internal nodes ---------------------------------------------------

// Common-prefix length of the augmented keys (key, position) at i and j;
// -1 when j is outside [0, n).
__device__ __forceinline__ int prefix_len(const uint64_t *__restrict__ k, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

__global__ __launch_bounds__(256) void k_karras(const uint64_t *__restrict__ keys, int64_t n,
                                                float4 *__restrict__ nodes, int32_t *__restrict__ parent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    // direction of the range: towards the neighbour sharing the longer prefix
    const int d = (prefix_len(keys, n, i, i + 1) - prefix_len(keys, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = prefix_len(keys, n, i, i - d);
    // exponential search for an upper bound of the range length, then binary search
    int64_t lmax = 2;
    while (prefix_len(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = prefix_len(keys, n, i, j);
    // split: the last position (counted from i) sharing more than dnode bits with i
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    const int32_t left = (lo == gamma) ? ~(int32_t)gamma : (int32_t)gamma;
    const int32_t right = (hi == gamma + 1) ? ~(int32_t)(gamma + 1) : (int32_t)(gamma + 1);
    // words 12-15: the children, then the first and last sorted leaf under i
    nodes[4 * i + 3] = make_float4(__int_as_float(left), __int_as_float(right), __int_as_float((int32_t)lo),
                                   __int_as_float((int32_t)hi));
    parent[left >= 0 ? left : (n - 1 + (int64_t)~left)] = (int32_t)i;
    parent[right >= 0 ? right : (n - 1 + (int64_t)~right)] = (int32_t)i;
    if (i == 0) parent[0] = -1;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, int64_t count, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---- refit -------------------------------------------------------------------
//
// Every internal node covers a contiguous range of sorted leaves (Karras), so
// the box of each child is the union of the leaf boxes over the child's range:
// min and max are exact in any order, so this equals the bottom-up union of
// the children's boxes, with no ordering between nodes to arrange. Unions of
// blocks of kBoxBlock consecutive leaves keep long ranges short: a range reads
// at most 2 kBoxBlock leaf boxes and its whole blocks' boxes.

// Running union (lo, hi) of boxes, and the wave-wide union by butterfly.
struct BoxAcc {
    float lo[3], hi[3];
    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = __builtin_inff();
            hi[a] = -__builtin_inff();
        }
    }
    __device__ __forceinline__ void add(const float *__restrict__ b) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], b[a]);
            hi[a] = fmaxf(hi[a], b[3 + a]);
        }
    }
    __device__ __forceinline__ void wave_union() {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(lo[a], __shfl_xor(lo[a], off));
                hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off));
            }
    }
    __device__ __forceinline__ void store(float *__restrict__ out) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out[a] = lo[a];
            out[3 + a] = hi[a];
        }
    }
};

// block_box[b] = union of the leaf boxes of leaves b kBoxBlock .. (b + 1) kBoxBlock - 1
// (one wave per block).
__global__ __launch_bounds__(256) void k_block_boxes(int64_t n, const float *__restrict__ leaf_box,
                                                     float *__restrict__ block_box, const float *__restrict__ header) {
    if (!tree_matches(header, n)) return;
    const int lane = threadIdx.x & 63;
    const int64_t nb = (n + kBoxBlock - 1) / kBoxBlock;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += (int64_t)gridDim.x * 4) {
        BoxAcc acc;
        acc.reset();
        const int64_t e = min(n, (b + 1) * kBoxBlock);
        for (int64_t m = b * kBoxBlock + lane; m < e; m += 64) acc.add(leaf_box + 6 * m);
        acc.wave_union();
        if (lane == 0) acc.store(block_box + 6 * b);
    }
}

// Union of the leaf boxes of sorted leaves [a, e) by one wave (result in
// every lane).
__device__ __forceinline__ void range_union(int64_t a, int64_t e, const float *__restrict__ leaf_box,
                                            const float *__restrict__ block_box, int lane, BoxAcc &acc) {
    acc.reset();
    const int64_t ba = (a + kBoxBlock - 1) / kBoxBlock, be = e / kBoxBlock;  // whole blocks [ba, be)
    if (ba >= be) {
        for (int64_t m = a + lane; m < e; m += 64) acc.add(leaf_box + 6 * m);
    } else {
        for (int64_t m = a + lane; m < ba * kBoxBlock; m += 64) acc.add(leaf_box + 6 * m);
        for (int64_t b = ba + lane; b < be; b += 64) acc.add(block_box + 6 * b);
        for (int64_t m = be * kBoxBlock + lane; m < e; m += 64) acc.add(leaf_box + 6 * m);
    }
    acc.wave_union();
}

// Nodes over at most kLaneRange leaves (most of them: every level below the
// top log2(n / kLaneRange) or so) are refit by one lane each; the others by
// one wave each. The two kernels write disjoint nodes.
constexpr int64_t kLaneRange = 32;

// Root box in the header from node 0's two child boxes.
__device__ __forceinline__ void store_root(float *__restrict__ header, const float *l_lo, const float *l_hi,
                                           const float *r_lo, const float *r_hi) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        header[6 + a] = fminf(l_lo[a], r_lo[a]);
        header[9 + a] = fmaxf(l_hi[a], r_hi[a]);
    }
}

// Child boxes of the internal nodes over at most kLaneRange leaves, one lane
// per node: the left child covers leaves [lo, gamma], the right
// [gamma + 1, hi], gamma being the left child's last leaf.
__global__ __launch_bounds__(256) void k_refit_lanes(int64_t n, const float *__restrict__ leaf_box,
                                                     float *__restrict__ nodes, float *__restrict__ header) {
    if (!tree_matches(header, n)) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n - 1) return;
    float *rec = nodes + 16 * i;
    const int64_t lo = __float_as_int(rec[14]), hi = __float_as_int(rec[15]);
    if (hi - lo + 1 > kLaneRange) return;
    const int32_t left = __float_as_int(rec[12]);
    const int64_t gamma = left < 0 ? (int64_t)~left : (int64_t)left;
    BoxAcc l, r;
    l.reset();
    r.reset();
    for (int64_t m = lo; m <= gamma; ++m) l.add(leaf_box + 6 * m);
    for (int64_t m = gamma + 1; m <= hi; ++m) r.add(leaf_box + 6 * m);
    l.store(rec);
    r.store(rec + 6);
    if (i == 0) store_root(header, l.lo, l.hi, r.lo, r.hi);
}

// Child boxes of the internal nodes over more than kLaneRange leaves, one
// wave per node; node 0's union is the root box in the header.
__global__ __launch_bounds__(256) void k_refit_ranges(int64_t n, const float *__restrict__ leaf_box,
                                                      const float *__restrict__ block_box, float *__restrict__ nodes,
                                                      float *__restrict__ header) {
    if (!tree_matches(header, n)) return;
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n - 1; i += (int64_t)gridDim.x * 4) {
        float *rec = nodes + 16 * i;
        const int64_t lo = __float_as_int(rec[14]), hi = __float_as_int(rec[15]);
        if (hi - lo + 1 <= kLaneRange) continue;
        const int32_t left = __float_as_int(rec[12]);
        // the split gamma is the left child's index, whether leaf (~gamma) or node
        const int64_t gamma = left < 0 ? (int64_t)~left : (int64_t)left;
        BoxAcc l, r;
        range_union(lo, gamma + 1, leaf_box, block_box, lane, l);
        range_union(gamma + 1, hi + 1, leaf_box, block_box, lane, r);
        if (lane == 0) {
            l.store(rec);
            r.store(rec + 6);
            if (i == 0) store_root(header, l.lo, l.hi, r.lo, r.hi);
        }
    }
}

// A single Gaussian: its leaf box is the root box.
__global__ void k_root_single(const float *__restrict__ leaf_box, float *__restrict__ header) {
    if (!tree_matches(header, 1)) return;
    if (threadIdx.x < 6) header[6 + threadIdx.x] = leaf_box[threadIdx.x];
}

// Refit of a tree built over n sorted leaves (nodes hold their ranges).
inline void launch_refit(int64_t n, const float *leaf_box, float *block_box, float *nodes, float *header,
                         hipStream_t s) {
    if (n > 1) {
        const int64_t nb = (n + kBoxBlock - 1) / kBoxBlock;
        hipLaunchKernelGGL(k_block_boxes, dim3((unsigned)std::min<int64_t>((nb + 3) / 4, 65536)), dim3(256), 0, s,
                           n, leaf_box, block_box, header);
        hipLaunchKernelGGL(k_refit_lanes, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, n, leaf_box, nodes,
                           header);
        hipLaunchKernelGGL(k_refit_ranges, dim3((unsigned)std::min<int64_t>((n - 1 + 3) / 4, 65536)), dim3(256), 0,
                           s, n, leaf_box, block_box, nodes, header);
    } else {
        hipLaunchKernelGGL(k_root_single, dim3(1), dim3(64), 0, s, leaf_box, header);
    }
}

// ---- four-wide nodes ----------------------------------------------------------

// Compressed wide record of internal node i: the children of i's two
// children (a child that is a leaf keeps its own slot, the next slot is
// empty), so one traversal step tests up to four boxes from three 16-byte
// loads. Every internal node gets a record; a traversal from the root only
// lands on nodes an even number of binary levels down. Layout (12 words in a
// 64-byte slot):
//   words 0-2   origin O (float), at or below the lowest child plane
//   word 3      bytes 0-2: per-axis step exponents, step_a = 2^(byte - 127);
//               byte 3: kind of slot j in bits 2j..2j+1 (0 empty, 1 internal
//               node, 3 leaf: bit 0 = used, bit 1 = leaf)
//   words 4-9   lo_x, lo_y, lo_z, hi_x, hi_y, hi_z planes, one byte per slot
//               (byte j = slot j): plane = O_a + q step_a
//   words 10-11 index of slot 2s for side s; slot 2s + 1 holds that index + 1
//               (a node's two children always have consecutive indices)
// Planes are rounded outward from the refitted binary boxes after widening
// them by eta = (largest root-box coordinate + root diagonal + 1) 2^-20, in
// exact (double) arithmetic, so a traversal that evaluates the plane
// distances as fma(q, step/d, (O - o)/d) (error below eta / 2) never rejects
// a box the exact ray enters.
__global__ __launch_bounds__(256) void k_collapse4(int64_t n, const float *__restrict__ nodes,
                                                   const float *__restrict__ header, float *__restrict__ nodes4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1 || !tree_matches(header, n)) return;
    double ext = 0.0, diag2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double l = header[6 + a], h = header[9 + a];
        ext = fmax(ext, fmax(fabs(l), fabs(h)));
        diag2 += (h - l) * (h - l);
    }
    const double eta = (ext + sqrt(diag2) + 1.0) * 0x1p-20;
    const float *r = nodes + 16 * i;
    float box[4][6];
    uint32_t kind[4];
    int32_t base[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int32_t c = __float_as_int(r[12 + side]);
        const int s0 = 2 * side, s1 = 2 * side + 1;
        if (c < 0) {
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                box[s0][a] = r[6 * side + a];
                box[s1][a] = r[6 * side + a];  // unused; keeps the node box unchanged
            }
            kind[s0] = 3u;
            kind[s1] = 0u;
            base[side] = ~c;
        } else {
            const float *rc = nodes + 16 * (int64_t)c;
            const int32_t lc = __float_as_int(rc[12]), rcid = __float_as_int(rc[13]);
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                box[s0][a] = rc[a];
                box[s1][a] = rc[6 + a];
            }
            kind[s0] = lc < 0 ? 3u : 1u;
            kind[s1] = rcid < 0 ? 3u : 1u;
            base[side] = lc < 0 ? ~lc : lc;
        }
    }
    uint32_t words[12];
    uint32_t meta = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double lo = box[0][a], hi = box[0][3 + a];
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            lo = fmin(lo, (double)box[j][a]);
            hi = fmax(hi, (double)box[j][3 + a]);
        }
        // origin: a float at or below lo - eta
        const double od = lo - eta;
        float O = (float)od;
        if ((double)O > od) O = nextafterf(O, -__builtin_inff());
        // smallest power-of-two step with 255 steps reaching hi + eta
        int e;
        frexp((hi + eta - (double)O) / 255.0, &e);
        e = max(-126, min(127, e));
        const double step = ldexp(1.0, e);
        uint32_t qlo = 0, qhi = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double fl = floor(((double)box[j][a] - eta - (double)O) / step);
            const double fh = ceil(((double)box[j][3 + a] + eta - (double)O) / step);
            qlo |= (uint32_t)fmin(fmax(fl, 0.0), 255.0) << (8 * j);
            qhi |= (uint32_t)fmin(fmax(fh, 0.0), 255.0) << (8 * j);
        }
        words[a] = __float_as_uint(O);
        words[4 + a] = qlo;
        words[7 + a] = qhi;
        meta |= (uint32_t)(e + 127) << (8 * a);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) meta |= kind[j] << (24 + 2 * j);
    words[3] = meta;
    words[10] = (uint32_t)base[0];
    words[11] = (uint32_t)base[1];
    uint4 *dst = reinterpret_cast<uint4 *>(nodes4) + 4 * i;
    dst[0] = make_uint4(words[0], words[1], words[2], words[3]);
    dst[1] = make_uint4(words[4], words[5], words[6], words[7]);
    dst[2] = make_uint4(words[8], words[9], words[10], words[11]);
    dst[3] = make_uint4(0u, 0u, 0u, 0u);
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

}  // namespace rv

using namespace rv;

extern "C" size_t rv_bvh_bytes(int64_t n) { return n < 1 ? 0 : bvh_layout(n).total; }

extern "C" size_t rv_build_workspace_bytes(int64_t n) { return n < 1 ? 0 : build_ws_layout(n).total; }

extern "C" rv_status rv_bvh_view(const void *bvh, int64_t n, rv_bvh_arrays *out) {
    clear_error();
    RV_REQUIRE(bvh && out, RV_ERR_INVALID_ARG, "rv_bvh_view: null pointer");
    RV_REQUIRE(n >= 1 && n <= RV_MAX_GAUSSIANS, RV_ERR_INVALID_ARG, "rv_bvh_view: n out of range");
    BvhLayout L = bvh_layout(n);
    out->n = n;
    out->header = at<float>(bvh, L.header);
    out->keys = at<uint64_t>(bvh, L.keys);
    out->perm = at<uint32_t>(bvh, L.perm);
    out->nodes = at<float>(bvh, L.nodes);
    out->parent = at<int32_t>(bvh, L.parent);
    out->leaf_records = at<float>(bvh, L.leaf_rec);
    out->leaf_boxes = at<float>(bvh, L.leaf_box);
    out->origins = at<float>(bvh, L.origins);
    out->nodes4 = at<uint32_t>(bvh, L.nodes4);
    return RV_OK;
}

extern "C" rv_status rv_build_bvh(const rv_gaussians *g, void *bvh, size_t bvh_bytes, void *ws, size_t ws_bytes,
                                  void *stream) {
    clear_error();
    RV_REQUIRE(g && bvh && ws, RV_ERR_INVALID_ARG, "rv_build_bvh: null argument (g, bvh or ws)");
    RV_REQUIRE(g->mean && g->quat && g->log_scale && g->opacity, RV_ERR_INVALID_ARG,
               "rv_build_bvh: null Gaussian array");
    const int64_t n = g->n;
    RV_REQUIRE(n >= 1 && n <= RV_MAX_GAUSSIANS, RV_ERR_INVALID_ARG, "rv_build_bvh: n=%lld out of range",
               (long long)n);
    RV_REQUIRE(((uintptr_t)bvh % kAlign) == 0 && ((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG,
               "rv_build_bvh: bvh and ws must be 256-byte aligned");
    const BvhLayout L = bvh_layout(n);
    const BuildWsLayout W = build_ws_layout(n);
    RV_REQUIRE(bvh_bytes >= L.total, RV_ERR_WORKSPACE, "rv_build_bvh: bvh_bytes %zu < %zu", bvh_bytes, L.total);
    RV_REQUIRE(ws_bytes >= W.total, RV_ERR_WORKSPACE, "rv_build_bvh: ws_bytes %zu < %zu", ws_bytes, W.total);
    hipStream_t s = (hipStream_t)stream;

    float *header = at<float>(bvh, L.header);
    uint64_t *keys = at<uint64_t>(bvh, L.keys);
    uint32_t *perm = at<uint32_t>(bvh, L.perm);
    float *nodes = at<float>(bvh, L.nodes);
    int32_t *parent = at<int32_t>(bvh, L.parent);
    float4 *rec = at<float4>(bvh, L.leaf_rec);
    float *box = at<float>(bvh, L.leaf_box);
    float4 *orig = at<float4>(bvh, L.origins);
    uint64_t *keys_tmp = at<uint64_t>(ws, W.keys_tmp);
    uint32_t *vals_tmp = at<uint32_t>(ws, W.vals_tmp);
    uint32_t *hist = at<uint32_t>(ws, W.hist);
    uint32_t *seg = at<uint32_t>(ws, W.seg);
    float *bpart = at<float>(ws, W.bounds);
    float *block_box = at<float>(ws, W.block_box);

    const int nb = (int)std::min<int64_t>(kBoundsBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_bounds_partial, dim3(nb), dim3(256), 0, s, g->mean, n, bpart);
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(256), 0, s, bpart, nb, header, n, 0);
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n, 256)), dim3(256), 0, s, g->mean, n, header, keys, perm);
    rv_status st = check_launch("morton");
    if (st != RV_OK) return st;

    // 8 passes of 8 bits; even count, so the result lands back in keys/perm
    uint64_t *ka = keys, *kb = keys_tmp;
    uint32_t *va = perm, *vb = vals_tmp;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)W.nblocks), dim3(kSortWave), 0, s, ka, n, shift, hist,
                           W.nblocks);
        hipLaunchKernelGGL(k_scan_seg_sum, dim3((unsigned)W.nseg), dim3(256), 0, s, hist, (int64_t)256 * W.nblocks,
                           seg);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, seg, W.nseg);
        hipLaunchKernelGGL(k_scan_seg_apply, dim3((unsigned)W.nseg), dim3(256), 0, s, hist, (int64_t)256 * W.nblocks,
                           seg);
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)W.nblocks), dim3(kSortWave), 0, s, ka, va, n, shift,
                           hist, W.nblocks, kb, vb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    st = check_launch("radix sort");
    if (st != RV_OK) return st;

    hipLaunchKernelGGL(k_leaf_prep, dim3(grid_for(n, 256)), dim3(256), 0, s, g->mean, g->quat, g->log_scale,
                       g->opacity, g->normal, n, perm, header, rec, box, orig);
    if (n > 1) {
        hipLaunchKernelGGL(k_karras, dim3(grid_for(n - 1, 256)), dim3(256), 0, s, keys, n,
                           reinterpret_cast<float4 *>(nodes), parent);
        launch_refit(n, box, block_box, nodes, header, s);
        hipLaunchKernelGGL(k_collapse4, dim3(grid_for(n - 1, 256)), dim3(256), 0, s, n, nodes, header,
                           at<float>(bvh, L.nodes4));
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(parent), (int64_t)1,
                           0xffffffffu);
        launch_refit(n, box, block_box, nodes, header, s);
    }
    return check_launch("leaf records / karras / refit");
}

extern "C" rv_status rv_refit_bvh(const rv_gaussians *g, void *bvh, size_t bvh_bytes, void *ws, size_t ws_bytes,
                                  void *stream) {
    clear_error();
    RV_REQUIRE(g && bvh && ws, RV_ERR_INVALID_ARG, "rv_refit_bvh: null argument (g, bvh or ws)");
    RV_REQUIRE(g->mean && g->quat && g->log_scale && g->opacity, RV_ERR_INVALID_ARG,
               "rv_refit_bvh: null Gaussian array");
    const int64_t n = g->n;
    RV_REQUIRE(n >= 1 && n <= RV_MAX_GAUSSIANS, RV_ERR_INVALID_ARG, "rv_refit_bvh: n=%lld out of range",
               (long long)n);
    RV_REQUIRE(((uintptr_t)bvh % kAlign) == 0 && ((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG,
               "rv_refit_bvh: bvh and ws must be 256-byte aligned");
    const BvhLayout L = bvh_layout(n);
    const BuildWsLayout W = build_ws_layout(n);
    RV_REQUIRE(bvh_bytes >= L.total, RV_ERR_WORKSPACE, "rv_refit_bvh: bvh_bytes %zu < %zu", bvh_bytes, L.total);
    RV_REQUIRE(ws_bytes >= W.total, RV_ERR_WORKSPACE, "rv_refit_bvh: ws_bytes %zu < %zu", ws_bytes, W.total);
    hipStream_t s = (hipStream_t)stream;
    float *header = at<float>(bvh, L.header);
    const uint32_t *perm = at<uint32_t>(bvh, L.perm);
    float *nodes = at<float>(bvh, L.nodes);
    float4 *rec = at<float4>(bvh, L.leaf_rec);
    float *box = at<float>(bvh, L.leaf_box);
    float4 *orig = at<float4>(bvh, L.origins);
    float *bpart = at<float>(ws, W.bounds);
    float *block_box = at<float>(ws, W.block_box);
    // the scene scale of the leaf widening follows the moved means; the sorted
    // order, keys and topology stay as built
    const int nb = (int)std::min<int64_t>(kBoundsBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_bounds_partial, dim3(nb), dim3(256), 0, s, g->mean, n, bpart);
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(256), 0, s, bpart, nb, header, n, 1);
    hipLaunchKernelGGL(k_leaf_prep, dim3(grid_for(n, 256)), dim3(256), 0, s, g->mean, g->quat, g->log_scale,
                       g->opacity, g->normal, n, perm, header, rec, box, orig);
    launch_refit(n, box, block_box, nodes, header, s);
    if (n > 1)
        hipLaunchKernelGGL(k_collapse4, dim3(grid_for(n - 1, 256)), dim3(256), 0, s, n, nodes, header,
                           at<float>(bvh, L.nodes4));
    return check_launch("rv_refit_bvh");
}
