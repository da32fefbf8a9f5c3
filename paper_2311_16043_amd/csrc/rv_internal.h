// rv_internal.h -- shared layout, error reporting and device helpers of the
// gfx950 visibility library (internal; the public ABI is include/rvis.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "rvis.h"

namespace rv {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define RV_REQUIRE(cond, code, ...)      \
    do {                                 \
        if (!(cond)) {                   \
            ::rv::set_error(__VA_ARGS__); \
            return (code);               \
        }                                \
    } while (0)

// Check the launch that was just enqueued.
rv_status check_launch(const char *what);

// ---------------------------------------------------------------------------
// BVH blob layout (byte offsets, every section 256-byte aligned)
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Half-width of the leaf boxes in standard deviations (3-sigma support).
constexpr float kBuildSigma = 3.0f;
// Header floats: lo[3], hi[3] of the means; root box lo[3], hi[3]; n (as float bits) ...
constexpr int kHeaderFloats = 16;

// Child id of an unused or missed slot of a four-wide node as the traversal
// reports it (leaves are ~m, internal nodes their binary id >= 0).
constexpr int32_t kEmptyChild = INT32_MIN;
// Bytes per compressed four-wide node (48 used).
constexpr size_t kNode4Bytes = 64;
// Leaf record, three float4 per sorted leaf: (mu, opacity), (W row 0,
// s0 s1 / s2), (W row 1, source index bits); W row 2 = (s0 s1 / s2) (row 0 x row 1).
constexpr int kLeafF4 = 3;

struct BvhLayout {
    size_t header, keys, perm, nodes, parent, leaf_rec, leaf_box, origins, nodes4, total;
};

inline BvhLayout bvh_layout(int64_t n) {
    BvhLayout L{};
    size_t nn = (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    L.header = off; off = align_up(off + kHeaderFloats * sizeof(float));
    L.keys = off; off = align_up(off + nn * 8);
    L.perm = off; off = align_up(off + nn * 4);
    L.nodes = off; off = align_up(off + (nn > 1 ? nn - 1 : 1) * 64);
    L.parent = off; off = align_up(off + (2 * nn - 1) * 4);
    L.leaf_rec = off; off = align_up(off + nn * 16 * kLeafF4);
    L.leaf_box = off; off = align_up(off + nn * 24);
    L.origins = off; off = align_up(off + nn * 16);
    L.nodes4 = off; off = align_up(off + (nn > 1 ? nn - 1 : 1) * kNode4Bytes);
    L.total = off;
    return L;
}

// Radix sort tiling: one wave64 per block, 32 rounds of 64 keys per tile.
constexpr int kSortWave = 64;
constexpr int kSortItems = 32;
constexpr int kSortTile = kSortWave * kSortItems;
constexpr int kSortAhead = 4;  // items per lane loaded ahead of their ranking
static_assert(kSortItems % kSortAhead == 0, "sort tile must hold whole load groups");
constexpr int kBoundsBlocks = 1024;

// Leaves per block box of the refit (unions of consecutive sorted leaves).
constexpr int64_t kBoxBlock = 256;

// Counts per segment of the radix sort's two-level prefix sum.
constexpr int64_t kScanSeg = 1024;

struct BuildWsLayout {
    size_t keys_tmp, vals_tmp, hist, seg, bounds, block_box, total;
    int64_t nblocks, nseg;
};

inline BuildWsLayout build_ws_layout(int64_t n) {
    BuildWsLayout W{};
    size_t nn = (size_t)(n > 0 ? n : 1);
    W.nblocks = (int64_t)((nn + kSortTile - 1) / kSortTile);
    size_t off = 0;
    W.keys_tmp = off; off = align_up(off + nn * 8);
    W.vals_tmp = off; off = align_up(off + nn * 4);
    W.hist = off; off = align_up(off + 256 * (size_t)W.nblocks * 4);
    W.nseg = (256 * W.nblocks + kScanSeg - 1) / kScanSeg;
    W.seg = off; off = align_up(off + (size_t)W.nseg * 4);
    W.bounds = off; off = align_up(off + kBoundsBlocks * 6 * sizeof(float));
    W.block_box = off; off = align_up(off + (size_t)((nn + kBoxBlock - 1) / kBoxBlock) * 6 * sizeof(float));
    W.total = off;
    return W;
}

template <typename T>
inline T *at(void *base, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }
template <typename T>
inline const T *at(const void *base, size_t off) {
    return reinterpret_cast<const T *>(static_cast<const char *>(base) + off);
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ f3 operator*(float s, f3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Header word 12 of a BVH blob holds the number of Gaussians it was built
// over. Every kernel that reads a tree compares it with the caller's n before
// touching anything else in the blob (the section offsets follow from n), so a
// blob built for another Gaussian set is never walked: traversals give NaN and
// a refit leaves the blob as it was.
__device__ __forceinline__ bool tree_matches(const float *__restrict__ header, int64_t n) {
    return __float_as_int(header[12]) == (int)(n & 0x7fffffff);
}

// Mask of the lanes whose `digit` equals this lane's, among `valid` lanes
// (eight ballots, one per digit bit).
__device__ __forceinline__ uint64_t match_digit8(uint32_t digit, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t m = __ballot((digit >> b) & 1u);
        peers &= ((digit >> b) & 1u) ? m : ~m;
    }
    return peers;
}

}  // namespace rv
