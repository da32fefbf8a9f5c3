// trace.hip -- visibility pre-computation (Sec. 4.2): for every Gaussian i and
// direction k, the transmittance of the ray leaving mean_i (Sec. 4.1), and the
// per-Gaussian average over the K directions (the "averaged visibility" of the
// ablation study, Sec. 5.4).
//
// Work mapping. Rays come in pools (see the pooled traversal below): 64
// Gaussians adjacent in Morton (sorted-leaf) order times one direction for the
// persistent all-ray kernel (which also serves the SH projection), times a
// chunk of 4 consecutive directions for the adjoint kernel, and 256
// consecutive entries for the list kernel. The all-ray forward runs a
// persistent grid that takes pools from eight queues, one per XCD, each a
// contiguous eighth of the Morton order, so each L2 sees a compact part of the
// tree; a wave whose queue is spent takes pools from the others, so no XCD
// idles while another still holds work. A wave keeps its lanes supplied
// across pool boundaries, refilling idle lanes a dozen at a time, so the
// skewed per-ray work leaves lanes idle mainly in a wave's last pool. Each ray writes
// its own T; per-Gaussian means are FP64 row sums in a fixed order
// (deterministic, no atomics).
#include <atomic>
#include <mutex>
#include <type_traits>

#include "trace_core.h"

namespace rv {
namespace {

constexpr int kTraceBlock = 256;
constexpr int kWavesPerBlock = kTraceBlock / 64;
constexpr int kXcds = 8;

// Renumber blocks so that the blocks dispatched to XCD x (b % 8 == x) form a
// contiguous range of logical blocks. A bijection on [0, nb).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t q = nb / kXcds, r = nb % kXcds;
    const int64_t x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Logical block of dispatched block b in rounds of kXcds chunks of C
// consecutive logical blocks: XCD x (b % 8 == x) takes chunk x of each round,
// so the XCDs walk the logical order side by side (each on a compact part of
// the scene at a time) and finish together; blocks past the last full round
// keep the contiguous split. A bijection on [0, nb).
template <int C>
__device__ __forceinline__ int64_t xcd_chunk_block(int64_t b, int64_t nb) {
    constexpr int64_t kRound = int64_t(kXcds) * C;
    const int64_t full = nb / kRound * kRound;
    if (b >= full) return full + xcd_block(b - full, nb - full);
    const int64_t x = b % kXcds, r = b / kXcds;
    return ((r / C) * kXcds + x) * C + r % C;
}

// Chunk of the adjoint's block order: 64 logical blocks (8 groups of 64
// Gaussians, every direction) per XCD and round. Against one contiguous eighth
// of the scene per XCD, the re-tracing adjoint runs 81.5 instead of 90.3 ms at
// object scale (200k x 128); chunks of 16 / 256 give 82.3 / 85.5 ms.
constexpr int kAdjChunk = 64;

// ---- pooled traversal -----------------------------------------------------------
//
// A wave drains pools of rays (64 Gaussians adjacent in sorted order times
// some directions, or consecutive list entries). Lanes that have no ray take
// the pool's next rays (ballot + popcount). Each iteration, lanes with
// traversal work and room in their leaf FIFO visit one node, appending hit
// leaves instead of testing them; the leaf test then runs as one block for
// all lanes with a pending leaf once enough of them have one, so the
// expensive exact test executes with most lanes active instead of inside
// every node step. Leaves are tested in discovery (FIFO) order, so each ray's
// product, and its early exit, do not depend on which pool the ray was drained
// from: the all-ray, ray-list, SH and adjoint paths give a ray the same bits.
constexpr int kPoolS = 4;
constexpr int kFifo = 8;
constexpr int kPoolRing = 8;
// The persistent all-ray and list kernels keep 16 stack entries per lane in
// LDS (24 KB per block with the FIFO, six blocks per CU): fewer deep entries
// go to the private spill array than with 8 (54.3 against 58.6 ms at object
// scale). The adjoint kernel, whose gradient table leaves no room, keeps 8.
constexpr int kStreamRing = 16;
// Directions per pool of the persistent all-ray kernel. With one, the pools
// in flight on an XCD cover the fewest Gaussians (about 256 against 1,024
// with four directions), and the tree they touch is most compact: 53.5 ms
// against 53.7 with two and 54.5 with four at object scale.
constexpr int kStreamPoolS = 1;
constexpr int kLeafMin = 32;
// Idle lanes that trigger a refill of a wave in the adjoint, unless no lane
// holds a ray (the forward kernels take Cuts::refill, set from the tree's
// size). Refilling at every finished ray ran the ray setup for one or two
// lanes nearly every iteration; waiting for 12 idle lanes costs a few lanes
// of traversal and saves most of those setups (object scale: 43.6 -> 40.4 ms,
// adjoint 59.7 -> 58.2 ms).
constexpr int kRefillMin = kRefillShallow;

struct PoolMap {
    int64_t n;
    int K, n_chunks;
    int64_t n_items;   // ceil(n / 64) * n_chunks
    int64_t n_blocks;
    int64_t w_off;     // first wave of this launch
};

// Waves per launch: a dispatch counts its work-items in 32 bits, so one grid
// stays at 2^24 waves (2^30 work-items).
constexpr int64_t kLaunchWaves = int64_t(1) << 24;

inline PoolMap make_pool(int64_t n, int K) {
    PoolMap pm;
    pm.n = n;
    pm.K = K;
    pm.n_chunks = (K + kPoolS - 1) / kPoolS;
    pm.n_items = ((n + 63) / 64) * (int64_t)pm.n_chunks;
    pm.n_blocks = (pm.n_items + kWavesPerBlock - 1) / kWavesPerBlock;
    pm.w_off = 0;
    return pm;
}

// One node visit of a pooled ray: hit leaves are appended to the lane's FIFO
// (slot order), the first hit internal child becomes the next node and the
// others are stacked to come off in slot order. The stack holds at most three
// siblings per wide level above the node, so in a tree of the bounded depth a
// visit starts with room for its three pushes; a malformed tree (visit budget
// spent, less room than that) ends the ray with NaN.
template <bool kCount, int kRing>
__device__ __forceinline__ void pool_node_step(const float4 *__restrict__ nodes4, f3 o, f3 inv, float tmin,
                                               int32_t &node, int32_t &budget, RingStack<kRing> &st,
                                               int32_t *my_fifo, int fhead, int &fcount, float &T, int64_t &cn) {
    if (--budget < 0) {
        node = -1;
        fcount = 0;
        T = __int_as_float(0x7fc00000);
        return;
    }
    int32_t id[4];
    visit4(nodes4, node, o, inv, tmin, id);
    if (kCount) ++cn;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (is_leaf(id[s])) {
            my_fifo[((fhead + fcount) & (kFifo - 1)) * kTraceBlock] = ~id[s];
            ++fcount;
        }
    }
    int32_t nxt = -1;
    const bool overflow = st.sp > kMaxStack - 3;
    if (!overflow) {
#pragma unroll
        for (int s = 3; s >= 0; --s) {
            if (id[s] >= 0) {
                if (nxt >= 0) st.push(nxt);
                nxt = id[s];
            }
        }
    }
    if (overflow) {
        node = -1;
        fcount = 0;
        T = __int_as_float(0x7fc00000);
    } else if (nxt >= 0) {
        node = nxt;
    } else if (!st.empty()) {
        node = st.pop();
    } else {
        node = -1;
    }
}

// Wave-level leaf phase condition: enough lanes hold a pending leaf, or some
// lane cannot walk for lack of FIFO room, or no lane can walk.
__device__ __forceinline__ bool leaf_phase_now(bool has, int32_t node, int fcount) {
    const uint64_t pend = __ballot(has && fcount > 0);
    const uint64_t blocked = __ballot(has && fcount > kFifo - 4);
    const uint64_t trav = __ballot(has && node >= 0 && fcount <= kFifo - 4);
    return pend != 0 && (__popcll(pend) >= kLeafMin || blocked != 0 || trav == 0);
}

// One ray as a pool source hands it out.
struct RaySetup {
    f3 o, d;
    float tmin;
    int32_t self;       // original index of the source Gaussian
    int32_t self_leaf;  // its sorted leaf position, or -1 if not known
    bool valid;         // false: not a ray of this scene (finishes at once with NaN)
    int64_t out;        // output position of its T
};

// Pools handed to one wave. XcdQueue: the pools are cut into kXcds
// contiguous ranges, one per XCD, each drained one pool at a time through an
// atomic counter (zero at launch). A wave takes from its own XCD's range
// first, so that adjacent Gaussians share that XCD's L2; once the range is
// spent it takes from the other ranges in turn, so no XCD idles while another
// still holds work. RangeQueue: a fixed run of consecutive pools.
struct XcdQueue {
    unsigned long long *ctrs;  // kXcds counters
    int64_t n_pools;
    int home, turn;  // the range being drained is (home + turn) % kXcds
    __device__ __forceinline__ void init(unsigned long long *c, int64_t np, int x) {
        ctrs = c;
        n_pools = np;
        home = x;
        turn = 0;
    }
    // Next pool in p, false once every range is spent. Called in wave-uniform
    // control flow; the first active lane takes the pool for the wave.
    __device__ __forceinline__ bool take(int64_t &p) {
        const int lane = threadIdx.x & 63;
        while (turn < kXcds) {
            const int x = (home + turn) % kXcds;
            unsigned long long t = 0;
            if (lane == __builtin_amdgcn_readfirstlane(lane)) t = atomicAdd(ctrs + x, 1ull);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)t);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(t >> 32));
            p = n_pools * x / kXcds + (int64_t)(((uint64_t)hi << 32) | lo);
            if (p < n_pools * (x + 1) / kXcds) return true;
            ++turn;
        }
        return false;
    }
};

struct RangeQueue {
    int64_t next, end;
    __device__ __forceinline__ bool take(int64_t &p) {
        p = next++;
        return p < end;
    }
};

// Trace the rays of the pools the queue hands out with the lanes of one
// wave. Once c.refill lanes are without a ray (or no lane has one), those
// lanes take the next rays of the current pool; when the pool is spent the
// wave takes the next pool at once, so lanes stay supplied across pool
// boundaries. A finished
// ray writes its T to out[r.out] (when out is given). stk and my_fifo are
// this lane's columns of the block's LDS stack ring and leaf FIFO.
template <bool kCount, class Queue, class Pools>
__device__ __forceinline__ void stream_rays(const float4 *__restrict__ nodes4, const float4 *__restrict__ rec,
                                            const Cuts &c, int64_t n, Queue &queue, Pools &pools,
                                            int32_t *stk, int32_t *my_fifo, float *__restrict__ out, int64_t &cn,
                                            int64_t &cl, int64_t &ch) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    RingStack<kStreamRing> st;
    int32_t spill[RingStack<kStreamRing>::kSpill];
    st.lds = stk;
    st.spill = spill;
    st.stride = kTraceBlock;
    st.sp = 0;
    int fhead = 0, fcount = 0;
    bool has = false;
    int64_t dst = 0;  // output position of the current ray
    f3 o = mk(0.f, 0.f, 0.f), d = o, inv = o;
    float tmin = 0.f, T = 1.f;
    int32_t self = -1, self_leaf = -1, node = -1;
    int32_t budget = 0;  // node visits left (n <= 2^30)
    NoHit none;
    // wave-uniform pool state
    int next = 0, pool_n = 0;
    bool more = true;

    while (true) {
        // refill idle lanes, moving on to further pools while lanes are idle;
        // only once c.refill lanes are idle (or none holds a ray), so that
        // the ray setup runs for several lanes at a time
        uint64_t need = __ballot(!has);
        if (__popcll(need) < c.refill && __ballot(has) != 0) need = 0;
        while (need != 0 && more) {
            if (next >= pool_n) {
                int64_t p;
                more = queue.take(p);
                pool_n = more ? pools.open(p) : 0;
                next = 0;
                continue;
            }
            const int idx = next + __popcll(need & lt);
            if (!has && idx < pool_n) {
                const RaySetup r = pools(idx);
                o = r.o;
                d = r.d;
                inv = safe_inv(d);
                tmin = r.tmin;
                self = r.self;
                self_leaf = r.self_leaf;
                T = r.valid ? 1.0f : __int_as_float(0x7fc00000);
                st.sp = 0;
                fhead = 0;
                fcount = 0;
                node = r.valid && n > 1 ? 0 : -1;
                budget = (int32_t)n;
                dst = r.out;
                has = true;
            }
            next += __popcll(need);
            need = __ballot(!has);
        }
        if (__ballot(has) == 0) break;  // queue spent, every ray finished

        // node phase: one four-wide node per lane with traversal work and FIFO
        // room for all four children
        if (has && node >= 0 && fcount <= kFifo - 4)
            pool_node_step<kCount>(nodes4, o, inv, tmin, node, budget, st, my_fifo, fhead, fcount, T, cn);

        // leaf phase: test one pending leaf per lane when enough lanes have one,
        // when a lane cannot traverse for lack of FIFO room, or when no lane can traverse
        if (leaf_phase_now(has, node, fcount)) {
            if (has && fcount > 0) {
                const int32_t leaf = my_fifo[fhead * kTraceBlock];
                fhead = (fhead + 1) & (kFifo - 1);
                --fcount;
                const float f = leaf_factor(rec, leaf, o, d, tmin, self, self_leaf, c, none, T);
                if (kCount) {
                    ++cl;
                    ch += (f != 1.0f);
                }
                T *= f;
                if (T < c.T_stop) {
                    node = -1;
                    fcount = 0;
                }
            }
        }

        if (has && node < 0 && fcount == 0) {
            if (out) out[dst] = T;
            has = false;
        }
    }
}

// Rays of the all-ray kernel: Gaussians m0 .. m0 + nv - 1 (sorted order) times
// directions k0 .. k0 + s - 1; pool index idx = j * nv + (m - m0). Origin data
// come from the prepared per-leaf records. The output position of ray
// (i, k) is i * K + k with i the Gaussian's original index.
struct GridSource {
    const float4 *rec, *origins;
    const float *dirs;
    int64_t m0;
    int nv, k0, dir_mode;
    float tmin_scale;
    float inv_nv;  // reciprocal of nv (within one ulp)
    int K = 0;
    // output position: i * K + k (by_leaf false), or (m - m_lo) * K + k with m
    // the Gaussian's sorted position (by_leaf true: rows of a batch)
    bool by_leaf = false;
    int64_t m_lo = 0;
    __device__ __forceinline__ RaySetup operator()(int idx) const {
        // idx / nv from the float quotient: (idx + 1/2) / nv lies at least
        // 1/(2 nv) >= 1/128 from an integer, far beyond its rounding error
        // (idx < 2^9: below 2^9 2^-22)
        const int j = (int)(((float)idx + 0.5f) * inv_nv);
        const int oi = idx - j * nv;
        const int64_t m = m0 + oi;
        const float4 r0 = rec[kLeafF4 * m];
        const float4 og = origins[m];
        const f3 nrm = mk(og.x, og.y, og.z);
        f3 b1, b2;
        onb_duff(nrm, b1, b2);
        RaySetup r;
        r.o = mk(r0.x, r0.y, r0.z);
        r.d = ray_direction(dirs, k0 + j, dir_mode, nrm, b1, b2);
        r.tmin = tmin_scale * og.w;
        r.self = __float_as_int(rec[kLeafF4 * m + 2].w);
        r.self_leaf = (int32_t)m;
        r.valid = true;
        r.out = (by_leaf ? m - m_lo : (int64_t)r.self) * K + k0 + j;
        return r;
    }
};

// All-ray pools: pool p = group * n_chunks + chunk covers the 64 Gaussians
// of the group (sorted order, groups counted from m_lo) times the chunk's
// kStreamPoolS directions.
struct GridPools : GridSource {
    int64_t m_hi;  // the pools cover sorted positions [m_lo, m_hi)
    int n_chunks;
    // Make pool p current; returns its number of rays.
    __device__ __forceinline__ int open(int64_t p) {
        const int64_t grp = p / n_chunks;
        const int chunk = (int)(p - grp * n_chunks);
        m0 = m_lo + grp * 64;
        nv = (int)min<int64_t>(64, m_hi - m0);
        inv_nv = __builtin_amdgcn_rcpf((float)nv);
        k0 = chunk * kStreamPoolS;
        return nv * min(kStreamPoolS, K - k0);
    }
};

// Rays given by id r = ids[base + idx] + id_offset = i * K + k. Origin data are
// recomputed from the input arrays with the same operations as the leaf
// preparation, so a ray gets the same bits as in the all-ray kernel.
struct ListSource {
    const float *mean, *normal, *log_scale, *dirs;
    int64_t n;
    int K, dir_mode;
    float tmin_scale;
    const int64_t *ids;
    int64_t id_offset, base;
    double inv_k;  // 1 / K
    bool out_by_value;
    bool tree_ok;  // the tree was built over these n Gaussians (else every ray is NaN)
    __device__ __forceinline__ RaySetup operator()(int idx) const {
        RaySetup r;
        const int64_t entry = ids[base + idx];
        const int64_t rid = entry + id_offset;
        r.out = out_by_value ? entry : base + idx;
        r.valid = tree_ok && rid >= 0 && rid < n * (int64_t)K;
        // rid / K from the FP64 quotient (off by at most one for rid < 2^52,
        // where rid converts exactly), corrected so that 0 <= k < K; integer
        // division beyond
        int64_t i = !r.valid ? 0 : rid < (int64_t(1) << 52) ? (int64_t)((double)rid * inv_k) : rid / K;
        int64_t k64 = r.valid ? rid - i * K : 0;
        if (k64 < 0) {
            --i;
            k64 += K;
        } else if (k64 >= K) {
            ++i;
            k64 -= K;
        }
        const int k = (int)k64;
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
        r.o = mk(mean[3 * i], mean[3 * i + 1], mean[3 * i + 2]);
        r.d = ray_direction(dirs, r.valid ? k : 0, dir_mode, nrm, b1, b2);
        r.tmin = tmin_scale * smax;
        r.self = (int32_t)i;
        r.self_leaf = -1;
        return r;
    }
};

// List pools: pool p covers list entries p * kPoolS * 64 onwards.
struct ListPools : ListSource {
    int64_t total;
    __device__ __forceinline__ int open(int64_t p) {
        base = p * (kPoolS * 64);
        return (int)min<int64_t>(kPoolS * 64, total - base);
    }
};

// The rays of the Gaussians at sorted positions [m_lo, m_hi) (all n K rays
// for [0, n)) through per-XCD queues of pools. The grid is persistent (a
// multiple of 8 blocks, about what the device holds at once) and block b
// serves the queue of XCD b % 8 (round-robin dispatch), whose range is a
// contiguous eighth of the pools: each L2 sees a compact part of the tree
// until its range is spent and its waves help with the other ranges.
template <bool kCount>
__global__ __launch_bounds__(kTraceBlock) void k_trace_stream(const float *__restrict__ header,
                                                              const float4 *__restrict__ nodes4,
                                                              const float4 *__restrict__ rec,
                                                              const float4 *__restrict__ origins,
                                                              const float *__restrict__ dirs, int64_t n, int K,
                                                              Cuts c, int64_t m_lo, int64_t m_hi, int by_leaf,
                                                              unsigned long long *__restrict__ queues,
                                                              float *__restrict__ vis_ray,
                                                              unsigned long long *__restrict__ totals) {
    __shared__ int32_t stk[kStreamRing * kTraceBlock];
    __shared__ int32_t fifo[kFifo * kTraceBlock];
    if (!tree_matches(header, n)) {
        // a tree built for another Gaussian set: every ray of the range is NaN
        if (vis_ray) {
            const int64_t rows = (m_hi - m_lo) * (int64_t)K;
            for (int64_t r = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x; r < rows;
                 r += (int64_t)gridDim.x * kTraceBlock)
                vis_ray[r] = __int_as_float(0x7fc00000);
        }
        return;
    }
    const int x = (int)(blockIdx.x % kXcds);
    GridPools pools;
    pools.rec = rec;
    pools.origins = origins;
    pools.dirs = dirs;
    pools.dir_mode = c.dir_mode;
    pools.tmin_scale = c.tmin_scale;
    pools.K = K;
    pools.by_leaf = by_leaf != 0;
    pools.m_lo = m_lo;
    pools.m_hi = m_hi;
    pools.n_chunks = (K + kStreamPoolS - 1) / kStreamPoolS;
    pools.m0 = 0;
    pools.nv = 1;
    pools.k0 = 0;
    pools.inv_nv = 1.0f;
    const int64_t n_pools = ((m_hi - m_lo + 63) / 64) * (int64_t)pools.n_chunks;
    XcdQueue q;
    q.init(queues, n_pools, x);
    int64_t cn = 0, cl = 0, ch = 0;
    stream_rays<kCount>(nodes4, rec, c, n, q, pools, stk + threadIdx.x, fifo + threadIdx.x, vis_ray, cn, cl, ch);
    if (kCount) {
        atomicAdd(totals + 0, (unsigned long long)cn);
        atomicAdd(totals + 1, (unsigned long long)cl);
        atomicAdd(totals + 2, (unsigned long long)ch);
    }
}

// Listed rays in pools of kPoolS * 64 list entries. The list holds *count
// entries when count is given (read on the device), else n_list.
// out_by_value: T goes to out[ids[j]] (the list holds output positions, the
// ray being id_offset + ids[j]); otherwise to out[j]. With kQueue the grid is
// persistent and takes pools from per-XCD queues (queues[8], zero at launch),
// each a contiguous eighth of the list, stealing from the others once its own
// is spent; otherwise wave w takes the run of
// pools [w R, (w + 1) R).
template <bool kQueue>
__global__ __launch_bounds__(kTraceBlock) void k_trace_list(
    const float *__restrict__ header, const float4 *__restrict__ nodes4, const float4 *__restrict__ rec, const float *__restrict__ mean,
    const float *__restrict__ normal, const float *__restrict__ log_scale, int64_t n, const float *__restrict__ dirs,
    int K, Cuts c, const int64_t *__restrict__ ids, int64_t n_list, const unsigned long long *__restrict__ count,
    int64_t id_offset, int out_by_value, int64_t run, unsigned long long *__restrict__ queues,
    float *__restrict__ out) {
    __shared__ int32_t stk[kStreamRing * kTraceBlock];
    __shared__ int32_t fifo[kFifo * kTraceBlock];
    constexpr int kPool = kPoolS * 64;
    const int64_t total = count ? min<int64_t>(n_list, (int64_t)*count) : n_list;
    const int64_t n_pools = (total + kPool - 1) / kPool;
    using Queue = typename std::conditional<kQueue, XcdQueue, RangeQueue>::type;
    Queue q;
    if constexpr (kQueue) {
        q.init(queues, n_pools, (int)(blockIdx.x % kXcds));
    } else {
        const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
        q.next = w * run;
        q.end = min(n_pools, q.next + run);
        if (q.next >= q.end) return;  // wave-uniform
    }
    ListPools pools;
    pools.mean = mean;
    pools.normal = normal;
    pools.log_scale = log_scale;
    pools.dirs = dirs;
    pools.n = n;
    pools.K = K;
    pools.dir_mode = c.dir_mode;
    pools.tmin_scale = c.tmin_scale;
    pools.ids = ids;
    pools.id_offset = id_offset;
    pools.base = 0;
    pools.inv_k = 1.0 / (double)K;
    pools.out_by_value = out_by_value != 0;
    pools.total = total;
    pools.tree_ok = tree_matches(header, n);
    int64_t cn = 0, cl = 0, ch = 0;
    stream_rays<false>(nodes4, rec, c, n, q, pools, stk + threadIdx.x, fifo + threadIdx.x, out, cn, cl, ch);
}

// vis_mean[i] = (1/K) sum_k vis[i K + k]: one wave per Gaussian, FP64 lane
// sums over a fixed stride and a fixed butterfly (deterministic).
__global__ __launch_bounds__(256) void k_mean_rows(const float *__restrict__ vis, int64_t n, int K,
                                                   float *__restrict__ vis_mean) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        const float *row = vis + i * K;
        double s = 0.0;
        for (int k = lane; k < K; k += 64) s += (double)row[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) vis_mean[i] = (float)(s / (double)K);
    }
}

// ---- visibility compressed to SH ----------------------------------------------
//
// Each Gaussian's visibility over its K directions projected onto the real
// spherical harmonics of degree <= 2 (9 coefficients, the "3-level SH" of
// Sec. 3.3) by the quadrature of Eq. (10): v_ij = sum_k V_ik Y_j(d_k) dw, with
// d_k the table's unit directions in the rays' frame (local about the normal
// in hemisphere mode). No per-ray output reaches the caller: the Gaussians are
// traced in batches of consecutive sorted positions by the persistent all-ray
// kernel into a bounded buffer of rows, and each row is projected in FP64 in a
// fixed order (deterministic).
constexpr int kShCoef = 9;
// Per-ray values held per batch: at most 2^28 (1 GiB).
constexpr int64_t kShBatchRays = int64_t(1) << 28;

// Gaussians per batch: a multiple of 64, at least 64, at most n.
inline int64_t sh_batch(int64_t n, int K) {
    int64_t b = kShBatchRays / K / 64 * 64;
    b = std::max<int64_t>(b, 64);
    return std::min<int64_t>(b, n);
}

// Real SH of degree <= 2 at the unit direction of table entry k.
__device__ __forceinline__ void sh_of_dir(const float *__restrict__ dirs, int k, float (&Y)[kShCoef]) {
    float x = dirs[3 * k], y = dirs[3 * k + 1], z = dirs[3 * k + 2];
    const float inv = 1.0f / sqrtf(x * x + y * y + z * z);
    x *= inv; y *= inv; z *= inv;
    Y[0] = 0.28209479177387814f;
    Y[1] = 0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = 0.4886025119029199f * x;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = 1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (3.0f * z * z - 1.0f);
    Y[7] = 1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (x * x - y * y);
}

// Y[k][j] = Y_j(d_k) for the K table directions.
__global__ __launch_bounds__(256) void k_sh_table(const float *__restrict__ dirs, int K, float *__restrict__ Y) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    float y[kShCoef];
    sh_of_dir(dirs, k, y);
#pragma unroll
    for (int j = 0; j < kShCoef; ++j) Y[k * kShCoef + j] = y[j];
}

// Rows m_lo .. m_lo + n_rows - 1 (sorted positions) of a traced batch: one
// wave per row adds T_k Y_j(d_k) and T_k over k in FP64, lanes over a fixed
// stride and a fixed butterfly; vis_sh and vis_mean go to the Gaussian's
// original index.
__global__ __launch_bounds__(256) void k_sh_rows(const float *__restrict__ rows, int64_t m_lo, int64_t n_rows, int K,
                                                 const float *__restrict__ Y, const float *__restrict__ header,
                                                 const float4 *__restrict__ rec, int64_t n, double dw,
                                                 float *__restrict__ vis_sh, float *__restrict__ vis_mean) {
    const int lane = threadIdx.x & 63;
    if (!tree_matches(header, n)) {
        // a tree built for another Gaussian set: NaN for the batch's rows,
        // placed by row (the batches together cover every Gaussian)
        for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n_rows; r += (int64_t)gridDim.x * 256) {
#pragma unroll
            for (int j = 0; j < kShCoef; ++j) vis_sh[(m_lo + r) * kShCoef + j] = __int_as_float(0x7fc00000);
            if (vis_mean) vis_mean[m_lo + r] = __int_as_float(0x7fc00000);
        }
        return;
    }
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n_rows; r += (int64_t)gridDim.x * 4) {
        const float *row = rows + r * K;
        double acc[kShCoef + 1];
#pragma unroll
        for (int j = 0; j <= kShCoef; ++j) acc[j] = 0.0;
        for (int k = lane; k < K; k += 64) {
            const double t = (double)row[k];
#pragma unroll
            for (int j = 0; j < kShCoef; ++j) acc[j] += t * (double)Y[k * kShCoef + j];
            acc[kShCoef] += t;
        }
#pragma unroll
        for (int j = 0; j <= kShCoef; ++j)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
        if (lane == 0) {
            const int64_t i = __float_as_int(rec[kLeafF4 * (m_lo + r) + 2].w);
#pragma unroll
            for (int j = 0; j < kShCoef; ++j) vis_sh[i * kShCoef + j] = (float)(acc[j] * dw);
            if (vis_mean) vis_mean[i] = (float)(acc[kShCoef] / (double)K);
        }
    }
}

// ---- adjoint ----------------------------------------------------------------

// Per-block accumulation table of the scatter: the four waves of a block
// trace 64 adjacent origins x 16 directions, whose hits concentrate on the
// same nearby Gaussians, so their seven sums are added in LDS and flushed
// with one set of global atomics per Gaussian at the end of the block. Hits
// whose Gaussian finds no slot are kept as records in a buffer of the block's
// own; once the table is flushed, a second pass sums the records per Gaussian
// in the emptied table and flushes it again.
// A Gaussian tries kHashProbes consecutive slots before its hit goes to the
// global atomics: once the table has filled, every further probe is a
// compare-and-swap that cannot succeed (2 / 4 / 8 / 16 probes: 59.5 / 57.7 /
// 57.8 / 60.9 ms with the forward's T, 88.3 / 90.2 / 94.6 / 104.0 ms
// re-tracing).
constexpr int kHashSlots = 1024;
// Record buffers for the hits that overflow a block's table: more buffers
// than blocks can be resident (3 per CU), 8,192 records (256 KB) each, 256 MB
// in all. Against seven device atomics per overflowing hit, the second pass
// takes the adjoint with the forward's T from 57.3 to 50.6 ms at object scale
// (200k x 128; 4,096 records: 51.7 ms, 16,384: 51.8 ms; 16 or 32 probes in the
// second pass: no change).
constexpr int kOvfSlots = 1024, kOvfCap = 8192;
constexpr int kHashProbes = 4;

struct GradTable {
    int32_t key[kHashSlots];         // Gaussian index, -1 when free
    float val[7][kHashSlots];        // opacity, mean xyz, log-scale xyz

    // Slot of Gaussian j (claimed if free), or -1 after kHashProbes probes.
    __device__ __forceinline__ int find(int32_t j) {
        const uint32_t h = ((uint32_t)j * 2654435761u) >> 22;   // 10 bits
#pragma unroll
        for (int p = 0; p < kHashProbes; ++p) {
            const int s = (int)((h + p) & (kHashSlots - 1));
            const int32_t k = atomicCAS(&key[s], -1, j);
            if (k == -1 || k == j) return s;
        }
        return -1;
    }
};

// Seven sums of Gaussian j added with device-scope atomics.
__device__ __forceinline__ void add_grad_global(float *go, float *gm, float *gl, int64_t j, const float (&v)[7]) {
    unsafeAtomicAdd(go + j, v[0]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        unsafeAtomicAdd(gm + 3 * j + c, v[1 + c]);
        unsafeAtomicAdd(gl + 3 * j + c, v[4 + c]);
    }
}

struct GradScatter {
    bool active;        // false on the pass that only recovers T_final
    float g_over;       // -(dL/dT) * T_final for the current ray
    float *go, *gm, *gl;
    GradTable *table;
    f3 origin;          // accumulated d/d(origin) of the current ray
    // the block's overflow records (two float4 each: source index and the
    // seven sums), or null; *ovf_n counts the records claimed (LDS)
    float4 *ovf;
    int *ovf_n;
    int ovf_cap;

    __device__ __forceinline__ void operator()(const LeafHit &h, float) {
        if (!active || h.clamped) return;
        const float ga = g_over / h.one_minus;   // dL/dalpha
        const float a = ga * h.alpha;
        const f3 wte = h.e.x * h.w0 + h.e.y * h.w1 + h.e.z * h.w2;   // W^T e
        const float v[7] = {a / h.opacity, a * wte.x, a * wte.y, a * wte.z,
                            a * h.e.x * h.e.x, a * h.e.y * h.e.y, a * h.e.z * h.e.z};
        const int slot = table->find(h.src);
        if (slot >= 0) {
#pragma unroll
            for (int c = 0; c < 7; ++c) atomicAdd(&table->val[c][slot], v[c]);
        } else {
            // no slot: keep the hit for the block's second pass when its
            // record buffer has room, else add it to the gradients at once
            const int r = ovf ? atomicAdd(ovf_n, 1) : ovf_cap;
            if (r < ovf_cap) {
                ovf[2 * r] = make_float4(__int_as_float(h.src), v[0], v[1], v[2]);
                ovf[2 * r + 1] = make_float4(v[3], v[4], v[5], v[6]);
            } else {
                add_grad_global(go, gm, gl, h.src, v);
            }
        }
        origin = origin - a * wte;
    }
};

// Adjoint over the same pools as the forward (64 Gaussians x a chunk of
// directions per wave). Each ray with a nonzero upstream gradient
// g = dL/dV_ik (grad_ray) + dL/dVbar_i / K (grad_mean) is traced once to
// recover T_final (skipped when the forward's T are given), then again with
// the same visits in the same order, scattering dL/dalpha_j = -g T_final /
// (1 - alpha_j) into each included, unclamped Gaussian's parameters (through
// the block's LDS table and its overflow records). The source's own term
// (through the ray origin) is summed per Gaussian in LDS and added once per
// wave. ovf_buf holds ovf_slots record buffers of ovf_cap records, each owned
// by the block that claimed its flag in ovf_flags (zero when free); null:
// every overflowing hit is added at once.
__global__ __launch_bounds__(kTraceBlock) void k_trace_backward(
    const float *__restrict__ header, const float4 *__restrict__ nodes4, const float4 *__restrict__ rec, const float4 *__restrict__ origins,
    const float *__restrict__ dirs, PoolMap pm, Cuts c, const float *__restrict__ grad_ray,
    const float *__restrict__ grad_mean_in, const float *__restrict__ vis_fwd, float *go, float *gm, float *gl,
    float4 *ovf_buf, uint32_t *ovf_flags, int ovf_slots, int ovf_cap) {
    __shared__ int32_t stk[kPoolRing * kTraceBlock];
    __shared__ int32_t fifo[kFifo * kTraceBlock];
    __shared__ float ogr[kWavesPerBlock][64 * 3];   // origin terms per item
    __shared__ GradTable table;
    // the block's four items (64 Gaussians x a chunk of directions each),
    // drained together: item sizes, their Gaussians and first directions
    __shared__ int item_n[kWavesPerBlock], item_nv[kWavesPerBlock], item_k0[kWavesPerBlock];
    __shared__ int64_t item_m0[kWavesPerBlock];
    __shared__ int blk_next;
    __shared__ int ovf_slot, ovf_n;   // the block's record buffer (-1: none) and its records
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (!tree_matches(header, pm.n)) {
        // a tree built for another Gaussian set: every gradient is NaN
        const float nan = __int_as_float(0x7fc00000);
        for (int64_t j = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x; j < pm.n;
             j += (int64_t)gridDim.x * kTraceBlock) {
            go[j] = nan;
#pragma unroll
            for (int c = 0; c < 3; ++c) gm[3 * j + c] = gl[3 * j + c] = nan;
        }
        return;
    }
    for (int s = threadIdx.x; s < kHashSlots; s += kTraceBlock) {
        table.key[s] = -1;
#pragma unroll
        for (int c = 0; c < 7; ++c) table.val[c][s] = 0.0f;
    }
    if (threadIdx.x == 0) {
        // claim a free record buffer: at most one pass over the flags, so a
        // block never waits on another (without one, overflow goes out at once)
        int got = -1;
        if (ovf_buf) {
            const int start = (int)(blockIdx.x % (unsigned)ovf_slots);
            for (int i = 0; i < ovf_slots && got < 0; ++i) {
                const int sl = start + i < ovf_slots ? start + i : start + i - ovf_slots;
                if (atomicCAS(ovf_flags + sl, 0u, 1u) == 0u) got = sl;
            }
        }
        ovf_slot = got;
        ovf_n = 0;
    }
    // item wv: every wave reaches the barriers; items past the end are empty
    int64_t w = pm.w_off + xcd_chunk_block<kAdjChunk>(blockIdx.x, gridDim.x) * kWavesPerBlock + wv;
    const bool wave_live = w < pm.n_items;
    if (!wave_live) w = 0;
    const int64_t grp = w / pm.n_chunks;
    const int chunk = (int)(w - grp * pm.n_chunks);
    const int64_t my_m0 = grp * 64;
    const int my_nv = (int)min<int64_t>(64, pm.n - my_m0);
    const int K = pm.K;
    if (lane == 0) {
        item_n[wv] = wave_live ? my_nv * min(kPoolS, K - chunk * kPoolS) : 0;
        item_nv[wv] = my_nv;
        item_k0[wv] = chunk * kPoolS;
        item_m0[wv] = my_m0;
    }
    if (threadIdx.x == 0) blk_next = 0;
    ogr[wv][lane] = 0.f;
    ogr[wv][64 + lane] = 0.f;
    ogr[wv][128 + lane] = 0.f;
    __syncthreads();
    // block ray r: item it with n_0 + .. + n_(it-1) <= r, local index r - that sum
    const int n_a = item_n[0], n_b = n_a + item_n[1], n_c = n_b + item_n[2], total = n_c + item_n[3];
    GridSource src;
    src.rec = rec;
    src.origins = origins;
    src.dirs = dirs;
    src.dir_mode = c.dir_mode;
    src.tmin_scale = c.tmin_scale;
    src.K = K;

    const uint64_t lt = (1ull << lane) - 1ull;
    RingStack<kPoolRing> st;
    int32_t spill[RingStack<kPoolRing>::kSpill];
    st.lds = stk + threadIdx.x;
    st.spill = spill;
    st.stride = kTraceBlock;
    st.sp = 0;
    int32_t *my_fifo = fifo + threadIdx.x;
    int fhead = 0, fcount = 0;
    bool has = false;
    int oi = 0, it = 0;  // item and item origin of the current ray
    float gk = 0.f;      // upstream gradient of the current ray
    f3 o = mk(0.f, 0.f, 0.f), d = o, inv = o;
    float tmin = 0.f, T = 1.f;
    int32_t self = -1, self_leaf = -1, node = -1;
    int32_t budget = 0;
    int64_t cn = 0;
    GradScatter gs;
    gs.active = false;
    gs.g_over = 0.f;
    gs.go = go;
    gs.gm = gm;
    gs.gl = gl;
    gs.table = &table;
    gs.origin = mk(0.f, 0.f, 0.f);
    gs.ovf = ovf_slot >= 0 ? ovf_buf + 2 * (int64_t)ovf_slot * ovf_cap : nullptr;
    gs.ovf_n = &ovf_n;
    gs.ovf_cap = ovf_cap;
    bool drained = false;  // wave-uniform: the block's rays are all handed out
    auto restart = [&]() {
        T = 1.0f;
        st.sp = 0;
        fhead = 0;
        fcount = 0;
        node = pm.n > 1 ? 0 : -1;
        budget = (int32_t)pm.n;
    };

    while (true) {
        const uint64_t need = __ballot(!has);
        if (need != 0 && !drained && (__popcll(need) >= kRefillMin || __ballot(has) == 0)) {
            // the wave's first active lane reserves one block ray per idle lane
            const int cnt = __popcll(need);
            int base = 0;
            if (lane == __builtin_amdgcn_readfirstlane(lane)) base = atomicAdd(&blk_next, cnt);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base + cnt >= total) drained = true;
            const int idx = base + __popcll(need & lt);
            if (!has && idx < total) {
                it = (idx >= n_a) + (idx >= n_b) + (idx >= n_c);
                const int local = idx - (it == 0 ? 0 : it == 1 ? n_a : it == 2 ? n_b : n_c);
                src.m0 = item_m0[it];
                src.nv = item_nv[it];
                src.inv_nv = __builtin_amdgcn_rcpf((float)src.nv);
                src.k0 = item_k0[it];
                const RaySetup r = src(local);
                oi = (int)(r.self_leaf - src.m0);
                // r.out = i K + k: the ray's place in grad_ray and vis_fwd
                gk = (grad_mean_in ? grad_mean_in[r.self] / (float)K : 0.0f) + (grad_ray ? grad_ray[r.out] : 0.0f);
                o = r.o;
                d = r.d;
                inv = safe_inv(d);
                tmin = r.tmin;
                self = r.self;
                self_leaf = r.self_leaf;
                restart();
                gs.origin = mk(0.f, 0.f, 0.f);
                gs.active = vis_fwd != nullptr;
                gs.g_over = vis_fwd ? -gk * vis_fwd[r.out] : 0.0f;
                if (gk == 0.0f) {   // nothing to propagate: the ray ends here
                    node = -1;
                    gs.active = true;
                }
                has = true;
            }
        }
        if (__ballot(has) == 0) break;

        if (has && node >= 0 && fcount <= kFifo - 4)
            pool_node_step<false>(nodes4, o, inv, tmin, node, budget, st, my_fifo, fhead, fcount, T, cn);

        if (leaf_phase_now(has, node, fcount)) {
            if (has && fcount > 0) {
                const int32_t leaf = my_fifo[fhead * kTraceBlock];
                fhead = (fhead + 1) & (kFifo - 1);
                --fcount;
                T *= leaf_factor(rec, leaf, o, d, tmin, self, self_leaf, c, gs, T);
                if (T < c.T_stop) {
                    node = -1;
                    fcount = 0;
                }
            }
        }

        if (has && node < 0 && fcount == 0) {
            if (!gs.active) {
                // T_final is known: trace the same ray again, scattering
                gs.g_over = -gk * T;
                gs.active = true;
                restart();
            } else {
                if (gs.origin.x != 0.f || gs.origin.y != 0.f || gs.origin.z != 0.f) {
                    atomicAdd(&ogr[it][3 * oi + 0], gs.origin.x);
                    atomicAdd(&ogr[it][3 * oi + 1], gs.origin.y);
                    atomicAdd(&ogr[it][3 * oi + 2], gs.origin.z);
                }
                has = false;
            }
        }
    }
    // every wave has finished: the origin sums of all items and the table
    // are complete
    __syncthreads();
    if (wave_live && lane < my_nv) {
        const float ox = ogr[wv][3 * lane], oy = ogr[wv][3 * lane + 1], oz = ogr[wv][3 * lane + 2];
        if (ox != 0.f || oy != 0.f || oz != 0.f) {
            const int64_t j = __float_as_int(rec[kLeafF4 * (my_m0 + lane) + 2].w);
            unsafeAtomicAdd(gm + 3 * j + 0, ox);
            unsafeAtomicAdd(gm + 3 * j + 1, oy);
            unsafeAtomicAdd(gm + 3 * j + 2, oz);
        }
    }
    // the block's table: one set of global atomics per Gaussian
    auto flush_table = [&]() {
        for (int s = threadIdx.x; s < kHashSlots; s += kTraceBlock) {
            const int64_t j = table.key[s];
            if (j < 0) continue;
            const float v[7] = {table.val[0][s], table.val[1][s], table.val[2][s], table.val[3][s],
                                table.val[4][s], table.val[5][s], table.val[6][s]};
            add_grad_global(go, gm, gl, j, v);
        }
    };
    flush_table();
    if (ovf_slot < 0) return;   // block-uniform
    // second pass: the hits that found no slot, summed per Gaussian in the
    // emptied table (most of them now fit), then flushed once more
    __syncthreads();
    for (int s = threadIdx.x; s < kHashSlots; s += kTraceBlock) {
        table.key[s] = -1;
#pragma unroll
        for (int c = 0; c < 7; ++c) table.val[c][s] = 0.0f;
    }
    __syncthreads();
    const float4 *rec_ovf = ovf_buf + 2 * (int64_t)ovf_slot * ovf_cap;
    const int n_rec = min(ovf_n, ovf_cap);
    for (int r = threadIdx.x; r < n_rec; r += kTraceBlock) {
        const float4 a = rec_ovf[2 * r], b = rec_ovf[2 * r + 1];
        const int32_t j = __float_as_int(a.x);
        const float v[7] = {a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        const int slot = table.find(j);
        if (slot >= 0) {
#pragma unroll
            for (int c = 0; c < 7; ++c) atomicAdd(&table.val[c][slot], v[c]);
        } else {
            add_grad_global(go, gm, gl, j, v);
        }
    }
    __syncthreads();
    flush_table();
    // every record has been read: hand the buffer back
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) atomicExch(ovf_flags + ovf_slot, 0u);
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


// Resident blocks per CU of the persistent traversal. Every wave in flight
// keeps its pools' part of the tree in the XCD's L2, so more waves hide more
// latency but thin the L2 out; six blocks (24 waves) per CU gave the shortest
// object-scale trace (58.8 ms, against 63.0 at the eight the registers allow
// and 68.0 at four).
constexpr int kStreamBlocksPerCu = 6;

// Blocks of a persistent traversal grid: what the device holds at once, up
// to kStreamBlocksPerCu per CU (a multiple of 8, at least 8: every XCD queue
// has blocks), no more than the pools need.
int64_t stream_blocks(int64_t n_pools) {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    int nb = (dev >= 0 && dev < 64) ? cached[dev].load() : 0;
    if (nb <= 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev < 0 ? 0 : dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_stream<false>, kTraceBlock, 0) !=
                hipSuccess ||
            per_cu <= 0)
            per_cu = 4;
        (void)hipGetLastError();  // a failed query above must not surface as a launch error
        nb = cus * std::min(per_cu, kStreamBlocksPerCu);
        if (dev >= 0 && dev < 64) cached[dev].store(nb);
    }
    int64_t want = std::min<int64_t>(nb, (n_pools + kWavesPerBlock - 1) / kWavesPerBlock);
    want = (want + kXcds - 1) / kXcds * kXcds;
    return std::max<int64_t>(want, kXcds);
}

// Waves of the list kernel beyond which each wave takes a run of several
// pools (about four times what the device holds at once).
constexpr int64_t kListTargetWaves = 32768;

}  // namespace

void launch_trace_list(const void *bvh, const rv_gaussians *g, const float *dirs, int K, const Cuts &c,
                       const int64_t *ids, int64_t n_list, const unsigned long long *count, int64_t id_offset,
                       bool out_by_value, float *out, unsigned long long *queues, hipStream_t stream) {
    if (n_list <= 0) return;
    const BvhLayout L = bvh_layout(g->n);
    const int64_t pools = (n_list + kPoolS * 64 - 1) / (kPoolS * 64);
    Cuts cc = c;
    cc.refill = refill_lanes(g->n);
    if (queues) {
        hipLaunchKernelGGL(k_fill_u32_trace, dim3(1), dim3(64), 0, stream, reinterpret_cast<uint32_t *>(queues),
                           (int64_t)(2 * kXcds), 0u);
        hipLaunchKernelGGL(k_trace_list<true>, dim3((unsigned)stream_blocks(pools)), dim3(kTraceBlock), 0, stream,
                           at<float>(bvh, L.header), at<float4>(bvh, L.nodes4), at<float4>(bvh, L.leaf_rec), g->mean,
                           c.dir_mode ? g->normal : nullptr, g->log_scale, g->n, dirs, K, cc, ids, n_list, count,
                           id_offset, out_by_value ? 1 : 0, (int64_t)0, queues, out);
        return;
    }
    const int64_t run = (pools + kListTargetWaves - 1) / kListTargetWaves;
    const int64_t waves = (pools + run - 1) / run;
    hipLaunchKernelGGL(k_trace_list<false>, dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock)),
                       dim3(kTraceBlock), 0, stream, at<float>(bvh, L.header), at<float4>(bvh, L.nodes4),
                       at<float4>(bvh, L.leaf_rec), g->mean,
                       c.dir_mode ? g->normal : nullptr, g->log_scale, g->n, dirs, K, cc, ids, n_list, count, id_offset,
                       out_by_value ? 1 : 0, run, (unsigned long long *)nullptr, out);
}

}  // namespace rv

using namespace rv;

extern "C" size_t rv_trace_workspace_bytes(int64_t n, int32_t K) {
    if (n < 1 || K < 1) return kAlign;
    return kAlign + align_up((size_t)n * (size_t)K * sizeof(float));
}

namespace {

// The persistent all-ray traversal: clear the XCD queues (first 64 bytes of
// ws), then trace every ray (writing vis_ray when given, counters into totals
// when counting).
template <bool kCount>
void launch_trace_stream(const void *bvh, const rv_gaussians *g, const float *dirs, int K, const Cuts &c,
                         void *ws, float *vis_ray, unsigned long long *totals, hipStream_t s, int64_t m_lo = 0,
                         int64_t m_hi = -1, bool by_leaf = false) {
    const BvhLayout L = bvh_layout(g->n);
    if (m_hi < 0) m_hi = g->n;
    const int64_t n_pools = ((m_hi - m_lo + 63) / 64) * (int64_t)((K + kStreamPoolS - 1) / kStreamPoolS);
    auto *queues = static_cast<unsigned long long *>(ws);
    hipLaunchKernelGGL(k_fill_u32_trace, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(queues),
                       (int64_t)(2 * kXcds), 0u);
    Cuts cc = c;
    cc.refill = refill_lanes(g->n);
    hipLaunchKernelGGL(k_trace_stream<kCount>, dim3((unsigned)stream_blocks(n_pools)), dim3(kTraceBlock), 0, s,
                       at<float>(bvh, L.header), at<float4>(bvh, L.nodes4), at<float4>(bvh, L.leaf_rec), at<float4>(bvh, L.origins), dirs, g->n,
                       K, cc, m_lo, m_hi, by_leaf ? 1 : 0, queues, vis_ray, totals);
}

// Enqueue the all-ray trace with its scratch at ws (256-byte aligned: the
// queue counters, then the per-ray values when vis_ray is NULL).
void trace_visibility_into(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                           const rv_trace_params *p, float *vis_ray, float *vis_mean, void *ws, hipStream_t s) {
    // the per-ray values go to vis_ray, else to the workspace after the queues
    float *rays = vis_ray ? vis_ray : reinterpret_cast<float *>(static_cast<char *>(ws) + kAlign);
    launch_trace_stream<false>(bvh, g, dirs, K, make_cuts(*p), ws, rays, nullptr, s);
    if (vis_mean) {
        const int64_t blocks = std::min<int64_t>((g->n + 3) / 4, int64_t(1) << 20);
        hipLaunchKernelGGL(k_mean_rows, dim3((unsigned)blocks), dim3(256), 0, s, rays, g->n, K, vis_mean);
    }
}

// ---- scratch of the allocation-free entry point ---------------------------
//
// One array per device, held until the process ends: the queue counters and,
// for calls without per-ray output, the per-ray values. In host code the
// array's name is a host-side stand-in, never a device address: its device
// address is looked up once per device (with that device current) and only
// that address is passed on.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch (looked up on its first use).
rv_status static_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    RV_REQUIRE(e == hipSuccess && dev >= 0 && dev < kMaxDevices, RV_ERR_HIP,
               "rv_trace_visibility_static: no current device (HIP error %d)", (int)e);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        RV_REQUIRE(e == hipSuccess && ptr, RV_ERR_HIP,
                   "rv_trace_visibility_static: hipGetSymbolAddress of the scratch failed on device %d: %s", dev,
                   hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RV_OK;
}

}  // namespace

extern "C" rv_status rv_trace_visibility(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                         const rv_trace_params *p, float *vis_ray, float *vis_mean, void *ws,
                                         size_t ws_bytes, void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_visibility", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(vis_ray || vis_mean, RV_ERR_INVALID_ARG, "rv_trace_visibility: both outputs are NULL");
    RV_REQUIRE(ws && ((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG,
               "rv_trace_visibility: needs a 256-byte aligned workspace");
    const size_t need = vis_ray ? kAlign : rv_trace_workspace_bytes(g->n, K);
    RV_REQUIRE(ws_bytes >= need, RV_ERR_WORKSPACE, "rv_trace_visibility: ws_bytes %zu < %zu", ws_bytes, need);
    trace_visibility_into(bvh, g, dirs, K, p, vis_ray, vis_mean, ws, (hipStream_t)stream);
    return check_launch("rv_trace_visibility");
}

extern "C" size_t rv_trace_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" rv_status rv_trace_visibility_static(const void *bvh, const rv_gaussians *g, const float *dirs,
                                                int32_t K, const rv_trace_params *p, float *vis_ray,
                                                float *vis_mean, void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_visibility_static", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(vis_ray || vis_mean, RV_ERR_INVALID_ARG, "rv_trace_visibility_static: both outputs are NULL");
    const size_t need = vis_ray ? kAlign : rv_trace_workspace_bytes(g->n, K);
    RV_REQUIRE(need <= kStaticScratchBytes, RV_ERR_WORKSPACE,
               "rv_trace_visibility_static: without vis_ray the %lld x %d per-ray values need %zu bytes of scratch, "
               "more than the %zu-byte static scratch (at most %zu rays; pass vis_ray or use rv_trace_visibility)",
               (long long)g->n, K, need, kStaticScratchBytes, (kStaticScratchBytes - kAlign) / sizeof(float));
    void *ws = nullptr;
    st = static_scratch(&ws);
    if (st != RV_OK) return st;
    trace_visibility_into(bvh, g, dirs, K, p, vis_ray, vis_mean, ws, (hipStream_t)stream);
    return check_launch("rv_trace_visibility_static");
}

extern "C" rv_status rv_trace_stats(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                    const rv_trace_params *p, int64_t *totals, void *ws, size_t ws_bytes,
                                    void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_stats", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(totals, RV_ERR_INVALID_ARG, "rv_trace_stats: null totals");
    RV_REQUIRE(ws && ((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG,
               "rv_trace_stats: needs a 256-byte aligned workspace");
    RV_REQUIRE(ws_bytes >= kAlign, RV_ERR_WORKSPACE, "rv_trace_stats: ws_bytes %zu < %zu", ws_bytes, kAlign);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_u32_trace, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(totals), (int64_t)6,
                       0u);
    launch_trace_stream<true>(bvh, g, dirs, K, make_cuts(*p), ws, nullptr, (unsigned long long *)totals, s);
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
    launch_trace_list(bvh, g, dirs, K, make_cuts(*p), ray_ids, n_rays, nullptr, 0, false, out, nullptr,
                      (hipStream_t)stream);
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
    const PoolMap pm = make_pool(g->n, K);
    const BvhLayout L = bvh_layout(g->n);
    const Cuts c = make_cuts(*p);
    // record buffers of the blocks' second pass (stream-ordered, freed after
    // the launches); without them every overflowing hit goes out at once
    hipStream_t s = (hipStream_t)stream;
    const size_t flag_bytes = align_up((size_t)kOvfSlots * sizeof(uint32_t));
    const size_t ovf_bytes = flag_bytes + (size_t)kOvfSlots * kOvfCap * 2 * sizeof(float4);
    void *ovf_mem = nullptr;
    if (hipMallocAsync(&ovf_mem, ovf_bytes, s) != hipSuccess) {
        ovf_mem = nullptr;
        (void)hipGetLastError();
    }
    uint32_t *ovf_flags = static_cast<uint32_t *>(ovf_mem);
    float4 *ovf_buf = ovf_mem ? reinterpret_cast<float4 *>(static_cast<char *>(ovf_mem) + flag_bytes) : nullptr;
    if (ovf_mem) hipLaunchKernelGGL(k_fill_u32_trace, dim3(1), dim3(64), 0, s, ovf_flags, (int64_t)kOvfSlots, 0u);
    for (int64_t w0 = 0; w0 < pm.n_items; w0 += kLaunchWaves) {
        PoolMap part = pm;
        part.w_off = w0;
        const int64_t nb = (std::min(kLaunchWaves, pm.n_items - w0) + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL(k_trace_backward, dim3((unsigned)nb), dim3(kTraceBlock), 0, s,
                           at<float>(bvh, L.header), at<float4>(bvh, L.nodes4), at<float4>(bvh, L.leaf_rec), at<float4>(bvh, L.origins), dirs,
                           part, c, grad_vis_ray, grad_vis_mean, vis_ray_fwd, grad_opacity, grad_mean, grad_log_scale,
                           ovf_buf, ovf_flags, kOvfSlots, kOvfCap);
    }
    const rv_status st_launch = check_launch("rv_trace_visibility_backward");
    if (ovf_mem) (void)hipFreeAsync(ovf_mem, s);
    return st_launch;
}

extern "C" size_t rv_trace_sh_workspace_bytes(int64_t n, int32_t K) {
    if (n < 1 || K < 1) return 0;
    return kAlign + align_up((size_t)K * kShCoef * sizeof(float)) +
           align_up((size_t)sh_batch(n, K) * (size_t)K * sizeof(float));
}

extern "C" rv_status rv_trace_visibility_sh(const void *bvh, const rv_gaussians *g, const float *dirs, int32_t K,
                                            const rv_trace_params *p, float *vis_sh, float *vis_mean, void *ws,
                                            size_t ws_bytes, void *stream) {
    clear_error();
    rv_status st = validate_trace("rv_trace_visibility_sh", bvh, g, dirs, K, p);
    if (st != RV_OK) return st;
    RV_REQUIRE(vis_sh, RV_ERR_INVALID_ARG, "rv_trace_visibility_sh: null vis_sh");
    const size_t need = rv_trace_sh_workspace_bytes(g->n, K);
    RV_REQUIRE(ws && ((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG,
               "rv_trace_visibility_sh: ws missing or unaligned");
    RV_REQUIRE(ws_bytes >= need, RV_ERR_WORKSPACE, "rv_trace_visibility_sh: ws_bytes %zu < %zu", ws_bytes, need);
    // ws: queue counters | Y table [K][9] | rows of one batch [batch][K]
    float *Y = reinterpret_cast<float *>(static_cast<char *>(ws) + kAlign);
    float *rows = reinterpret_cast<float *>(static_cast<char *>(ws) + kAlign +
                                            align_up((size_t)K * kShCoef * sizeof(float)));
    const BvhLayout L = bvh_layout(g->n);
    const Cuts c = make_cuts(*p);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sh_table, dim3(grid_for(K, 256)), dim3(256), 0, s, dirs, (int)K, Y);
    const double dw = (p->dir_mode ? 2.0 : 4.0) * 3.14159265358979323846 / (double)K;
    const int64_t batch = sh_batch(g->n, K);
    for (int64_t m_lo = 0; m_lo < g->n; m_lo += batch) {
        const int64_t m_hi = std::min(g->n, m_lo + batch);
        launch_trace_stream<false>(bvh, g, dirs, K, c, ws, rows, nullptr, s, m_lo, m_hi, true);
        const int64_t blocks = std::min<int64_t>((m_hi - m_lo + 3) / 4, int64_t(1) << 20);
        hipLaunchKernelGGL(k_sh_rows, dim3((unsigned)blocks), dim3(256), 0, s, rows, m_lo, m_hi - m_lo, (int)K, Y,
                           at<float>(bvh, L.header), at<float4>(bvh, L.leaf_rec), g->n, dw, vis_sh, vis_mean);
    }
    return check_launch("rv_trace_visibility_sh");
}
