// copy.hip -- measurement kernels: the streaming copy (achievable HBM
// bandwidth, and the known-size reference for hardware byte counters) and the
// record-gather probe (achievable rate of the traversal's access pattern:
// divergent 16-byte lane loads of 48-byte records from an L2-resident table).
#include "rv_internal.h"

namespace rv {
namespace {

constexpr int kCopyBlock = 256;
constexpr int kCopyUnroll = 4;      // 16-byte vectors in flight per thread
constexpr int kCopyBlocksPerCu = 64;  // grid cap: 16,384 blocks on 256 CUs
// a native 16-byte vector (the non-temporal builtins take no struct types)
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

// Each thread moves kCopyUnroll 16-byte vectors per iteration with
// non-temporal loads and stores (the data is touched once), grid-stride over
// chunks of kCopyUnroll * blockDim vectors so that a wave's loads are
// contiguous. Measured on 2 GiB: 4 vectors in flight and 64 blocks per CU
// move 5.75 TB/s (8 vectors and 8 blocks per CU: 5.35; without the
// non-temporal hint: 5.38).
__global__ __launch_bounds__(kCopyBlock) void k_stream_copy(const v4u32 *__restrict__ src, v4u32 *__restrict__ dst,
                                                            int64_t n16) {
    const int64_t chunk = (int64_t)kCopyUnroll * kCopyBlock;
    const int64_t n_full = n16 / chunk;
    for (int64_t c = blockIdx.x; c < n_full; c += gridDim.x) {
        const int64_t base = c * chunk + threadIdx.x;
        v4u32 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + base + u * kCopyBlock);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + base + u * kCopyBlock);
    }
    // the tail (fewer than one chunk): plain grid-stride
    for (int64_t i = n_full * chunk + (int64_t)blockIdx.x * kCopyBlock + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * kCopyBlock)
        dst[i] = src[i];
}

// Read-only stream: the same chunking, each thread folding what it reads
// into one word (stored once, so nothing is optimised away): the achievable
// read bandwidth, the denominator for kernels whose HBM traffic is reads
// (6.54 TB/s measured on 2 GiB, against 5.06 TB/s for writes alone).
__global__ __launch_bounds__(kCopyBlock) void k_stream_read(const v4u32 *__restrict__ src, int64_t n16,
                                                            uint32_t *__restrict__ sink) {
    const int64_t chunk = (int64_t)kCopyUnroll * kCopyBlock;
    const int64_t n_full = n16 / chunk;
    v4u32 acc = {0u, 0u, 0u, 0u};
    for (int64_t c = blockIdx.x; c < n_full; c += gridDim.x) {
        const int64_t base = c * chunk + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) acc ^= __builtin_nontemporal_load(src + base + u * kCopyBlock);
    }
    for (int64_t i = n_full * chunk + (int64_t)blockIdx.x * kCopyBlock + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * kCopyBlock)
        acc ^= src[i];
    sink[(int64_t)blockIdx.x * kCopyBlock + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// Record-gather probe: every lane reads `rounds` records of three 16-byte
// words from a table of n_rec records (48 bytes used of 64), at indices drawn
// independently per lane and round from a counter-based hash, so the lanes of
// a wave diverge as traversal lanes do, and `kProbeBatch` records are in
// flight per lane. The XOR of everything read goes to sink[thread] so nothing
// is optimised away.
constexpr int kProbeBatch = 4;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // a 32-bit integer hash of xorshift-multiply rounds (the "lowbias32"
    // constants of C. Wellons' published hash-prospector search)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void k_gather_probe(const uint4 *__restrict__ table, uint32_t n_rec, int rounds,
                                                      uint32_t *__restrict__ sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (int r = 0; r < rounds; r += kProbeBatch) {
        uint32_t idx[kProbeBatch];
#pragma unroll
        for (int b = 0; b < kProbeBatch; ++b) idx[b] = mix32(tid * 0x9e3779b9u + (uint32_t)(r + b)) % n_rec;
        uint4 w[kProbeBatch][3];
#pragma unroll
        for (int b = 0; b < kProbeBatch; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) w[b][k] = table[4 * (size_t)idx[b] + k];
#pragma unroll
        for (int b = 0; b < kProbeBatch; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc.x ^= w[b][k].x;
                acc.y ^= w[b][k].y;
                acc.z ^= w[b][k].z;
                acc.w ^= w[b][k].w;
            }
    }
    sink[tid] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// Blocks of a streaming launch: up to kCopyBlocksPerCu per CU on 256 CUs, no
// more than the chunks need.
inline unsigned copy_grid(int64_t n16) {
    const int64_t chunks = (n16 + kCopyUnroll * kCopyBlock - 1) / (kCopyUnroll * kCopyBlock);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(chunks, 256 * kCopyBlocksPerCu));
}

}  // namespace
}  // namespace rv

using namespace rv;

extern "C" size_t rv_stream_read_sink_words(size_t bytes) {
    return (size_t)copy_grid((int64_t)(bytes / 16)) * kCopyBlock;
}

extern "C" rv_status rv_stream_read(const void *src, size_t bytes, uint32_t *sink, void *stream) {
    clear_error();
    RV_REQUIRE(src && sink, RV_ERR_INVALID_ARG, "rv_stream_read: null pointer");
    RV_REQUIRE(bytes % 16 == 0 && bytes > 0 && ((uintptr_t)src % 16) == 0, RV_ERR_INVALID_ARG,
               "rv_stream_read: size must be a positive multiple of 16 bytes and src 16-byte aligned");
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(k_stream_read, dim3(copy_grid(n16)), dim3(kCopyBlock), 0, (hipStream_t)stream,
                       static_cast<const v4u32 *>(src), n16, sink);
    return check_launch("rv_stream_read");
}

extern "C" rv_status rv_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    clear_error();
    RV_REQUIRE(src && dst, RV_ERR_INVALID_ARG, "rv_stream_copy: null pointer");
    RV_REQUIRE(bytes % 16 == 0 && ((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0, RV_ERR_INVALID_ARG,
               "rv_stream_copy: size and pointers must be multiples of 16 bytes");
    if (bytes == 0) return RV_OK;
    const int64_t n16 = (int64_t)(bytes / 16);
    const unsigned grid = copy_grid(n16);
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kCopyBlock), 0, (hipStream_t)stream,
                       static_cast<const v4u32 *>(src), static_cast<v4u32 *>(dst), n16);
    return check_launch("rv_stream_copy");
}

extern "C" rv_status rv_gather_probe(const void *table, int64_t n_records, int32_t rounds, int32_t blocks,
                                     uint32_t *sink, void *stream) {
    clear_error();
    RV_REQUIRE(table && sink, RV_ERR_INVALID_ARG, "rv_gather_probe: null pointer");
    RV_REQUIRE(((uintptr_t)table % 16) == 0, RV_ERR_INVALID_ARG, "rv_gather_probe: table must be 16-byte aligned");
    RV_REQUIRE(n_records >= 1 && n_records <= (int64_t)UINT32_MAX, RV_ERR_INVALID_ARG,
               "rv_gather_probe: n_records out of range");
    RV_REQUIRE(rounds >= kProbeBatch && rounds % kProbeBatch == 0, RV_ERR_INVALID_ARG,
               "rv_gather_probe: rounds must be a positive multiple of %d", kProbeBatch);
    RV_REQUIRE(blocks >= 1 && blocks <= (1 << 20), RV_ERR_INVALID_ARG, "rv_gather_probe: blocks out of range");
    hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const uint4 *>(table), (uint32_t)n_records, (int)rounds, sink);
    return check_launch("rv_gather_probe");
}
