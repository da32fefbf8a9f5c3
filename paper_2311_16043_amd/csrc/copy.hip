// copy.hip -- streaming copy used as the achievable-HBM-bandwidth probe and as
// the known-size reference for hardware byte counters.
#include "rv_internal.h"

namespace rv {
namespace {

// Each thread moves 64 bytes per iteration (four 16-byte vectors), grid-stride.
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace rv

using namespace rv;

extern "C" rv_status rv_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    clear_error();
    RV_REQUIRE(src && dst, RV_ERR_INVALID_ARG, "rv_stream_copy: null pointer");
    RV_REQUIRE(bytes % 16 == 0 && ((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0, RV_ERR_INVALID_ARG,
               "rv_stream_copy: size and pointers must be multiples of 16 bytes");
    if (bytes == 0) return RV_OK;
    const int64_t n16 = (int64_t)(bytes / 16);
    // 8 blocks of 256 threads per CU on 256 CUs
    const int64_t want = (n16 + 255) / 256;
    const unsigned grid = (unsigned)std::min<int64_t>(want, 256 * 8);
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
    return check_launch("rv_stream_copy");
}
