// surrogate.hip -- MLP visibility surrogate on the gfx950 matrix cores.
//
// Every product runs as v_mfma_f32_16x16x32_bf16 in the transposed form
//   C[16 outputs x 16 samples] += A[16 outputs x 32 inputs] * B[32 inputs x 16 samples],
// so that the accumulator layout (lane = one sample, four consecutive outputs)
// is reused unchanged as the next product's B operand: a matrix product is
// invariant under a common permutation of its summation index, so the packed
// weights (A operands) are laid out in the order in which the previous layer
// leaves its outputs in the lanes (kfeat below). Activations of a 32-sample
// wave never leave registers in inference.
//
// Parameter blob: header | FP32 master | Adam m | Adam v | BF16 forward A
// operands | BF16 backward A operands (W used as [in x out] for the
// gradient through the layer).
#include "trace_core.h"

namespace rv {
namespace {

constexpr int kHid = 256, kIn = 64, kEnc = 42;
constexpr int64_t kNParams = 214530;
__host__ __device__ constexpr int64_t off_w(int l) {  // l = 0..4 (layers 1..5)
    return l == 0 ? 0 : l == 1 ? 16640 : l == 2 ? 82432 : l == 3 ? 148224 : 214016;
}
__host__ __device__ constexpr int64_t off_b(int l) {
    return l == 0 ? 16384 : l == 1 ? 82176 : l == 2 ? 147968 : l == 3 ? 213760 : 214528;
}
__host__ __device__ constexpr int n_in(int l) { return l == 0 ? kIn : kHid; }
__host__ __device__ constexpr int n_out(int l) { return l == 4 ? 2 : kHid; }
// packed A operands, in bf16 elements: forward layer l = 0..4
__host__ __device__ constexpr int64_t fwd_off(int l) {
    return l == 0 ? 0 : l == 1 ? 16384 : l == 2 ? 81920 : l == 3 ? 147456 : 212992;
}
constexpr int64_t kFwdTotal = 217088;
// backward A operands: j = 0 for W5, 1 for W4, 2 for W3, 3 for W2
__host__ __device__ constexpr int64_t bwd_off(int j) { return j == 0 ? 0 : j == 1 ? 8192 : j == 2 ? 73728 : 139264; }
constexpr int64_t kBwdTotal = 204800;

struct SurLayout {
    size_t header, master, m, v, fwd, bwd, total;
};
inline SurLayout sur_layout() {
    SurLayout L{};
    size_t off = 0;
    L.header = off; off = align_up(off + 64 * sizeof(float));
    L.master = off; off = align_up(off + kNParams * sizeof(float));
    L.m = off; off = align_up(off + kNParams * sizeof(float));
    L.v = off; off = align_up(off + kNParams * sizeof(float));
    L.fwd = off; off = align_up(off + kFwdTotal * 2);
    L.bwd = off; off = align_up(off + kBwdTotal * 2);
    L.total = off;
    return L;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// bfloat16 bits of x, round to nearest even (finite inputs)
__host__ __device__ __forceinline__ uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
// two bfloat16 values (round to nearest even) in one word, lo in bits 0-15:
// one v_cvt_pk_bf16_f32 on gfx950
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}
__device__ __forceinline__ float bf16_val(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// ReLU of two bf16 values in one word: read as 16-bit integers, a bf16 value
// is negative exactly when its sign bit is set, so the per-half integer max
// with 0 is the ReLU (-0 becomes +0). Rounding to bf16 preserves sign and
// zero, so this equals rounding the ReLU of the FP32 values.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w) {
    typedef short i16x2 __attribute__((ext_vector_type(2)));
    const i16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, w), z));
}

// Feature carried by slot s (0..7) of lane group g (lane / 16) in k-block kb of
// a B operand built from accumulators: blocks 2kb and 2kb+1 of 16 outputs,
// four consecutive outputs per lane group.
__host__ __device__ constexpr int kfeat(int kb, int g, int s) { return (2 * kb + (s >> 2)) * 16 + 4 * g + (s & 3); }

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// ---- encoding -----------------------------------------------------------------

// Feature f of the encoding of u[0..5]: u, sin(pi u), cos(pi u), sin(2 pi u),
// cos(2 pi u), sin(4 pi u), cos(4 pi u) for each scalar; 0 for f >= 42.
__device__ __forceinline__ float enc_feature(int f, float u0, float u1, float u2, float u3, float u4, float u5) {
    if (f >= kEnc) return 0.0f;
    const int a = f / 7, c = f - 7 * a;
    const float v = a == 0 ? u0 : a == 1 ? u1 : a == 2 ? u2 : a == 3 ? u3 : a == 4 ? u4 : u5;
    if (c == 0) return v;
    const int lvl = (c - 1) >> 1;
    const float w = 3.14159265358979323846f * (float)(1 << lvl);
    return (c & 1) ? __sinf(w * v) : __cosf(w * v);
}

// ---- forward -----------------------------------------------------------------------

enum FwdMode { kModeXd = 0, kModeGrid = 1, kModeTrain = 2 };

struct FwdArgs {
    const float *master;
    const u32x4 *fwd;
    const float *header;
    int64_t n;               // samples (queries) in all launches of this call
    int64_t s_off;           // first sample of this launch (a grid covers at most 2^30 samples)
    // explicit inputs (xd and train)
    const float *x, *d, *T;
    // training: sample draw and saved tensors
    int hashed;              // 1: sample index = hash(seed, step, s) mod n_samples
    int64_t n_samples;
    uint64_t seed;
    int64_t step;
    uint16_t *ht;            // activations, feature-major: section j at ht + ht_off(j) * stride
    int64_t stride;          // samples per feature row (>= padded n)
    uint16_t *dz5;           // [2][stride]
    float *loss_part;        // per wave
    // outputs
    float *vis, *unc;
    // grid queries
    const float *gmean, *gnormal, *dirs;
    int K, dir_mode;
    int64_t q_begin;
    float tau;
    uint8_t *fb_flag;  // per query: 1 = to be traced (grid mode with a BVH), else NULL
};

// Training takes the batch in blocks of kTrainNT 16-sample tiles, each block
// kTrainWaves waves that split every layer's outputs (kTrainOps k-blocks of
// the next layer's input per wave), and covers the batch rounded up to 32
// samples: the padded samples' activations and gradients are stored as zeros
// for the weight-gradient products, which step over 32 samples at a time.
constexpr int kTrainWaves = 8, kTrainNT = 2;
constexpr int kTrainOps = 8 / kTrainWaves;
constexpr int64_t kTrainPad = 16 * kTrainNT > 32 ? 16 * kTrainNT : 32;
static_assert(kTrainWaves * kTrainOps == 8 && kTrainPad % (16 * kTrainNT) == 0 && kTrainPad <= 128,
              "training block shape");
__host__ __device__ constexpr int64_t train_pad(int64_t n) { return ((n + kTrainPad - 1) / kTrainPad) * kTrainPad; }

// feature-major activation sections: HT0 (64 rows), HT1..HT4 (256 rows each)
__host__ __device__ constexpr int64_t ht_row(int j) { return j == 0 ? 0 : 64 + (int64_t)(j - 1) * 256; }
constexpr int64_t kHtRows = 64 + 4 * 256;
constexpr int64_t kDzRows = 4 * 256 + 16;  // dZ1..dZ4 (256 rows each), dZ5 (2 rows, 16 reserved)
__host__ __device__ constexpr int64_t dz_row(int l) { return l < 4 ? (int64_t)l * 256 : 1024; }  // l = 0..4

// Output blocks 2 op and 2 op + 1 of a hidden layer for NT 16-sample tiles:
// act (B operands, k-blocks of the input) -> the ReLU outputs as k-block op of
// the next layer's B operand (bias in FP32, one v_cvt_pk_bf16_f32 per pair, then the ReLU
// on the packed word).
template <int KB, int NT>
__device__ __forceinline__ void fwd_pair(const u32x4 *__restrict__ A, const float *__restrict__ bias,
                                         const u32x4 (&act)[8][NT], int op, int lane, u32x4 (&out)[NT]) {
    const int g = lane >> 4;
    f32x4 acc[2][NT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[h][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const u32x4 a0 = A[((2 * op) * KB + kb) * 64 + lane];
        const u32x4 a1 = A[((2 * op + 1) * KB + kb) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            acc[0][nt] = mfma16(a0, act[kb][nt], acc[0][nt]);
            acc[1][nt] = mfma16(a1, act[kb][nt], acc[1][nt]);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float4 bv = *reinterpret_cast<const float4 *>(bias + (2 * op + h) * 16 + 4 * g);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            out[nt][2 * h + 0] = relu_bf16x2(pack2(acc[h][nt][0] + bv.x, acc[h][nt][1] + bv.y));
            out[nt][2 * h + 1] = relu_bf16x2(pack2(acc[h][nt][2] + bv.z, acc[h][nt][3] + bv.w));
        }
    }
}

// The word of the lane next to this one (lanes 2c and 2c+1 swap): one DPP
// quad permute [1, 0, 3, 2].
__device__ __forceinline__ uint32_t pair_swap(uint32_t w) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0xB1, 0xF, 0xF, false);
}

// Feature-major rows are written and read two samples (one 32-bit word) per
// lane: in a word holding rows ra (low halves) and rb (high halves) of this
// lane's sample, the even lane of a pair (samples s, s + 1) takes row ra of
// both samples and the odd lane (samples s - 1, s) row rb of both.
__device__ __forceinline__ uint32_t pair_row_word(uint32_t own, bool odd) {
    const uint32_t nb = pair_swap(own);
    return odd ? ((nb >> 16) | (own & 0xffff0000u)) : ((own & 0xffffu) | (nb << 16));
}

// Store k-block kb of a tile's B operand (features kfeat(kb, ., .)) as
// feature-major rows of ht, samples at or past n as zeros.
__device__ __forceinline__ void store_kblock(uint16_t *__restrict__ ht, int64_t stride, const u32x4 &frag, int kb,
                                             int lane, int64_t s_base, int64_t n) {
    const int g = lane >> 4, col = lane & 15;
    const bool odd = col & 1;
    const int64_t s2 = s_base + (col & ~1);   // first sample of the lane pair
    const uint32_t keep = (s2 < n ? 0x0000ffffu : 0u) | (s2 + 1 < n ? 0xffff0000u : 0u);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t word = pair_row_word(frag[w], odd) & keep;
        const int f = kfeat(kb, g, 2 * w + (odd ? 1 : 0));
        *reinterpret_cast<uint32_t *>(ht + (int64_t)f * stride + s2) = word;
    }
}

// The encoded inputs of NT tiles of 16 samples from s_base as B operands
// (k-blocks 0 and 1 of act; features kfeat), and the targets in training.
// Every wave of a training block encodes its block's tiles itself.
template <int kMode, int NT>
__device__ __forceinline__ void encode_tiles(const FwdArgs &a, int64_t s_base, int lane, u32x4 (&act)[8][NT],
                                             float (&Tv)[NT]) {
    const int g = lane >> 4, col = lane & 15;
    const float lo0 = a.header[0], lo1 = a.header[1], lo2 = a.header[2];
    const float hi0 = a.header[3], hi1 = a.header[4], hi2 = a.header[5];
    auto nrm = [](float x, float lo, float hi) {
        const float span = hi - lo;
        return span > 0.f ? 2.0f * (x - lo) / span - 1.0f : 0.0f;
    };

#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t s = s_base + nt * 16 + col;
        const bool valid = s < a.n;
        // grid queries q = i K + k: the tile's first query is split once per
        // wave (scalar), each lane's is at most 15 further on
        int64_t gi = 0;
        int gk = 0;
        if (kMode == kModeGrid) {
            const int64_t qt = a.q_begin + s_base + nt * 16;
            const int64_t q0 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(qt >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)qt);
            const int64_t i0 = q0 / a.K;
            gi = i0;
            gk = (int)(q0 - i0 * a.K) + col;
            while (gk >= a.K) {
                gk -= a.K;
                ++gi;
            }
        }
        float x0 = 0.f, x1 = 0.f, x2 = 0.f, d0 = 0.f, d1 = 0.f, d2 = 1.f;
        if (valid) {
            if (kMode == kModeGrid) {
                const int64_t i = gi;
                const int k = gk;
                float nx = 0.f, ny = 0.f, nz = 1.f;
                if (a.gnormal) {
                    nx = a.gnormal[3 * i]; ny = a.gnormal[3 * i + 1]; nz = a.gnormal[3 * i + 2];
                    const float nl = sqrtf(nx * nx + ny * ny + nz * nz);
                    nx /= nl; ny /= nl; nz /= nl;
                }
                f3 b1, b2;
                const f3 nv = mk(nx, ny, nz);
                onb_duff(nv, b1, b2);
                const f3 dv = ray_direction(a.dirs, k, a.dir_mode, nv, b1, b2);
                x0 = a.gmean[3 * i]; x1 = a.gmean[3 * i + 1]; x2 = a.gmean[3 * i + 2];
                d0 = dv.x; d1 = dv.y; d2 = dv.z;
            } else {
                int64_t idx = s;
                if (kMode == kModeTrain && a.hashed)
                    idx = (int64_t)(splitmix64(a.seed ^ splitmix64((uint64_t)a.step * 0x100000000ull + (uint64_t)s)) %
                                    (uint64_t)a.n_samples);
                x0 = a.x[3 * idx]; x1 = a.x[3 * idx + 1]; x2 = a.x[3 * idx + 2];
                d0 = a.d[3 * idx]; d1 = a.d[3 * idx + 1]; d2 = a.d[3 * idx + 2];
                if (kMode == kModeTrain) Tv[nt] = a.T[idx];
            }
        }
        const float u0 = nrm(x0, lo0, hi0), u1 = nrm(x1, lo1, hi1), u2 = nrm(x2, lo2, hi2);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int w = 0; w < 4; ++w)
                act[kb][nt][w] = pack2(enc_feature(kfeat(kb, g, 2 * w), u0, u1, u2, d0, d1, d2),
                                       enc_feature(kfeat(kb, g, 2 * w + 1), u0, u1, u2, d0, d1, d2));
    }
}

// Training forward: one block of kTrainWaves waves per kTrainNT 16-sample
// tiles. Of every hidden layer's 16 output blocks (8 k-blocks of the next
// layer's input), wave w produces k-blocks kTrainOps w .. kTrainOps (w + 1) - 1
// and stores them as feature-major rows; the waves exchange each layer's
// output through LDS (double-buffered, one barrier per layer). Wave 0
// evaluates the head and the loss.
__global__ __launch_bounds__(kTrainWaves * 64, 16 / kTrainWaves) void k_mlp_forward_train(FwdArgs a) {
    constexpr int NT = kTrainNT;
    __shared__ u32x4 xb[2][8][NT][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t s_base = tile * (16 * NT);
    if (s_base >= train_pad(a.n)) return;  // block-uniform
    const int g = lane >> 4, col = lane & 15;
    u32x4 act[8][NT];
    float Tv[NT] = {};
    encode_tiles<kModeTrain, NT>(a, s_base, lane, act, Tv);
    if (w < 2) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            store_kblock(a.ht + ht_row(0) * a.stride, a.stride, w == 0 ? act[0][nt] : act[1][nt], w, lane,
                         s_base + 16 * nt, a.n);
    }
    const float *master = a.master;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const u32x4 *A = a.fwd + fwd_off(l) / 8;
        uint16_t *ht = a.ht + ht_row(l + 1) * a.stride;
#pragma unroll
        for (int q = 0; q < kTrainOps; ++q) {
            const int op = kTrainOps * w + q;
            u32x4 o[NT];
            if (l == 0)
                fwd_pair<2, NT>(A, master + off_b(0), act, op, lane, o);
            else
                fwd_pair<8, NT>(A, master + off_b(l), act, op, lane, o);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                store_kblock(ht, a.stride, o[nt], op, lane, s_base + 16 * nt, a.n);
                xb[l & 1][op][nt][lane] = o[nt];
            }
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) act[kb][nt] = xb[l & 1][kb][nt][lane];
    }
    if (w != 0) return;

    // head: one block of 16 outputs, rows 0 and 1 are z0, z1
    f32x4 acc5[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc5[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 *A5 = a.fwd + fwd_off(4) / 8;
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
        const u32x4 av = A5[kb * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc5[nt] = mfma16(av, act[kb][nt], acc5[nt]);
    }
    const float b50 = master[off_b(4)], b51 = master[off_b(4) + 1];
    const float inv_n = 1.0f / (float)a.n;
    float lsum = 0.f;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t s = s_base + 16 * nt + col;
        const bool valid = s < a.n;
        const float z0 = acc5[nt][0] + b50, z1 = acc5[nt][1] + b51;
        const float V = 1.0f / (1.0f + expf(-z0));
        const float U = z1;   // predicted |T - V|, linear (no saturating activation)
        const float T = Tv[nt];
        const float e = fabsf(T - V);
        const float dz0 = (V - T) * inv_n;
        // squared error of U against |T - V| (V held constant)
        const float dz1 = 2.0f * (U - e) * inv_n;
        if (g == 0) {
            a.dz5[s] = valid ? (uint16_t)bf16_bits(dz0) : (uint16_t)0;
            a.dz5[a.stride + s] = valid ? (uint16_t)bf16_bits(dz1) : (uint16_t)0;
            if (valid) {
                const float bce = -(T * logf(fmaxf(V, 1e-12f)) + (1.f - T) * logf(fmaxf(1.f - V, 1e-12f)));
                lsum += bce + (U - e) * (U - e);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) a.loss_part[tile] = lsum;
}

// ---- inference with the weights staged through LDS ------------------------------
//
// Inference takes 32 samples per wave (two tiles) and eight waves per block,
// one block per CU (two waves per SIMD). The waves of a block share every
// weight fragment: the packed A operands are streamed layer by layer, in
// chunks of at most 64 KB, into one of two LDS buffers by direct
// global-to-LDS loads (no registers held), the next chunk loading while the
// current one is multiplied, one barrier per chunk (eight per 256 samples).
// Every A operand is then read from LDS. When each wave fetched all 424 KB of
// packed weights itself (48 samples per wave), those fetches ran at the rate
// of the CU's vector-memory path (TD busy 96 %) and held the matrix cores at
// 42 % of peak. Three tiles per wave do not fit 256 registers next to the LDS
// pipeline (the compiler spills ~150).
constexpr int kInferWaves = 8;
constexpr int kInferNT = 2;
constexpr int kInferSamples = kInferWaves * 16 * kInferNT;  // 256 per block
constexpr int kChunkVec = 4096;                             // 16-byte vectors per LDS buffer (64 KB)

typedef __attribute__((address_space(3))) void lds_void;

// This wave's share of copying `count` vectors (a multiple of 64) of packed
// operands from src to the LDS buffer dst: the 1 KB pieces wv, wv + 8, ...
// (a global_load_lds_dwordx4 writes 16 bytes per lane from the wave's LDS base).
__device__ __forceinline__ void load_chunk(const u32x4 *__restrict__ src, int count, u32x4 *dst, int wv, int lane) {
    for (int p = wv; p < count / 64; p += kInferWaves)
        __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + p * 64 + lane),
                                         (lds_void *)(dst + p * 64), 16, 0, 0);
}

// This wave's loads into LDS have landed, then every wave's have, and every
// wave has finished reading the buffer the next loads will overwrite.
__device__ __forceinline__ void chunk_barrier() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Output pair OP0 + o of a layer (the same arithmetic as hidden_layer) from
// the LDS chunk holding the A operands of pairs OP0, OP0 + 1, ...

template <int KB, int NT, int OP0>
__device__ __forceinline__ void layer_ops_lds_one(const u32x4 *A, int o, const float *__restrict__ bias,
                                                  const u32x4 (&act)[8][NT], u32x4 (&out)[8][NT], int lane) {
    const int g = lane >> 4;
    f32x4 acc[2][NT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[h][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const u32x4 a0 = A[((2 * o) * KB + kb) * 64 + lane];
        const u32x4 a1 = A[((2 * o + 1) * KB + kb) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            acc[0][nt] = mfma16(a0, act[kb][nt], acc[0][nt]);
            acc[1][nt] = mfma16(a1, act[kb][nt], acc[1][nt]);
        }
        // per k-block: its two LDS reads, then its products
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * NT, 0);
    }
    // bias in FP32, then the bf16 pair, then the ReLU on the packed words
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float4 bv = *reinterpret_cast<const float4 *>(bias + (2 * (OP0 + o) + h) * 16 + 4 * g);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            out[OP0 + o][nt][2 * h + 0] = relu_bf16x2(pack2(acc[h][nt][0] + bv.x, acc[h][nt][1] + bv.y));
            out[OP0 + o][nt][2 * h + 1] = relu_bf16x2(pack2(acc[h][nt][2] + bv.z, acc[h][nt][3] + bv.w));
        }
    }
}

// A 256 -> 256 layer from two LDS chunks (output pairs 0-3, then 4-7);
// `between` runs once the first half is done (the chunk hand-over). The
// output array is local, as in hidden_layer, so the input array's registers
// are reused as soon as the layer ends.
// Output pairs [OP0, OP0 + NOP) of a layer from one LDS chunk.
template <int KB, int NT, int OP0, int NOP>
__device__ __forceinline__ void layer_ops_lds(const u32x4 *A, const float *__restrict__ bias,
                                              const u32x4 (&act)[8][NT], u32x4 (&out)[8][NT], int lane) {
#pragma unroll
    for (int o = 0; o < NOP; ++o) layer_ops_lds_one<KB, NT, OP0>(A, o, bias, act, out, lane);
}

template <int NT, class Between>
__device__ __forceinline__ void hidden_layer_lds(const u32x4 *A_lo, const u32x4 *A_hi, const float *__restrict__ bias,
                                                 u32x4 (&act)[8][NT], int lane, Between between) {
    u32x4 out[8][NT];
    layer_ops_lds<8, NT, 0, 4>(A_lo, bias, act, out, lane);
    between();
    layer_ops_lds<8, NT, 4, 4>(A_hi, bias, act, out, lane);
#pragma unroll
    for (int kb = 0; kb < 8; ++kb)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) act[kb][nt] = out[kb][nt];
}

// Chunks, in 16-byte vectors of the packed forward operands: layer 1 whole
// (2,048), layers 2-4 in halves of four output pairs (4,096 each), the head
// (512). Chunk c is multiplied from buffer c % 2 while chunk c + 1 loads into
// the other. A k-block's two LDS reads are scheduled right before its
// products: hoisted further, as the compiler otherwise does, they spill the
// activations.
template <int kMode>
__global__ __launch_bounds__(kInferWaves * 64, 1) void k_mlp_forward(FwdArgs a) {
    constexpr int NT = kInferNT;
    __shared__ u32x4 wbuf[2][kChunkVec];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    // every wave takes part in the loads and barriers; waves past the end
    // encode zeros and write nothing
    const int64_t s_base = a.s_off + ((int64_t)blockIdx.x * kInferWaves + wv) * (16 * NT);
    const u32x4 *F = a.fwd;
    const float *master = a.master;
    load_chunk(F + fwd_off(0) / 8, 2048, wbuf[0], wv, lane);
    u32x4 act[8][NT];
    float Tv[NT] = {};
    encode_tiles<kMode, NT>(a, s_base, lane, act, Tv);
    chunk_barrier();
    // layer 1 (64 -> 256) from buffer 0; layer 2's first half loads into buffer 1
    load_chunk(F + fwd_off(1) / 8, kChunkVec, wbuf[1], wv, lane);
    {
        u32x4 out[8][NT];
        layer_ops_lds<2, NT, 0, 8>(wbuf[0], master + off_b(0), act, out, lane);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) act[kb][nt] = out[kb][nt];
    }
    chunk_barrier();
    // layers 2-4, each from buffer 1 (first half) then buffer 0 (second half)
    // while the following chunk loads into the other buffer
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
        load_chunk(F + fwd_off(l) / 8 + kChunkVec, kChunkVec, wbuf[0], wv, lane);
        hidden_layer_lds<NT>(wbuf[1], wbuf[0], master + off_b(l), act, lane, [&]() {
            chunk_barrier();
            if (l < 3) load_chunk(F + fwd_off(l + 1) / 8, kChunkVec, wbuf[1], wv, lane);
            else load_chunk(F + fwd_off(4) / 8, 512, wbuf[1], wv, lane);
        });
        chunk_barrier();
    }
    // head: one block of 16 outputs, rows 0 and 1 are z0, z1
    f32x4 acc5[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc5[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
        const u32x4 av = wbuf[1][kb * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc5[nt] = mfma16(av, act[kb][nt], acc5[nt]);
    }
    const float b50 = master[off_b(4)], b51 = master[off_b(4) + 1];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t s = s_base + nt * 16 + col;
        if (g == 0 && s < a.n) {
            const float z0 = acc5[nt][0] + b50, z1 = acc5[nt][1] + b51;
            const float V = 1.0f / (1.0f + expf(-z0));
            const float U = z1;
            a.vis[s] = V;
            if (a.unc) a.unc[s] = U;
            if (kMode == kModeGrid && a.fb_flag) a.fb_flag[s] = U > a.tau ? 1 : 0;
        }
    }
}

// ---- backward through the layers ----------------------------------------------

// Output blocks 2 op and 2 op + 1 of dH = W dZ for NT 16-sample tiles (A =
// the layer's backward operands, KB k-blocks of the output gradient in act),
// masked by the ReLU of the layer's input (feature-major rows ht_in): the
// pre-activation gradient of the layer below, stored as feature-major rows of
// dz_out and returned as k-block op of the next product's B operand.
template <int KB, int NT>
__device__ __forceinline__ void bwd_pair(const u32x4 *__restrict__ A, const uint16_t *__restrict__ ht_in,
                                         uint16_t *__restrict__ dz_out, int64_t stride, const u32x4 (&act)[8][NT],
                                         int op, int lane, int64_t s_base, u32x4 (&out)[NT]) {
    const int g = lane >> 4, col = lane & 15;
    const bool odd = col & 1;
    f32x4 acc[2][NT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[h][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const u32x4 a0 = A[((2 * op) * KB + kb) * 64 + lane];
        const u32x4 a1 = A[((2 * op + 1) * KB + kb) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            acc[0][nt] = mfma16(a0, act[kb][nt], acc[0][nt]);
            acc[1][nt] = mfma16(a1, act[kb][nt], acc[1][nt]);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        // rows mb 16 + 4 g + r of this lane's sample; the pair's loads and
        // stores cover rows r = 0, 2 (even lane) and 1, 3 (odd lane)
        const int64_t f0 = (2 * op + h) * 16 + 4 * g + (odd ? 1 : 0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t s2 = s_base + 16 * nt + (col & ~1);   // first sample of the lane pair
            // the pair's words of rows (0 | 1) and (2 | 3), both samples; the
            // same exchange turns them into rows 0 (low) and 1 (high), and 2
            // and 3, of this lane's own sample
            const uint32_t r01 = pair_row_word(*reinterpret_cast<const uint32_t *>(ht_in + f0 * stride + s2), odd);
            const uint32_t r23 =
                pair_row_word(*reinterpret_cast<const uint32_t *>(ht_in + (f0 + 2) * stride + s2), odd);
            // the ReLU mask of the layer input (bf16 output > 0; padded samples are 0)
            const float z0 = (r01 & 0xffffu) != 0u ? acc[h][nt][0] : 0.0f;
            const float z1 = (r01 >> 16) != 0u ? acc[h][nt][1] : 0.0f;
            const float z2 = (r23 & 0xffffu) != 0u ? acc[h][nt][2] : 0.0f;
            const float z3 = (r23 >> 16) != 0u ? acc[h][nt][3] : 0.0f;
            const uint32_t p01 = pack2(z0, z1), p23 = pack2(z2, z3);
            out[nt][2 * h + 0] = p01;
            out[nt][2 * h + 1] = p23;
            *reinterpret_cast<uint32_t *>(dz_out + f0 * stride + s2) = pair_row_word(p01, odd);
            *reinterpret_cast<uint32_t *>(dz_out + (f0 + 2) * stride + s2) = pair_row_word(p23, odd);
        }
    }
}

struct BwdArgs {
    const u32x4 *bwd;
    const uint16_t *ht;
    uint16_t *dz;
    int64_t stride;
    int64_t n;
};

// Backward through the layers, split as the training forward: one block of
// kTrainWaves waves per kTrainNT 16-sample tiles, wave w producing k-blocks
// kTrainOps w .. kTrainOps (w + 1) - 1 of each layer's input gradient,
// exchanged through LDS.
__global__ __launch_bounds__(kTrainWaves * 64, 16 / kTrainWaves) void k_mlp_backward(BwdArgs a) {
    constexpr int NT = kTrainNT;
    __shared__ u32x4 xb[2][8][NT][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t s_base = (int64_t)blockIdx.x * (16 * NT);
    if (s_base >= train_pad(a.n)) return;  // block-uniform
    const int g = lane >> 4, col = lane & 15;
    u32x4 act[8][NT];
    // head gradient as a B operand: outputs 0 and 1 sit in slots 0, 1 of lane group 0
    const uint16_t *dz5 = a.dz + dz_row(4) * a.stride;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t s = s_base + 16 * nt + col;
        act[0][nt] = u32x4{0u, 0u, 0u, 0u};
        if (g == 0) act[0][nt][0] = (uint32_t)dz5[s] | ((uint32_t)dz5[a.stride + s] << 16);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // j = 0: through W5 (input rows h4, gradient dZ4); j = 3: through W2 (h1, dZ1)
        const u32x4 *A = a.bwd + bwd_off(j) / 8;
        const uint16_t *ht_in = a.ht + ht_row(4 - j) * a.stride;
        uint16_t *dz_out = a.dz + dz_row(3 - j) * a.stride;
#pragma unroll
        for (int q = 0; q < kTrainOps; ++q) {
            const int op = kTrainOps * w + q;
            u32x4 o[NT];
            if (j == 0)
                bwd_pair<1, NT>(A, ht_in, dz_out, a.stride, act, op, lane, s_base, o);
            else
                bwd_pair<8, NT>(A, ht_in, dz_out, a.stride, act, op, lane, s_base, o);
            if (j < 3) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) xb[j & 1][op][nt][lane] = o[nt];
            }
        }
        if (j == 3) break;
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) act[kb][nt] = xb[j & 1][kb][nt][lane];
    }
}

// ---- weight gradients ----------------------------------------------------------------

// One block of four waves: a 128 x 128 tile of dW_l[k][o] = sum_s h[k][s]
// dz[o][s] over one slice of the batch, wave w holding the 64 x 64 quarter
// (k half w / 2, o half w % 2) as C[k][o] += A[k x 32 samples] B[32 samples x
// o], plus the bias gradient of its 64 outputs when it holds the layer's
// first 64 rows. Each 32-sample step stages the tile's 128 h rows and 128 dz
// rows (64 bytes each) in LDS once for the four waves (double-buffered, one
// barrier per step); rows are padded to 80 bytes so that a fragment read
// (16 rows x 16 bytes per lane group) hits 16 distinct bank quadruples.
struct WgradArgs {
    const uint16_t *ht, *dz;
    int64_t stride;
    int64_t n_pad;       // samples covered (a multiple of 32)
    int64_t slice_len;   // multiple of 32
    int n_slices;
    float *partial;      // [n_slices][n_params]
};

// tiles per slice: l0 (64 x 256): 1 x 2, l1-3 (256 x 256): 2 x 2, l4 (256 x 2): 2 x 1 -> 16
__device__ __forceinline__ void tile_of(int t, int &l, int &kt, int &ot) {
    if (t < 2) { l = 0; kt = 0; ot = t; return; }
    t -= 2;
    if (t < 12) { l = 1 + t / 4; kt = (t % 4) / 2; ot = t % 2; return; }
    t -= 12;
    l = 4; kt = t; ot = 0;
}
constexpr int kTiles = 16;
constexpr int kWgRow = 40;   // LDS row stride in bf16 elements (80 bytes: 32 samples + padding)

__global__ __launch_bounds__(256) void k_mlp_wgrad(WgradArgs a) {
    __shared__ __align__(16) uint16_t hs[2][128 * kWgRow];
    __shared__ __align__(16) uint16_t ds[2][128 * kWgRow];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tile = (int)(blockIdx.x % kTiles);
    const int slice = (int)(blockIdx.x / kTiles);
    int l, kt, ot;
    tile_of(tile, l, kt, ot);
    const int Nin = n_in(l), Nout = n_out(l);
    const int k0 = kt * 128, o0 = ot * 128;
    const uint16_t *H = a.ht + ht_row(l) * a.stride;
    const uint16_t *D = a.dz + dz_row(l) * a.stride;
    const int64_t s0 = (int64_t)slice * a.slice_len;
    const int64_t s1 = min(a.n_pad, s0 + a.slice_len);
    // staging: thread t moves 16-byte part t % 4 of rows t / 4 and 64 + t / 4,
    // of h and of dz (rows past the layer's inputs or outputs as zeros). A
    // step's rows are fetched into registers two steps before they are written
    // to LDS, so each fetch has two steps of products to arrive.
    const int srow = threadIdx.x >> 2, spart = threadIdx.x & 3;
    auto fetch = [&](int64_t s, u32x4 (&r)[4]) {
        if (s >= s1) return;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = srow + 64 * u;
            r[2 * u] = k0 + row < Nin ? *reinterpret_cast<const u32x4 *>(H + (int64_t)(k0 + row) * a.stride + s + 8 * spart)
                                      : u32x4{0u, 0u, 0u, 0u};
            r[2 * u + 1] = o0 + row < Nout
                               ? *reinterpret_cast<const u32x4 *>(D + (int64_t)(o0 + row) * a.stride + s + 8 * spart)
                               : u32x4{0u, 0u, 0u, 0u};
        }
    };
    auto put = [&](const u32x4 (&r)[4], int buf) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = srow + 64 * u;
            *reinterpret_cast<u32x4 *>(&hs[buf][row * kWgRow + 8 * spart]) = r[2 * u];
            *reinterpret_cast<u32x4 *>(&ds[buf][row * kWgRow + 8 * spart]) = r[2 * u + 1];
        }
    };
    const int wk = w >> 1, wo = w & 1;
    // a wave whose quarter lies past the layer's inputs or outputs only stages
    const bool live = k0 + 64 * wk < Nin && o0 + 64 * wo < Nout;
    const bool bias = live && k0 + 64 * wk == 0;
    const int g = lane >> 4, col = lane & 15;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[4] = {0.f, 0.f, 0.f, 0.f};
    // products of the 32 samples staged in buffer buf
    auto step = [&](int buf) {
        if (!live) return;
        u32x4 av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            av[i] = *reinterpret_cast<const u32x4 *>(&hs[buf][(64 * wk + 16 * i + col) * kWgRow + 8 * g]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bv[j] = *reinterpret_cast<const u32x4 *>(&ds[buf][(64 * wo + 16 * j + col) * kWgRow + 8 * g]);
        if (bias) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) bsum[j] += bf16_val(bv[j][q] & 0xffffu) + bf16_val(bv[j][q] >> 16);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(av[i], bv[j], acc[i][j]);
    };
    u32x4 ra[4], rb[4];
    fetch(s0, ra);
    fetch(s0 + 32, rb);
    put(ra, 0);
    fetch(s0 + 64, ra);
    __syncthreads();
    // two steps per pass: buffer 0 holds step s, registers rb step s + 32 and
    // ra step s + 64
    for (int64_t s = s0; s < s1; s += 64) {
        step(0);
        if (s + 32 < s1) put(rb, 1);
        fetch(s + 96, rb);
        __syncthreads();
        if (s + 32 >= s1) break;
        step(1);
        if (s + 64 < s1) put(ra, 0);
        fetch(s + 128, ra);
        __syncthreads();
    }
    if (!live) return;
    float *P = a.partial + (int64_t)slice * kNParams;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = o0 + 64 * wo + j * 16 + col;
            if (o < Nout) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = k0 + 64 * wk + i * 16 + 4 * g + r;
                    P[off_w(l) + (int64_t)k * Nout + o] = acc[i][j][r];
                }
            }
        }
    if (bias) {
        // lanes col, col+16, col+32, col+48 hold the same output: add the four groups in a fixed order
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = bsum[j];
            const float v1 = __shfl(v, col + 16), v2 = __shfl(v, col + 32), v3 = __shfl(v, col + 48);
            const float v0 = __shfl(v, col);
            const int o = o0 + 64 * wo + j * 16 + col;
            if (g == 0 && o < Nout) P[off_b(l) + o] = ((v0 + v1) + v2) + v3;
        }
    }
}

// grad[p] = sum over slices (in order) of partial[slice][p], eight loads in
// flight per thread; loss = sum of the wave partials / n, by the first wave of
// block 0 (lane l takes partials l, l + 64, ..., then a fixed butterfly).
__global__ __launch_bounds__(256) void k_reduce_grad(const float *__restrict__ partial, int n_slices,
                                                     float *__restrict__ grad, const float *__restrict__ loss_part,
                                                     int64_t n_waves, int64_t n, float *__restrict__ loss_out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) {
        float s = 0.f;
        int i = 0;
        for (; i + 8 <= n_slices; i += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(i + u) * kNParams + p];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; i < n_slices; ++i) s += partial[(int64_t)i * kNParams + p];
        grad[p] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x < 64 && loss_out) {
        double s = 0.0;
        for (int64_t w = threadIdx.x; w < n_waves; w += 64) s += loss_part[w];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (threadIdx.x == 0) *loss_out = (float)(s / (double)n);
    }
}

// ---- optimiser and packing ---------------------------------------------------------------

// BF16 A operands from the FP32 master weights (see kfeat).
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ master, uint16_t *__restrict__ fwd,
                                              uint16_t *__restrict__ bwd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kFwdTotal) {
        int l = 0;
        while (l < 4 && e >= fwd_off(l + 1)) ++l;
        const int64_t r = e - fwd_off(l);
        const int KB = n_in(l) / 32;
        const int s = (int)(r & 7), lane = (int)((r >> 3) & 63);
        const int64_t blk = r >> 9;
        const int kb = (int)(blk % KB), ob = (int)(blk / KB);
        const int o = ob * 16 + (lane & 15), k = kfeat(kb, lane >> 4, s);
        const float w = (o < n_out(l)) ? master[off_w(l) + (int64_t)k * n_out(l) + o] : 0.0f;
        fwd[e] = (uint16_t)bf16_bits(w);
    } else if (e < kFwdTotal + kBwdTotal) {
        const int64_t eb = e - kFwdTotal;
        int j = 0;
        while (j < 3 && eb >= bwd_off(j + 1)) ++j;
        const int l = 4 - j;  // layer index of the weights
        const int64_t r = eb - bwd_off(j);
        const int KB = (l == 4) ? 1 : 8;
        const int s = (int)(r & 7), lane = (int)((r >> 3) & 63);
        const int64_t blk = r >> 9;
        const int kb = (int)(blk % KB), mb = (int)(blk / KB);
        const int k = mb * 16 + (lane & 15), o = kfeat(kb, lane >> 4, s);
        const float w = (o < n_out(l)) ? master[off_w(l) + (int64_t)k * n_out(l) + o] : 0.0f;
        bwd[eb] = (uint16_t)bf16_bits(w);
    }
}

// Positions of weight W_l[k][o] (l = 0..4) in the packed operands: its
// forward A-operand element, and for l >= 1 its backward A-operand element
// (the inverse of the element -> weight map of k_pack).
__device__ __forceinline__ int64_t fwd_pos(int l, int k, int o) {
    const int KB = n_in(l) / 32;
    const int kb = k >> 5, g = (k & 15) >> 2, sl = ((k & 31) >> 4) * 4 + (k & 3);
    const int64_t blk = (int64_t)(o >> 4) * KB + kb;
    return fwd_off(l) + blk * 512 + (g * 16 + (o & 15)) * 8 + sl;
}
__device__ __forceinline__ int64_t bwd_pos(int l, int k, int o) {
    const int KB = (l == 4) ? 1 : 8;
    const int kb = o >> 5, g = (o & 15) >> 2, sl = ((o & 31) >> 4) * 4 + (o & 3);
    const int64_t blk = (int64_t)(k >> 4) * KB + kb;
    return bwd_off(4 - l) + blk * 512 + (g * 16 + (k & 15)) * 8 + sl;
}

// One training step's update, fused per parameter: the gradient as the
// in-order sum of the slice partials (as k_reduce_grad), the Adam update with
// bias-corrected moments (c1 = 1 - beta1^t, c2 = 1 - beta2^t), and the bf16
// copies of a weight in the packed operands (as k_pack; the padding elements
// stay the zeros written at initialisation). The loss is summed as in
// k_reduce_grad.
__global__ __launch_bounds__(256) void k_adam_pack(const float *__restrict__ partial, int n_slices,
                                                   float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                                   uint16_t *__restrict__ fwd, uint16_t *__restrict__ bwd, float lr,
                                                   float beta1, float beta2, float eps, float c1, float c2,
                                                   const float *__restrict__ loss_part, int64_t n_waves, int64_t n,
                                                   float *__restrict__ loss_out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) {
        float gr = 0.f;
        int i = 0;
        for (; i + 8 <= n_slices; i += 8) {
            float vs[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vs[u] = partial[(int64_t)(i + u) * kNParams + p];
#pragma unroll
            for (int u = 0; u < 8; ++u) gr += vs[u];
        }
        for (; i < n_slices; ++i) gr += partial[(int64_t)i * kNParams + p];
        const float mm = beta1 * m[p] + (1.f - beta1) * gr;
        const float vv = beta2 * v[p] + (1.f - beta2) * gr * gr;
        m[p] = mm;
        v[p] = vv;
        const float wn = w[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        w[p] = wn;
        int l = 0;
        while (l < 4 && p >= off_w(l + 1)) ++l;
        const int64_t r = p - off_w(l);
        if (r < (int64_t)n_in(l) * n_out(l)) {   // a weight (the layer's biases follow its weights)
            const int k = (int)(r / n_out(l)), o = (int)(r - (int64_t)k * n_out(l));
            const uint16_t b = (uint16_t)bf16_bits(wn);
            fwd[fwd_pos(l, k, o)] = b;
            if (l >= 1) bwd[bwd_pos(l, k, o)] = b;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 64 && loss_out) {
        double s = 0.0;
        for (int64_t q = threadIdx.x; q < n_waves; q += 64) s += loss_part[q];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (threadIdx.x == 0) *loss_out = (float)(s / (double)n);
    }
}

// He-uniform from a counter-based hash, zero biases.
__global__ __launch_bounds__(256) void k_init_hash(float *__restrict__ master, uint64_t seed) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParams) return;
    int l = 0;
    while (l < 4 && p >= off_w(l + 1)) ++l;
    if (p >= off_b(l)) {
        master[p] = 0.0f;
        return;
    }
    const float lim = sqrtf(6.0f / (float)n_in(l));
    const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)p));
    const float u = (float)(h >> 40) * (1.0f / 16777216.0f);  // [0, 1)
    master[p] = (2.0f * u - 1.0f) * lim;
}

__global__ __launch_bounds__(256) void k_copy_f32(const float *__restrict__ src, float *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_fill_f32(float *__restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(64) void k_set_header(float *__restrict__ h, float l0, float l1, float l2, float h0,
                                                   float h1, float h2) {
    if (threadIdx.x == 0) {
        h[0] = l0; h[1] = l1; h[2] = l2; h[3] = h0; h[4] = h1; h[5] = h2;
        for (int i = 6; i < 64; ++i) h[i] = 0.0f;
    }
}

// ---- fallback tracing and ray setup -----------------------------------------------------------------

__global__ void k_store_count(const unsigned long long *__restrict__ count, int64_t *__restrict__ out) {
    if (threadIdx.x == 0) *out = (int64_t)*count;
}

// Fallback list in the BVH's leaf (Morton) order, direction by direction:
// one wave per group of 64 consecutive sorted positions (lane l holds
// Gaussian i = src(64 g + l)) appends the group's flagged queries that lie
// in [q_begin, q_begin + q_count) as positions s = q - q_begin, direction k
// by direction k and lane by lane within a direction, after one atomic
// reservation per group. A pool of consecutive list entries then holds rays
// of nearby Gaussians in the same few directions, which walk the same part of
// the tree together. The list order between groups depends on scheduling;
// each ray's result does not.
__global__ __launch_bounds__(256) void k_fallback_rows(const float *__restrict__ header,
                                                       const float4 *__restrict__ rec, int64_t n, int K,
                                                       int64_t q_begin, int64_t q_count,
                                                       const uint8_t *__restrict__ flag,
                                                       unsigned long long *__restrict__ count,
                                                       int64_t *__restrict__ list) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t n_groups = (n + 63) / 64;
    // with a tree built for another Gaussian set the records are not read:
    // Gaussians are taken in index order (the traversal then gives NaN)
    const bool tree_ok = tree_matches(header, n);
    const bool aligned = K % 16 == 0 && q_begin % 16 == 0;
    for (int64_t grp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); grp < n_groups; grp += (int64_t)gridDim.x * 4) {
        const int64_t m = grp * 64 + lane;
        // this lane's Gaussian and the directions of it that lie in the range
        int64_t row = 0;  // s of direction 0
        int k_lo = 0, k_hi = 0;
        if (m < n) {
            const int64_t i = tree_ok ? (int64_t)__float_as_int(rec[kLeafF4 * m + 2].w) : m;
            row = i * K - q_begin;
            // clamped to [0, K] in 64 bits: rows far outside the range give k_lo >= k_hi
            k_lo = (int)min<int64_t>(K, max<int64_t>(0, -row));
            k_hi = (int)max<int64_t>(0, min<int64_t>(K, q_count - row));
        }
        const bool any = __ballot(k_lo < k_hi) != 0;
        if (!any) continue;  // wave-uniform
        int total = 0;
        unsigned long long base = 0;
        if (aligned) {
            // rows start on 16-byte boundaries: 16 flags per lane per load
            // (the flag buffer is padded to 256 bytes, so a row's last load
            // stays inside it); two passes, counting then writing
            for (int pass = 0; pass < 2; ++pass) {
                for (int k0 = 0; k0 < K; k0 += 16) {
                    u32x4 w = u32x4{0u, 0u, 0u, 0u};
                    if (k0 + 16 > k_lo && k0 < k_hi)
                        w = *reinterpret_cast<const u32x4 *>(flag + row + k0);
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int k = k0 + u;
                        const bool f = k >= k_lo && k < k_hi && ((w[u >> 2] >> (8 * (u & 3))) & 0xffu) != 0;
                        const uint64_t b = __ballot(f);
                        if (pass == 0) {
                            total += __popcll(b);
                        } else {
                            if (f) list[base + __popcll(b & lt)] = row + k;
                            base += __popcll(b);
                        }
                    }
                }
                if (pass == 0) {
                    if (total == 0) break;
                    if (lane == 0) base = atomicAdd(count, (unsigned long long)total);
                    base = __shfl(base, 0);
                }
            }
            continue;
        }
        for (int k = 0; k < K; ++k) {
            const bool f = k >= k_lo && k < k_hi && flag[row + k] != 0;
            total += __popcll(__ballot(f));
        }
        if (total == 0) continue;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)total);
        base = __shfl(base, 0);
        for (int k = 0; k < K; ++k) {
            const bool f = k >= k_lo && k < k_hi && flag[row + k] != 0;
            const uint64_t b = __ballot(f);
            if (f) list[base + __popcll(b & lt)] = row + k;
            base += __popcll(b);
        }
    }
}

__global__ __launch_bounds__(256) void k_ray_setup(const float *__restrict__ mean, const float *__restrict__ normal,
                                                   int64_t n, const float *__restrict__ dirs, int K, int dir_mode,
                                                   const int64_t *__restrict__ ids, int64_t n_rays,
                                                   float *__restrict__ out_o, float *__restrict__ out_d) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_rays) return;
    const int64_t r = ids[s];
    if (r < 0 || r >= n * (int64_t)K) {
        const float nan = __int_as_float(0x7fc00000);
        for (int a = 0; a < 3; ++a) out_o[3 * s + a] = out_d[3 * s + a] = nan;
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
    const f3 nrm = mk(nx, ny, nz);
    f3 b1, b2;
    onb_duff(nrm, b1, b2);
    const f3 d = ray_direction(dirs, k, dir_mode, nrm, b1, b2);
    out_o[3 * s] = mean[3 * i]; out_o[3 * s + 1] = mean[3 * i + 1]; out_o[3 * s + 2] = mean[3 * i + 2];
    out_d[3 * s] = d.x; out_d[3 * s + 1] = d.y; out_d[3 * s + 2] = d.z;
}

// ---- training workspace --------------------------------------------------------------------------------

// The weight gradients are summed over at most kMaxSlices slices of the
// batch (a multiple of 32 samples each), so that the 16 tiles of every slice
// give 256 blocks whatever the batch; the slice partials are added in order.
constexpr int kMaxSlices = 16;
inline int64_t slice_len_for(int64_t n_pad) {
    const int64_t per = (n_pad + kMaxSlices - 1) / kMaxSlices;
    return std::max<int64_t>(32, ((per + 31) / 32) * 32);
}
inline int slices_for(int64_t n_pad) {
    const int64_t len = slice_len_for(n_pad);
    return (int)((n_pad + len - 1) / len);
}

struct TrainWs {
    size_t ht, dz, partial, loss_part, loss, total;
    int64_t stride, n_slices, n_waves;
};

inline TrainWs train_ws(int64_t batch) {
    TrainWs W{};
    const int64_t pad = ((batch + 127) / 128) * 128;
    W.stride = pad;
    W.n_slices = kMaxSlices;
    W.n_waves = train_pad(batch) / (16 * kTrainNT);   // one loss partial per training block
    size_t off = 0;
    W.ht = off; off = align_up(off + (size_t)kHtRows * pad * 2);
    W.dz = off; off = align_up(off + (size_t)kDzRows * pad * 2);
    W.partial = off; off = align_up(off + (size_t)W.n_slices * kNParams * 4);
    W.loss_part = off; off = align_up(off + (size_t)W.n_waves * 4);
    W.loss = off; off = align_up(off + 256);
    W.total = off;
    return W;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }
// Samples per inference launch: a dispatch counts its work-items in 32 bits,
// so one grid stays at 2^30 samples (below 2^31 work-items at 48 samples per
// wave).
constexpr int64_t kLaunchSamples = int64_t(1) << 30;

// forward (train) + backward + weight gradients + reduction on samples [0, n)
// With grad == nullptr the slice partials are left for k_adam_pack.
rv_status loss_grad_impl(const void *params, const float *x, const float *d, const float *T, int64_t n, bool hashed,
                         int64_t n_samples, uint64_t seed, int64_t step, float *grad, float *loss_out, void *ws,
                         const TrainWs &W, hipStream_t s) {
    const SurLayout L = sur_layout();
    const int64_t n_pad = train_pad(n);
    FwdArgs fa{};
    fa.master = at<float>(params, L.master);
    fa.fwd = at<u32x4>(params, L.fwd);
    fa.header = at<float>(params, L.header);
    fa.n = n;
    fa.x = x;
    fa.d = d;
    fa.T = T;
    fa.hashed = hashed ? 1 : 0;
    fa.n_samples = n_samples;
    fa.seed = seed;
    fa.step = step;
    fa.ht = at<uint16_t>(ws, W.ht);
    fa.stride = W.stride;
    fa.dz5 = at<uint16_t>(ws, W.dz) + dz_row(4) * W.stride;
    fa.loss_part = at<float>(ws, W.loss_part);
    const int64_t tiles = n_pad / (16 * kTrainNT);   // one block per kTrainNT 16-sample tiles
    hipLaunchKernelGGL(k_mlp_forward_train, dim3((unsigned)tiles), dim3(kTrainWaves * 64), 0, s, fa);
    BwdArgs ba{at<u32x4>(params, L.bwd), at<uint16_t>(ws, W.ht), at<uint16_t>(ws, W.dz), W.stride, n};
    hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)tiles), dim3(kTrainWaves * 64), 0, s, ba);
    WgradArgs wa{};
    wa.ht = at<uint16_t>(ws, W.ht);
    wa.dz = at<uint16_t>(ws, W.dz);
    wa.stride = W.stride;
    wa.n_pad = n_pad;
    wa.slice_len = slice_len_for(n_pad);
    wa.n_slices = slices_for(n_pad);
    wa.partial = at<float>(ws, W.partial);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)(kTiles * wa.n_slices)), dim3(256), 0, s, wa);
    if (grad)
        hipLaunchKernelGGL(k_reduce_grad, dim3(blocks_for(kNParams, 256)), dim3(256), 0, s, wa.partial, wa.n_slices,
                           grad, at<float>(ws, W.loss_part), tiles, n, loss_out);
    return check_launch("surrogate loss/gradient");
}

}  // namespace
}  // namespace rv

using namespace rv;

extern "C" int64_t rv_surrogate_n_params(void) { return kNParams; }

extern "C" size_t rv_surrogate_bytes(void) { return sur_layout().total; }

extern "C" rv_status rv_surrogate_view(const void *params, rv_surrogate_arrays *out) {
    clear_error();
    RV_REQUIRE(params && out, RV_ERR_INVALID_ARG, "rv_surrogate_view: null pointer");
    const SurLayout L = sur_layout();
    void *p = const_cast<void *>(params);
    out->header = at<float>(p, L.header);
    out->master = at<float>(p, L.master);
    out->adam_m = at<float>(p, L.m);
    out->adam_v = at<float>(p, L.v);
    out->packed = at<char>(p, L.fwd);
    return RV_OK;
}

extern "C" size_t rv_surrogate_train_workspace_bytes(int32_t batch) {
    if (batch < 1) return 0;
    return train_ws(batch).total;
}

// Inference scratch: [0, 256) the fallback count (byte 0) and the tracer's
// eight queue counters (byte 64); the list of q_count int64; q_count flags.
extern "C" size_t rv_surrogate_infer_workspace_bytes(int64_t q_count) {
    if (q_count < 0) return 0;
    return kAlign + align_up((size_t)q_count * sizeof(int64_t)) + align_up((size_t)q_count);
}

extern "C" rv_status rv_surrogate_init(void *params, uint64_t seed, const float *box_lo_host, const float *box_hi_host,
                                       const float *init_weights, void *stream) {
    clear_error();
    RV_REQUIRE(params && box_lo_host && box_hi_host, RV_ERR_INVALID_ARG, "rv_surrogate_init: null argument");
    RV_REQUIRE(((uintptr_t)params % kAlign) == 0, RV_ERR_INVALID_ARG, "rv_surrogate_init: params not 256-byte aligned");
    const SurLayout L = sur_layout();
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_set_header, dim3(1), dim3(64), 0, s, at<float>(params, L.header), box_lo_host[0],
                       box_lo_host[1], box_lo_host[2], box_hi_host[0], box_hi_host[1], box_hi_host[2]);
    if (init_weights)
        hipLaunchKernelGGL(k_copy_f32, dim3(blocks_for(kNParams, 256)), dim3(256), 0, s, init_weights,
                           at<float>(params, L.master), kNParams);
    else
        hipLaunchKernelGGL(k_init_hash, dim3(blocks_for(kNParams, 256)), dim3(256), 0, s, at<float>(params, L.master),
                           seed);
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(kNParams, 256)), dim3(256), 0, s, at<float>(params, L.m), kNParams,
                       0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(kNParams, 256)), dim3(256), 0, s, at<float>(params, L.v), kNParams,
                       0.0f);
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(kFwdTotal + kBwdTotal, 256)), dim3(256), 0, s,
                       at<float>(params, L.master), at<uint16_t>(params, L.fwd), at<uint16_t>(params, L.bwd));
    return check_launch("rv_surrogate_init");
}

extern "C" rv_status rv_surrogate_loss_grad(const void *params, const float *x, const float *d, const float *T,
                                            int64_t n, float *grad_out, float *loss_out, void *ws, size_t ws_bytes,
                                            void *stream) {
    clear_error();
    RV_REQUIRE(params && x && d && T && grad_out && ws, RV_ERR_INVALID_ARG, "rv_surrogate_loss_grad: null argument");
    RV_REQUIRE(n >= 1 && n <= (1LL << 30), RV_ERR_INVALID_ARG, "rv_surrogate_loss_grad: n out of range");
    RV_REQUIRE(((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG, "rv_surrogate_loss_grad: ws not 256-byte aligned");
    const TrainWs W = train_ws(n);
    RV_REQUIRE(ws_bytes >= W.total, RV_ERR_WORKSPACE, "rv_surrogate_loss_grad: ws_bytes %zu < %zu", ws_bytes, W.total);
    return loss_grad_impl(params, x, d, T, n, false, n, 0, 0, grad_out, loss_out, ws, W, (hipStream_t)stream);
}

extern "C" rv_status rv_surrogate_train(void *params, const float *x, const float *d, const float *T,
                                        int64_t n_samples, const rv_train_opts *o, float *loss_log, void *ws,
                                        size_t ws_bytes, void *stream) {
    clear_error();
    RV_REQUIRE(params && x && d && T && o && ws, RV_ERR_INVALID_ARG, "rv_surrogate_train: null argument");
    RV_REQUIRE(n_samples >= 1, RV_ERR_INVALID_ARG, "rv_surrogate_train: n_samples < 1");
    RV_REQUIRE(o->steps >= 0 && o->batch >= 128 && o->batch % 128 == 0, RV_ERR_INVALID_ARG,
               "rv_surrogate_train: need steps >= 0 and batch a positive multiple of 128");
    RV_REQUIRE(o->lr >= 0.f && o->beta1 >= 0.f && o->beta1 < 1.f && o->beta2 >= 0.f && o->beta2 < 1.f && o->eps > 0.f,
               RV_ERR_INVALID_ARG, "rv_surrogate_train: bad optimiser settings");
    RV_REQUIRE(((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG, "rv_surrogate_train: ws not 256-byte aligned");
    const TrainWs W = train_ws(o->batch);
    RV_REQUIRE(ws_bytes >= W.total, RV_ERR_WORKSPACE, "rv_surrogate_train: ws_bytes %zu < %zu", ws_bytes, W.total);
    const SurLayout L = sur_layout();
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_pad = train_pad(o->batch);
    const int n_slices = slices_for(n_pad);
    const int64_t n_parts = n_pad / (16 * kTrainNT);
    for (int64_t it = 0; it < o->steps; ++it) {
        const int64_t gstep = o->step0 + it;
        rv_status st = loss_grad_impl(params, x, d, T, o->batch, true, n_samples, o->seed, gstep, nullptr, nullptr,
                                      ws, W, s);
        if (st != RV_OK) return st;
        // cosine-decayed step size and bias corrections (host arithmetic, FP64)
        double lr = o->lr;
        if (o->total_steps > 0) {
            double t = (double)std::min<int64_t>(std::max<int64_t>(gstep, 0), o->total_steps) / (double)o->total_steps;
            lr = o->lr_min + 0.5 * (o->lr - o->lr_min) * (1.0 + std::cos(3.14159265358979323846 * t));
        }
        const double tt = (double)(gstep + 1);
        const float c1 = (float)(1.0 - std::pow((double)o->beta1, tt));
        const float c2 = (float)(1.0 - std::pow((double)o->beta2, tt));
        hipLaunchKernelGGL(k_adam_pack, dim3(blocks_for(kNParams, 256)), dim3(256), 0, s, at<float>(ws, W.partial),
                           n_slices, at<float>(params, L.master), at<float>(params, L.m), at<float>(params, L.v),
                           at<uint16_t>(params, L.fwd), at<uint16_t>(params, L.bwd), (float)lr, o->beta1, o->beta2,
                           o->eps, c1, c2, at<float>(ws, W.loss_part), n_parts, (int64_t)o->batch,
                           loss_log ? loss_log + it : nullptr);
        st = check_launch("rv_surrogate_train");
        if (st != RV_OK) return st;
    }
    return RV_OK;
}

extern "C" rv_status rv_surrogate_infer_xd(const void *params, const float *x, const float *d, int64_t n, float *vis,
                                           float *unc, void *stream) {
    clear_error();
    RV_REQUIRE(params && vis && (n == 0 || (x && d)), RV_ERR_INVALID_ARG, "rv_surrogate_infer_xd: null argument");
    RV_REQUIRE(n >= 0, RV_ERR_INVALID_ARG, "rv_surrogate_infer_xd: n < 0");
    if (n == 0) return RV_OK;
    const SurLayout L = sur_layout();
    FwdArgs fa{};
    fa.master = at<float>(params, L.master);
    fa.fwd = at<u32x4>(params, L.fwd);
    fa.header = at<float>(params, L.header);
    fa.n = n;
    fa.x = x;
    fa.d = d;
    fa.vis = vis;
    fa.unc = unc;
    for (int64_t off = 0; off < n; off += kLaunchSamples) {
        fa.s_off = off;
        const int64_t cnt = std::min(kLaunchSamples, n - off);
        hipLaunchKernelGGL(k_mlp_forward<kModeXd>, dim3(blocks_for(cnt, kInferSamples)), dim3(kInferWaves * 64), 0,
                           (hipStream_t)stream, fa);
    }
    return check_launch("rv_surrogate_infer_xd");
}

extern "C" rv_status rv_surrogate_infer(const void *params, const void *bvh, const rv_gaussians *g, const float *dirs,
                                        int32_t K, const rv_trace_params *p, int64_t q_begin, int64_t q_count,
                                        float tau, float *vis, float *unc, int64_t *n_fallback, void *ws,
                                        size_t ws_bytes, void *stream) {
    clear_error();
    RV_REQUIRE(params && g && dirs && p && vis, RV_ERR_INVALID_ARG, "rv_surrogate_infer: null argument");
    RV_REQUIRE(g->mean && g->log_scale && g->n >= 1 && g->n <= RV_MAX_GAUSSIANS && K >= 1, RV_ERR_INVALID_ARG,
               "rv_surrogate_infer: bad scene (null arrays, n out of range or K < 1)");
    RV_REQUIRE(p->dir_mode == 0 || (p->dir_mode == 1 && g->normal), RV_ERR_INVALID_ARG,
               "rv_surrogate_infer: bad dir_mode or missing normals");
    RV_REQUIRE(p->sigma_cut > 0.0f && p->sigma_cut <= kBuildSigma && p->alpha_min > 0.0f && p->alpha_max < 1.0f &&
                   p->T_min >= 0.0f && p->T_min < 1.0f,
               RV_ERR_INVALID_ARG, "rv_surrogate_infer: bad trace parameters");
    RV_REQUIRE(q_begin >= 0 && q_count >= 0 && q_begin + q_count <= g->n * (int64_t)K, RV_ERR_INVALID_ARG,
               "rv_surrogate_infer: query range outside [0, n*K)");
    if (q_count == 0) return RV_OK;
    RV_REQUIRE(ws && ((uintptr_t)ws % kAlign) == 0, RV_ERR_INVALID_ARG, "rv_surrogate_infer: ws missing or unaligned");
    RV_REQUIRE(ws_bytes >= rv_surrogate_infer_workspace_bytes(q_count), RV_ERR_WORKSPACE,
               "rv_surrogate_infer: ws_bytes %zu < %zu", ws_bytes, rv_surrogate_infer_workspace_bytes(q_count));
    const SurLayout L = sur_layout();
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *count = at<unsigned long long>(ws, 0);
    unsigned long long *queues = at<unsigned long long>(ws, 64);
    int64_t *list = at<int64_t>(ws, kAlign);
    uint8_t *flag = at<uint8_t>(ws, kAlign + align_up((size_t)q_count * sizeof(int64_t)));
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(256), 0, s, reinterpret_cast<float *>(count), (int64_t)2, 0.0f);
    FwdArgs fa{};
    fa.master = at<float>(params, L.master);
    fa.fwd = at<u32x4>(params, L.fwd);
    fa.header = at<float>(params, L.header);
    fa.n = q_count;
    fa.vis = vis;
    fa.unc = unc;
    fa.gmean = g->mean;
    fa.gnormal = p->dir_mode ? g->normal : nullptr;
    fa.dirs = dirs;
    fa.K = K;
    fa.dir_mode = p->dir_mode;
    fa.q_begin = q_begin;
    fa.tau = tau;
    fa.fb_flag = bvh ? flag : nullptr;
    for (int64_t off = 0; off < q_count; off += kLaunchSamples) {
        fa.s_off = off;
        const int64_t cnt = std::min(kLaunchSamples, q_count - off);
        hipLaunchKernelGGL(k_mlp_forward<kModeGrid>, dim3(blocks_for(cnt, kInferSamples)), dim3(kInferWaves * 64), 0,
                           s, fa);
    }
    if (bvh) {
        const Cuts c = make_cuts(*p);
        // the compacted fallback list holds positions s; the ray is q_begin + s
        const BvhLayout BL = bvh_layout(g->n);
        const int64_t rows_blocks = std::min<int64_t>(((g->n + 63) / 64 + 3) / 4, int64_t(1) << 16);
        hipLaunchKernelGGL(k_fallback_rows, dim3((unsigned)rows_blocks), dim3(256), 0, s, at<float>(bvh, BL.header),
                           at<float4>(bvh, BL.leaf_rec),
                           g->n, (int)K, q_begin, q_count, flag, count, list);
        launch_trace_list(bvh, g, dirs, K, c, (const int64_t *)list, q_count, (const unsigned long long *)count,
                          q_begin, true, vis, queues, s);
        if (n_fallback)
            hipLaunchKernelGGL(k_store_count, dim3(1), dim3(64), 0, s, (const unsigned long long *)count, n_fallback);
    } else if (n_fallback) {
        hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, s, reinterpret_cast<float *>(n_fallback), (int64_t)2,
                           0.0f);
    }
    return check_launch("rv_surrogate_infer");
}

extern "C" rv_status rv_ray_setup(const rv_gaussians *g, const float *dirs, int32_t K, const rv_trace_params *p,
                                  const int64_t *ray_ids, int64_t n, float *out_o, float *out_d, void *stream) {
    clear_error();
    RV_REQUIRE(g && dirs && p && g->mean, RV_ERR_INVALID_ARG, "rv_ray_setup: null argument");
    RV_REQUIRE(g->n >= 1 && g->n <= RV_MAX_GAUSSIANS && K >= 1 && n >= 0, RV_ERR_INVALID_ARG,
               "rv_ray_setup: bad sizes");
    RV_REQUIRE(p->dir_mode == 0 || (p->dir_mode == 1 && g->normal), RV_ERR_INVALID_ARG,
               "rv_ray_setup: bad dir_mode or missing normals");
    if (n == 0) return RV_OK;
    RV_REQUIRE(ray_ids && out_o && out_d, RV_ERR_INVALID_ARG, "rv_ray_setup: null ids or outputs");
    hipLaunchKernelGGL(k_ray_setup, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, g->mean,
                       p->dir_mode ? g->normal : nullptr, g->n, dirs, K, p->dir_mode, ray_ids, n, out_o, out_d);
    return check_launch("rv_ray_setup");
}
