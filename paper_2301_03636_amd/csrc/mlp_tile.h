// The fused tile pipeline of the cost model: a persistent workgroup loops
// over tiles of M variant rows; for each tile it builds the standardized
// input (from descriptors or from features), runs every hidden layer on the
// matrix cores with the activations held in LDS, reduces the output layer
// with wavefront shuffles, and either stores the predictions or folds them
// into per-kernel argmin keys.
//
// Matrix-core mapping (v_mfma_f32_32x32x{2f32,16_bf16,64_f8f6f4}): operand A
// is a 32-row block of the layer's weights W_l[n][k] (rows = output neurons),
// operand B a 32-column block of the transposed activations (columns =
// variants), so D[n][m] = sum_k W[n][k] h[m][k]. Lane l of an operand holds
// row (or column) l % 32; how the k values are spread over the two lane
// halves is described at Geo below. D's lane l holds column m = l % 32 and
// rows n = 8 * (r / 4) + 4 * (l / 32) + r % 4 for accumulator r = 0..15.
// Weights are pre-packed fragment-major so each A operand is one contiguous
// 64-lane load from global memory (L2-resident: every tile re-reads them);
// activations live in LDS as [m][k] rows padded by one 16-byte bank step so
// the 32 rows of a B operand fall in distinct banks.
#pragma once

#include <type_traits>

#include "features.h"

namespace adv {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef __bf16 v16bf __attribute__((ext_vector_type(16)));

enum {
    PREC_FP32 = ADVISOR_FP32,
    PREC_BF16 = ADVISOR_BF16,
    PREC_FP8 = ADVISOR_FP8_E4M3,
    PREC_X3 = ADVISOR_BF16X3
};
enum { SRC_DESC = 0, SRC_FEAT = 1 };
// SINK_GROUP: several models that share the input tile (same precision,
// tile width and Z-score statistics) ranked in one pass, each exactly as
// SINK_RANK would rank it.
enum { SINK_PRED = 0, SINK_RANK = 1, SINK_TRAIN = 2, SINK_GROUP = 3 };

// Per-precision fragment geometry. A lane loads KV consecutive k values in
// one vector (16 or 32 bytes); each matrix-core op consumes KL of them per
// lane, so one vector feeds KV / KL ops. A k-group of KG = 2 * KV inputs is
// split as: lane half h holds k = group * KG + h * KV + e, e < KV, and op t of
// the group uses e in [t * KL, (t + 1) * KL). A and B use the same mapping,
// which is all the dot product needs. EB bytes per element; PAD is the LDS
// row padding (one 16-byte bank step).
template <int P> struct Geo;
template <> struct Geo<PREC_FP32> {
    using Vec = v4f;
    static constexpr int KV = 4, KL = 1, KG = 8, EB = 4, PAD = 16;
};
template <> struct Geo<PREC_BF16> {
    using Vec = v8bf;
    static constexpr int KV = 8, KL = 8, KG = 16, EB = 2, PAD = 16;
};
template <> struct Geo<PREC_FP8> {
    using Vec = v8i;
    static constexpr int KV = 32, KL = 32, KG = 64, EB = 1, PAD = 16;
};
// bf16x3: every value is a pair of bf16 (its rounding hi and the rounding lo
// of the remainder). Storage runs in chunks of 8 consecutive k (or neuron)
// values: 16 bytes of hi parts, then 16 bytes of lo parts, so EB = 4 and the
// fp32 address arithmetic of a k-group holds; a vector is one chunk (the
// 8 hi parts in elements 0-7, the lo parts in 8-15).
template <> struct Geo<PREC_X3> {
    using Vec = v16bf;
    static constexpr int KV = 8, KL = 8, KG = 16, EB = 4, PAD = 16;
};

// Byte offset of the hi part of value i in bf16x3 storage (its lo part is 16
// bytes further on).
__host__ __device__ __forceinline__ constexpr int64_t x3_off(int64_t i)
{
    return (i >> 3) * 32 + (i & 7) * 2;
}

__device__ __forceinline__ v16f mma(float a, float b, v16f c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v16f mma(v8bf a, v8bf b, v16f c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// bf16x3: a*b ~ hi(a)hi(b) + hi(a)lo(b) + lo(a)hi(b) (lo*lo, about 2^-18 of
// the product, is dropped), the small terms first
__device__ __forceinline__ v16f mma(v16bf a, v16bf b, v16f c)
{
    const v8bf ah = __builtin_shufflevector(a, a, 0, 1, 2, 3, 4, 5, 6, 7);
    const v8bf al = __builtin_shufflevector(a, a, 8, 9, 10, 11, 12, 13, 14, 15);
    const v8bf bh = __builtin_shufflevector(b, b, 0, 1, 2, 3, 4, 5, 6, 7);
    const v8bf bl = __builtin_shufflevector(b, b, 8, 9, 10, 11, 12, 13, 14, 15);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
}
__device__ __forceinline__ v16f mma(v8i a, v8i b, v16f c)
{
    // OCP e4m3 for both operands, no block scales
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// Precision of the first layer (K = 32 input features): the model's own
// for fp32 and bf16x3, bf16 otherwise (the fp8 k-step of 64 does not fit 32
// inputs).
template <int P> struct FirstP {
    static constexpr int value = (P == PREC_FP32 || P == PREC_X3) ? P : PREC_BF16;
};

// Packed weight index of element (n, k) of a layer with Kp (padded) inputs:
// fragment-major, [n-block][k-group][lane][KV].
template <int P>
__host__ __device__ __forceinline__ int64_t pack_index(int n, int k, int Kp)
{
    constexpr int KV = Geo<P>::KV, KG = Geo<P>::KG;
    const int nb = n >> 5, kg = k / KG, kk = k % KG;
    const int lane = (n & 31) + 32 * (kk / KV);
    return (((int64_t)nb * (Kp / KG) + kg) * 64 + lane) * KV + (kk % KV);
}

// OCP e4m3 (1-4-3, bias 7, max 448, no infinities) from fp32 with
// round-to-nearest-even and saturation to +-448; NaN maps to 0x7f.
__device__ __forceinline__ uint32_t f32_to_e4m3(float x)
{
    uint32_t u = __float_as_uint(x);
    const uint32_t sign = (u >> 24) & 0x80u;
    u &= 0x7fffffffu;
    if (u > 0x7f800000u) return 0x7fu;              // NaN
    if (u >= 0x43e00000u) return sign | 0x7eu;      // >= 448 (and inf): saturate
    if (u < 0x3c800000u) {                          // below 2^-6: subnormal range
        // value = m * 2^-9 with m in [0, 8): round x * 2^9 to nearest even
        const float y = __uint_as_float(u) * 512.0f;
        const float r = __builtin_rintf(y);        // RNE, exact in fp32
        return sign | (uint32_t)r;                 // r = 8 encodes 2^-6 (exponent 1)
    }
    // normal: keep 3 mantissa bits, RNE on the 20 dropped bits
    const uint32_t lsb = (u >> 20) & 1u;
    u += 0x7ffffu + lsb;
    const uint32_t e = (u >> 23) - 127 + 7;
    const uint32_t mant = (u >> 20) & 7u;
    const uint32_t code = (e << 3) | mant;
    return sign | (code > 0x7eu ? 0x7eu : code);
}

struct TileArgs {
    // input
    const int64_t *kdesc;
    const int64_t *vdesc;
    const int64_t *feat;
    const int64_t *offsets;
    int64_t n_k;
    int64_t n_rows;
    // network
    NetView net;
    // output
    float *pred;          // [n_rows] or null
    uint64_t *keys;       // [n_k] argmin keys (rank)
    // training forward: transposed copies of what each layer consumed,
    // x^T [32][save_ld] then h_l^T [W][save_ld] per hidden layer, in the
    // layer's compute precision; rows >= n_rows are stored as zero
    void *save_x;
    void *save_h;
    int64_t save_ld;
    // and, when not null, the ReLU masks of hidden layers 0 .. n_hidden-2:
    // word [(l * W / 32 + b) * save_ld + row] has bit t set when neuron
    // 32 b + t of layer l is positive (as stored) for that row
    uint32_t *save_mask;
};

// A grouped pass: the descriptors, segments and statistics of `base` (its
// `net` is the first model), then per model its network and its outputs.
constexpr int GROUP_MAX = 8;
struct GroupArgs {
    TileArgs base;
    int n_models;
    NetView nets[GROUP_MAX];
    uint64_t *keys[GROUP_MAX];   // [n_k] argmin keys of each model
    float *pred[GROUP_MAX];      // [n_rows] predictions of each model, or null
};

template <int SINK> struct KernelArgs { using type = TileArgs; };
template <> struct KernelArgs<SINK_GROUP> { using type = GroupArgs; };
__host__ __device__ __forceinline__ const TileArgs &base_args(const TileArgs &a) { return a; }
__host__ __device__ __forceinline__ const TileArgs &base_args(const GroupArgs &a) { return a.base; }
__device__ __forceinline__ int group_size(const TileArgs &) { return 1; }
__device__ __forceinline__ int group_size(const GroupArgs &a) { return a.n_models; }
__device__ __forceinline__ const NetView &group_net(const TileArgs &a, int) { return a.net; }
__device__ __forceinline__ const NetView &group_net(const GroupArgs &a, int t) { return a.nets[t]; }
__device__ __forceinline__ uint64_t *group_keys(const TileArgs &a, int) { return a.keys; }
__device__ __forceinline__ uint64_t *group_keys(const GroupArgs &a, int t) { return a.keys[t]; }
__device__ __forceinline__ float *group_pred(const TileArgs &a, int) { return a.pred; }
__device__ __forceinline__ float *group_pred(const GroupArgs &a, int t) { return a.pred[t]; }

// Store one value of a saved activation (transposed layout) in precision P.
template <int P>
__device__ __forceinline__ void save_elem(void *base, int64_t idx, float v)
{
    if constexpr (P == PREC_FP32)
        reinterpret_cast<float *>(base)[idx] = v;
    else
        reinterpret_cast<__bf16 *>(base)[idx] = (__bf16)v;
}

template <int P, int W, int M, int NWAVES, int NSPLIT_ = 1, bool VPF_ = false, bool BL_ = false>
struct TileCfg {
    static constexpr int NSPLIT = NSPLIT_;                 // passes over a wave's neurons
    using G = Geo<P>;
    using G0 = Geo<FirstP<P>::value>;
    static constexpr int NB = W / 32;                      // n-blocks of a layer
    static constexpr int MB = M / 32;                      // m-blocks of a tile
    static constexpr int WN = NB < NWAVES ? NB : NWAVES;   // waves along n
    static constexpr int WM = NWAVES / WN;                 // waves along m
    static constexpr int NBW = NB / WN;                    // n-blocks per wave
    static constexpr int MBW = MB / WM;                    // m-blocks per wave
    static_assert(NB % WN == 0 && MB % WM == 0 && NWAVES % WN == 0, "tile split");
    static constexpr int NBP = NBW / NSPLIT;               // n-blocks per pass
    static_assert(NBW % NSPLIT == 0, "passes split the wave's n-blocks evenly");
    static constexpr int XS = 32 * G0::EB + G0::PAD;       // input row stride (bytes)
    static constexpr int AS = W * G::EB + G::PAD;          // activation row stride (bytes)
    static constexpr int THREADS = NWAVES * 64;
    static constexpr int PARTS = THREADS / M;              // threads per row in the input stage
    static_assert(PARTS >= 1 && NFEAT % PARTS == 0, "input split");
    static constexpr int FPP = NFEAT / PARTS;              // features per thread
    static constexpr size_t ACT_BYTES = (size_t)M * AS;
    static constexpr size_t LDS_BASE = (size_t)M * XS + ACT_BYTES + (size_t)WN * M * 4 + M * 8;
    // descriptor prefetch (VPF): the next tile's variant rows (M x 64 B) and
    // the output-layer weights
    static constexpr bool VPF = VPF_;
    static constexpr size_t VST_BYTES = VPF ? (size_t)M * 64 : 0;
    // bias staging (BL): every hidden layer's bias and the output-layer
    // weights copied into LDS once per workgroup, for epilogues that add the
    // bias after the products (fp8)
    static constexpr bool BL = BL_;
    static constexpr size_t HW_BYTES = (VPF || BL) ? (size_t)W * 4 : 0;
    static constexpr size_t BIAS_BYTES = BL ? (size_t)(MAX_LAYERS - 1) * W * 4 : 0;
    static constexpr size_t LDS = LDS_BASE + VST_BYTES + HW_BYTES + BIAS_BYTES;
    static_assert(M % 32 == 0 && (M * XS) % 16 == 0 && ACT_BYTES % 16 == 0, "LDS alignment");
    static_assert(LDS <= 160 * 1024, "tile does not fit the 160 KiB of LDS");
};

// Waves per SIMD the register allocation of a tile kernel aims at: the
// workgroups that fit a CU's LDS times the waves each puts on a SIMD, between
// one and two (two leave 256 registers per wave). Computed apart from
// TileCfg so that naming a kernel does not check its tile split.
template <int P, int W, int M, int NWAVES>
constexpr int tile_waves_per_simd()
{
    constexpr int xs = 32 * Geo<FirstP<P>::value>::EB + Geo<FirstP<P>::value>::PAD;
    constexpr int as = W * Geo<P>::EB + Geo<P>::PAD;
    constexpr int wn = W / 32 < NWAVES ? W / 32 : NWAVES;
    constexpr size_t lds = (size_t)M * xs + (size_t)M * as + (size_t)wn * M * 4 + M * 8;
    constexpr int blocks = (int)((160 * 1024) / lds);
    constexpr int w = blocks * NWAVES / 4;
    return w < 1 ? 1 : (w > 2 ? 2 : w);
}

// Whether the fused kernel reading descriptors stages the next tile's
// variant rows in LDS: only where the staging (plus the output weights it
// moves to LDS) leaves the workgroups per CU unchanged, and not for fp8
// tiles (their scaled last layer reads its bias in the epilogue, and the
// extra registers spill).
template <int P, int W, int M, int NWAVES>
constexpr bool tile_vdesc_prefetch()
{
    constexpr int xs = 32 * Geo<FirstP<P>::value>::EB + Geo<FirstP<P>::value>::PAD;
    constexpr int as = W * Geo<P>::EB + Geo<P>::PAD;
    constexpr int wn = W / 32 < NWAVES ? W / 32 : NWAVES;
    constexpr size_t base = (size_t)M * xs + (size_t)M * as + (size_t)wn * M * 4 + M * 8;
    constexpr size_t extra = (size_t)M * 64 + (size_t)W * 4;
    constexpr int by_regs = tile_waves_per_simd<P, W, M, NWAVES>() * 4 / NWAVES;
    constexpr int r = by_regs < 1 ? 1 : by_regs;
    constexpr int b0 = (int)((160 * 1024) / base), b1 = (int)((160 * 1024) / (base + extra));
    return P != PREC_FP8 && base + extra <= 160 * 1024 && (b0 < r ? b0 : r) == (b1 < r ? b1 : r);
}

// Whether an fp8 tile kernel stages its biases and output-layer weights in
// LDS (their epilogues read the bias after the products): only where that
// leaves the workgroups per CU unchanged.
template <int P, int W, int M, int NWAVES>
constexpr bool tile_bias_lds()
{
    constexpr int xs = 32 * Geo<FirstP<P>::value>::EB + Geo<FirstP<P>::value>::PAD;
    constexpr int as = W * Geo<P>::EB + Geo<P>::PAD;
    constexpr int wn = W / 32 < NWAVES ? W / 32 : NWAVES;
    constexpr size_t base = (size_t)M * xs + (size_t)M * as + (size_t)wn * M * 4 + M * 8;
    constexpr size_t extra = (size_t)W * 4 + (size_t)(MAX_LAYERS - 1) * W * 4;
    constexpr int by_regs = tile_waves_per_simd<P, W, M, NWAVES>() * 4 / NWAVES;
    constexpr int r = by_regs < 1 ? 1 : by_regs;
    constexpr int b0 = (int)((160 * 1024) / base), b1 = (int)((160 * 1024) / (base + extra));
    return P == PREC_FP8 && base + extra <= 160 * 1024 && (b0 < r ? b0 : r) == (b1 < r ? b1 : r);
}

// 16-byte-aligned LDS vector load (an fp8 or bf16x3 vector is two 16-byte
// halves).
template <int P>
__device__ __forceinline__ typename Geo<P>::Vec lds_vec(const unsigned char *p)
{
    using V = typename Geo<P>::Vec;
    if constexpr (sizeof(V) == 32) {
        typedef int v4i_ __attribute__((ext_vector_type(4)));
        const v4i_ lo = *reinterpret_cast<const v4i_ *>(p);
        const v4i_ hi = *reinterpret_cast<const v4i_ *>(p + 16);
        v8i r;
        r[0] = lo[0]; r[1] = lo[1]; r[2] = lo[2]; r[3] = lo[3];
        r[4] = hi[0]; r[5] = hi[1]; r[6] = hi[2]; r[7] = hi[3];
        return __builtin_bit_cast(V, r);
    } else {
        return *reinterpret_cast<const V *>(p);
    }
}

// Depth of the weight ring of a layer with K inputs: two k-groups ahead when
// the group count is even and a vector fits 16 bytes, else one (32-byte fp8).
template <int PL, int K>
constexpr int ring_depth()
{
    constexpr int kgroups = K / Geo<PL>::KG;
    return (kgroups % 2 == 0 && sizeof(typename Geo<PL>::Vec) <= 16) ? 2 : 1;
}

// Request the first ring_depth k-groups of the weight vectors of n-blocks
// nb0 .. nb0 + NBW - 1 (they do not depend on the activations, so this can be
// issued before the layer's input is ready).
template <int PL, int K, int NBW>
__device__ __forceinline__ void ring_load(const typename Geo<PL>::Vec *__restrict__ wl, int nb0,
                                          int lane,
                                          typename Geo<PL>::Vec (&ring)[ring_depth<PL, K>()][NBW])
{
    constexpr int KGROUPS = K / Geo<PL>::KG;
    const typename Geo<PL>::Vec *abase = wl + (int64_t)nb0 * KGROUPS * 64 + lane;
#pragma unroll
    for (int p = 0; p < ring_depth<PL, K>(); ++p)
#pragma unroll
        for (int i = 0; i < NBW; ++i) ring[p][i] = abase[((int64_t)i * KGROUPS + p) * 64];
}

// One k-group of layer_mma: take the weight vectors of group kg from ring
// slot U and request those of group kg + PF into it, read the LDS operands of
// group kg + 1 (all before the multiplies, or for bf16 each m-block's right
// after its own), and multiply. The first group starts from `init` (the bias)
// through the matrix core's C operand, so the accumulators need no copies.
template <int PL, int K, int NBW, int MBW, int U, bool FIRST>
__device__ __forceinline__ void mma_group(const typename Geo<PL>::Vec *__restrict__ abase,
                                          const unsigned char *bbase, int stride, int kg,
                                          typename Geo<PL>::Vec (&ring)[ring_depth<PL, K>()][NBW],
                                          typename Geo<PL>::Vec (&bcur)[MBW],
                                          v16f (&acc)[NBW][MBW], const v16f (&init)[NBW])
{
    using G = Geo<PL>;
    using V = typename G::Vec;
    constexpr int KGROUPS = K / G::KG;
    constexpr int PF = ring_depth<PL, K>();
    V a[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) a[i] = ring[U][i];
    if (kg + PF < KGROUPS) {
#pragma unroll
        for (int i = 0; i < NBW; ++i) ring[U][i] = abase[((int64_t)i * KGROUPS + kg + PF) * 64];
    }
    if constexpr (PL == PREC_BF16 || (PL == PREC_FP8 && MBW >= 4)) {
        // bf16, and fp8 with four or more m-blocks: single-buffered B
        // operands. Those of m-block j for group kg + 1 are read into bcur[j]
        // as soon as group kg's multiplies by it are issued, which frees the
        // registers of a second buffer (measured: 4-15% faster bf16 tiles;
        // the 128-row fp8 512-wide tile stops spilling, 7.74 -> 7.62 ms;
        // fp32 and the other fp8 tiles are as fast or faster with the double
        // buffer below)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < MBW; ++j) {
#pragma unroll
            for (int i = 0; i < NBW; ++i) {
                if constexpr (PL == PREC_FP32) {
                    acc[i][j] = mma(a[i][0], bcur[j][0], FIRST ? init[i] : acc[i][j]);
#pragma unroll
                    for (int t = 1; t < G::KV; ++t) acc[i][j] = mma(a[i][t], bcur[j][t], acc[i][j]);
                } else {
                    acc[i][j] = mma(a[i], bcur[j], FIRST ? init[i] : acc[i][j]);
                }
            }
            if (kg + 1 < KGROUPS)
                bcur[j] = lds_vec<PL>(bbase + (size_t)j * 32 * stride + (kg + 1) * G::KG * G::EB);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        V bnext[MBW];
        if (kg + 1 < KGROUPS) {
#pragma unroll
            for (int j = 0; j < MBW; ++j)
                bnext[j] = lds_vec<PL>(bbase + (size_t)j * 32 * stride + (kg + 1) * G::KG * G::EB);
        }
        // keep the requests above ahead of the multiplies below: without this
        // the scheduler sinks each load next to its first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < NBW; ++i)
#pragma unroll
            for (int j = 0; j < MBW; ++j) {
                if constexpr (PL == PREC_FP32) {
                    acc[i][j] = mma(a[i][0], bcur[j][0], FIRST ? init[i] : acc[i][j]);
#pragma unroll
                    for (int t = 1; t < G::KV; ++t) acc[i][j] = mma(a[i][t], bcur[j][t], acc[i][j]);
                } else {
                    acc[i][j] = mma(a[i], bcur[j], FIRST ? init[i] : acc[i][j]);
                }
            }
        if (kg + 1 < KGROUPS) {
#pragma unroll
            for (int j = 0; j < MBW; ++j) bcur[j] = bnext[j];
        }
    }
}

// acc[i][j] = bias + W (A vectors streamed from global/L2) x act^T (B vectors
// from LDS) over the K inputs of one layer; a null bias starts from zero.
// Software-pipelined: `ring` arrives holding the weight vectors of the first
// PF k-groups (ring_load), those of k-group kg + PF are requested while group
// kg is multiplied (PF dividing the group count so every slot index is a
// compile-time constant), and the LDS operands of kg + 1 are read while kg is
// multiplied.
template <int PL, int K, int NBW, int MBW>
__device__ __forceinline__ void layer_mma(const typename Geo<PL>::Vec *__restrict__ wl,
                                          const unsigned char *lds_in, int stride, int nb0,
                                          int mb0, int lane, v16f (&acc)[NBW][MBW],
                                          const float *__restrict__ bias,
                                          typename Geo<PL>::Vec (&ring)[ring_depth<PL, K>()][NBW])
{
    using G = Geo<PL>;
    using V = typename G::Vec;
    constexpr int KGROUPS = K / G::KG;
    constexpr int PF = ring_depth<PL, K>();
    const int half = lane >> 5, col = lane & 31;
    // accumulator r of block i holds neuron (nb0 + i) * 32 + 8 * (r / 4) + 4 * half + r % 4
    v16f init[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
        init[i] = v16f{0};
        if (bias) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const v4f bv = *reinterpret_cast<const v4f *>(bias + (nb0 + i) * 32 + 8 * g + 4 * half);
#pragma unroll
                for (int e = 0; e < 4; ++e) init[i][4 * g + e] = bv[e];
            }
        }
    }
    const unsigned char *bbase = lds_in + (size_t)(mb0 * 32 + col) * stride + half * G::KV * G::EB;
    const V *abase = wl + (int64_t)nb0 * KGROUPS * 64 + lane;
    V bcur[MBW];
#pragma unroll
    for (int j = 0; j < MBW; ++j) bcur[j] = lds_vec<PL>(bbase + (size_t)j * 32 * stride);
    mma_group<PL, K, NBW, MBW, 0, true>(abase, bbase, stride, 0, ring, bcur, acc, init);
    if constexpr (PF == 2) mma_group<PL, K, NBW, MBW, 1, false>(abase, bbase, stride, 1, ring, bcur, acc, init);
    for (int kg0 = PF; kg0 < KGROUPS; kg0 += PF) {
        mma_group<PL, K, NBW, MBW, 0, false>(abase, bbase, stride, kg0, ring, bcur, acc, init);
        if constexpr (PF == 2)
            mma_group<PL, K, NBW, MBW, 1, false>(abase, bbase, stride, kg0 + 1, ring, bcur, acc, init);
    }
}

// layer_mma with its own ring load (no prefetch across calls).
template <int PL, int K, int NBW, int MBW>
__device__ __forceinline__ void layer_mma(const typename Geo<PL>::Vec *__restrict__ wl,
                                          const unsigned char *lds_in, int stride, int nb0,
                                          int mb0, int lane, v16f (&acc)[NBW][MBW],
                                          const float *__restrict__ bias = nullptr)
{
    typename Geo<PL>::Vec ring[ring_depth<PL, K>()][NBW];
    ring_load<PL, K, NBW>(wl, nb0, lane, ring);
    layer_mma<PL, K, NBW, MBW>(wl, lds_in, stride, nb0, mb0, lane, acc, bias, ring);
}

// Four consecutive neurons of one variant in a layer's activation precision
// (fp8: scaled by 1/s first), as held in registers until they are stored.
template <int P> struct Held;
template <> struct Held<PREC_FP32> { using T = v4f; };
template <> struct Held<PREC_BF16> { using T = v4bf; };
template <> struct Held<PREC_FP8> { using T = uint32_t; };
template <> struct Held<PREC_X3> { using T = v8bf; };  // hi parts in 0-3, lo parts in 4-7

template <int P>
__device__ __forceinline__ typename Held<P>::T pack4(v4f v, float qinv)
{
    if constexpr (P == PREC_FP32) {
        return v;
    } else if constexpr (P == PREC_BF16) {
        v4bf o;
        o[0] = (__bf16)v[0];
        o[1] = (__bf16)v[1];
        o[2] = (__bf16)v[2];
        o[3] = (__bf16)v[3];
        return o;
    } else if constexpr (P == PREC_X3) {
        v8bf o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            o[e] = (__bf16)v[e];
            o[4 + e] = (__bf16)(v[e] - (float)o[e]);  // the remainder is exact in fp32
        }
        return o;
    } else {
        // the values are ReLU outputs (>= 0, never NaN): clamping at 448
        // gives f32_to_e4m3's saturation, and the hardware pair conversion
        // then rounds to nearest even exactly as f32_to_e4m3 does for every
        // float in [0, 448]
        const float a0 = fminf(v[0] * qinv, 448.0f), a1 = fminf(v[1] * qinv, 448.0f);
        const float a2 = fminf(v[2] * qinv, 448.0f), a3 = fminf(v[3] * qinv, 448.0f);
        const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a0, a1, 0, false);
        return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a2, a3, lo, true);
    }
}

template <int P>
__device__ __forceinline__ void store_held(unsigned char *row, int n, typename Held<P>::T h)
{
    if constexpr (P == PREC_X3) {
        // n is a multiple of 4: the four hi parts, and the lo parts 16 bytes on
        *reinterpret_cast<v4bf *>(row + x3_off(n)) = __builtin_shufflevector(h, h, 0, 1, 2, 3);
        *reinterpret_cast<v4bf *>(row + x3_off(n) + 16) = __builtin_shufflevector(h, h, 4, 5, 6, 7);
    } else {
        *reinterpret_cast<typename Held<P>::T *>(row + n * Geo<P>::EB) = h;
    }
}

// Bias + ReLU have been applied; store four consecutive neurons of one
// variant into a next-layer activation row.
template <int P>
__device__ __forceinline__ void store4(unsigned char *row, int n, v4f v, float qinv)
{
    store_held<P>(row, n, pack4<P>(v, qinv));
}

// An fp8 layer's output that feeds another fp8 layer, quantized in one step:
// with sq = qs / s_next (or 1 / s_next for the unscaled first layer) and the
// bias bq already divided by s_next, the e4m3 codes of
// clamp(acc * sq + bq, 0, 448) (ReLU and saturation in one clamp).
__device__ __forceinline__ uint32_t quant4_fp8(v4f acc, bool scaled, float sq, v4f bq)
{
    v4f v;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        v[e] = __builtin_amdgcn_fmed3f(scaled ? __builtin_fmaf(acc[e], sq, bq[e]) : acc[e] * sq, 0.0f,
                                       448.0f);
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], lo, true);
}

// Transposed access to a tile's activations: an LDS tile is row-major
// ([M][W], rows of stride AS), the saved layouts are neuron-major
// (dst[n * ld + row], rows contiguous). The work unit of a thread is four
// consecutive neurons of two row groups (CE = 16 / element-size rows each) of
// one 128-byte line block (8 row groups): per row one 8-byte (bf16) or
// 16-byte (fp32) LDS access holds the four neurons, and each neuron's CE rows
// leave as one 16-byte vector. Lane bits 0-1 pick the row group within half
// a line block (the second row group of the unit is 4 further on), bits 2-5
// the neuron quad, so an LDS access of a wave meets each bank no more often
// than its width forces, and four consecutive lanes store 64 contiguous bytes
// of each neuron.
template <int P, int W, int M, int THREADS>
struct TUnits {
    using T = typename std::conditional<P == PREC_FP32, float, __bf16>::type;
    static constexpr int CE = 16 / (int)sizeof(T);  // rows of a row group
    static constexpr int RG = M / CE;               // row groups of a tile
    static constexpr int LINES = RG / 8;            // 128-byte line blocks per neuron
    static constexpr int QH = W / 64;               // neuron quads per 16 lanes
    static constexpr int UNITS = LINES * QH * 64;   // = RG * W / 8, whole waves
    static_assert(M % CE == 0 && RG % 8 == 0, "row groups come in line blocks of eight");
    static_assert(W % 64 == 0, "sixteen neuron quads per wave");
    static_assert(UNITS % THREADS == 0 || THREADS % UNITS == 0, "units split over whole waves");
    // unit c (c < UNITS): first row group, neuron quad, line block
    __device__ static void decode(int c, int &rg, int &nq, int &line)
    {
        const int v = c >> 6;
        line = v / QH;
        nq = (v % QH) * 16 + ((c >> 2) & 15);
        rg = line * 8 + (c & 3);
    }
};

typedef int v4i_t __attribute__((ext_vector_type(4)));

// Four neurons nq*4 .. nq*4+3 of rows m0 .. m0+CE-1 from a row-major LDS
// tile into one 16-byte vector per neuron (rows in order).
template <int P>
__device__ __forceinline__ void lds_gather4(const unsigned char *act, int as, int m0, int nq,
                                            v4i_t (&out)[4])
{
    if constexpr (P == PREC_FP32) {
        v4i_t r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            r[e] = *reinterpret_cast<const v4i_t *>(act + (size_t)(m0 + e) * as + nq * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) out[q][e] = r[e][q];
    } else {
        typedef unsigned v2u_ __attribute__((ext_vector_type(2)));
        v2u_ r[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            r[e] = *reinterpret_cast<const v2u_ *>(act + (size_t)(m0 + e) * as + nq * 8);
        // dword p of neuron q's vector = rows 2p (low half) and 2p + 1
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const v2u_ a = r[2 * p], b = r[2 * p + 1];
            out[0][p] = (int)((a[0] & 0xffffu) | (b[0] << 16));
            out[1][p] = (int)((a[0] >> 16) | (b[0] & 0xffff0000u));
            out[2][p] = (int)((a[1] & 0xffffu) | (b[1] << 16));
            out[3][p] = (int)((a[1] >> 16) | (b[1] & 0xffff0000u));
        }
    }
}

// The inverse of lds_gather4: four neuron vectors back into the rows.
template <int P>
__device__ __forceinline__ void lds_scatter4(unsigned char *act, int as, int m0, int nq,
                                             const v4i_t (&in)[4])
{
    if constexpr (P == PREC_FP32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v4i_t r;
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = in[q][e];
            *reinterpret_cast<v4i_t *>(act + (size_t)(m0 + e) * as + nq * 16) = r;
        }
    } else {
        typedef unsigned v2u_ __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const unsigned n0 = (unsigned)in[0][p], n1 = (unsigned)in[1][p];
            const unsigned n2 = (unsigned)in[2][p], n3 = (unsigned)in[3][p];
            v2u_ a, b;  // rows 2p and 2p + 1
            a[0] = (n0 & 0xffffu) | (n1 << 16);
            a[1] = (n2 & 0xffffu) | (n3 << 16);
            b[0] = (n0 >> 16) | (n1 & 0xffff0000u);
            b[1] = (n2 >> 16) | (n3 & 0xffff0000u);
            *reinterpret_cast<v2u_ *>(act + (size_t)(m0 + 2 * p) * as + nq * 8) = a;
            *reinterpret_cast<v2u_ *>(act + (size_t)(m0 + 2 * p + 1) * as + nq * 8) = b;
        }
    }
}

// Zero the elements of rows >= n_rows in a neuron vector of rows r0 ...
template <int P>
__device__ __forceinline__ v4i_t zero_rows_past(v4i_t v, int64_t r0, int64_t n_rows)
{
    if (r0 + 16 / (P == PREC_FP32 ? 4 : 2) <= n_rows) return v;
    if constexpr (P == PREC_FP32) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (r0 + e >= n_rows) v[e] = 0;
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            unsigned w = (unsigned)v[p];
            if (r0 + 2 * p >= n_rows) w &= 0xffff0000u;
            if (r0 + 2 * p + 1 >= n_rows) w &= 0x0000ffffu;
            v[p] = (int)w;
        }
    }
    return v;
}

// Copy a tile's activations [M][W] (LDS rows of stride AS) to the transposed
// global layout dst[n * ld + row0 + m] (rows >= n_rows as zero), by the
// units of TUnits.
template <int P, int W, int M, int THREADS, int AS>
__device__ __forceinline__ void copy_act_transposed(const unsigned char *act, void *dst,
                                                    int64_t ld, int64_t row0, int64_t n_rows,
                                                    int tid)
{
    using U = TUnits<P, W, M, THREADS>;
    using T = typename U::T;
    T *d = reinterpret_cast<T *>(dst);
    for (int c0 = tid; c0 < U::UNITS; c0 += THREADS) {
        int c = c0;
        asm volatile("" : "+v"(c));  // address math here, not hoisted out of the tile loop
        int rg, nq, line;
        U::decode(c, rg, nq, line);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int m0 = (rg + 4 * s) * U::CE;
            v4i_t v[4];
            lds_gather4<P>(act, AS, m0, nq, v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<v4i_t *>(d + (int64_t)(nq * 4 + q) * ld + row0 + m0) =
                    zero_rows_past<P>(v[q], row0 + m0, n_rows);
        }
    }
}

// Input stage of a tile: PARTS threads per row. Each reads the row's
// descriptors (from LDS when the kernel stages them, else global; repeated
// reads are cache hits), forms the row's integer features in registers, and
// standardizes its own FPP of them into the input tile in the first layer's
// precision; part 0 records the row's validity and kernel id.
template <class C, int P, int M, int SRC, int SINK>
__device__ __forceinline__ void tile_input(const TileArgs &args, int64_t row0, int tid,
                                           unsigned char *xin, int *meta_ok, int *meta_kid,
                                           const unsigned char *vst)
{
    constexpr int P0 = FirstP<P>::value;
    using G0 = Geo<P0>;
    constexpr bool VPF = C::VPF;
    const NetView &net = args.net;
    const int64_t n = args.n_rows;
    {
        // with M a multiple of 64 a wave's threads share one part: made known
        // to the compiler, the part becomes a scalar branch below
        const int r = tid % M;
        const int part = M % 64 == 0 ? __builtin_amdgcn_readfirstlane(tid / M) : tid / M;
        const int64_t row = row0 + r;
        const bool inrow = row < n;
        uint64_t fsel[C::FPP];
        bool ok = inrow;
        if constexpr (SRC == SRC_DESC && M % 64 == 0) {
            // one copy of the feature code per part: each copy keeps only the
            // arithmetic its FPP features need (the 64-bit division of the
            // launch-wave count, for one, lives in a single part), and only
            // part 0 checks the kernel segment it records in meta_ok (the
            // other parts' inputs of a row that fails it are never used)
            int kid = -1;
#pragma unroll
            for (int q = 0; q < C::FPP; ++q) fsel[q] = 0;
#pragma unroll
            for (int p = 0; p < C::PARTS; ++p)
                if (part == p && inrow) {
                    const int64_t *vrow = VPF ? reinterpret_cast<const int64_t *>(vst + (size_t)r * 64)
                                              : args.vdesc + row * VD;
                    Feat f;
                    ok = featurize_one(args.kdesc, vrow, args.n_k, f);
#pragma unroll
                    for (int q = 0; q < C::FPP; ++q) fsel[q] = f.f[p * C::FPP + q];
                    if (p == 0) {
                        const int64_t k = vrow[0];
                        kid = (int)k;  // in [0, n_k) when ok, and n_k < 2^31
                        if (SINK == SINK_RANK && ok)  // the variant must sit in its kernel's segment
                            ok = args.offsets[k] <= row && row < args.offsets[k + 1];
                    }
                }
            if (part == 0) {
                meta_ok[r] = ok ? 1 : 0;
                meta_kid[r] = kid;
            }
        } else if constexpr (SRC == SRC_DESC) {
            Feat f;
            int kid = -1;
            if (inrow) {
                const int64_t *vrow =
                    VPF ? reinterpret_cast<const int64_t *>(vst + (size_t)r * 64) : args.vdesc + row * VD;
                ok = featurize_one(args.kdesc, vrow, args.n_k, f);
                const int64_t k = vrow[0];
                kid = (int)k;  // in [0, n_k) when ok, and n_k < 2^31
                if (SINK == SINK_RANK && ok)  // the variant must sit in its kernel's segment
                    ok = args.offsets[k] <= row && row < args.offsets[k + 1];
            } else {
#pragma unroll
                for (int j = 0; j < NFEAT; ++j) f.f[j] = 0;
            }
            // this thread's FPP features (part is not a compile-time value)
#pragma unroll
            for (int q = 0; q < C::FPP; ++q) fsel[q] = 0;
#pragma unroll
            for (int j = 0; j < NFEAT; ++j)
                if (j / C::FPP == part) fsel[j % C::FPP] = f.f[j];
            if (part == 0) {
                meta_ok[r] = ok ? 1 : 0;
                meta_kid[r] = kid;
            }
        } else {
#pragma unroll
            for (int q = 0; q < C::FPP; ++q)
                fsel[q] = inrow ? (uint64_t)args.feat[row * NFEAT + part * C::FPP + q] : 0;
            if (part == 0) {
                meta_ok[r] = inrow ? 1 : 0;
                meta_kid[r] = -1;
            }
        }
        unsigned char *xr = xin + (size_t)r * C::XS + part * C::FPP * G0::EB;
#pragma unroll
        for (int q = 0; q < C::FPP; ++q) {
            const int j = part * C::FPP + q;
            const float x = ok ? zscore_fast((int64_t)fsel[q], net.mu[j], net.sigma[j]) : 0.0f;
            if constexpr (P0 == PREC_FP32) {
                reinterpret_cast<float *>(xr)[q] = x;
            } else if constexpr (P0 == PREC_X3) {
                unsigned char *xe = xin + (size_t)r * C::XS + x3_off(j);
                const __bf16 h = (__bf16)x;
                *reinterpret_cast<__bf16 *>(xe) = h;
                *reinterpret_cast<__bf16 *>(xe + 16) = (__bf16)(x - (float)h);
            } else {
                reinterpret_cast<__bf16 *>(xr)[q] = (__bf16)x;
            }
            if constexpr (SINK == SINK_TRAIN)
                save_elem<P0>(args.save_x, (int64_t)j * args.save_ld + row, inrow ? x : 0.0f);
        }
    }
}

// Output stage of a tile: one thread per row (whole waves, for the
// shuffles) adds the output bias to the waves' partial dot products (fixed
// order) and stores the prediction or folds it into the per-kernel argmin
// keys.
template <class C, int M, int SINK>
__device__ __forceinline__ void tile_output(const TileArgs &args, int64_t row0, int tid, int lane,
                                            int wave, const float *hpart, const int *meta_ok,
                                            const int *meta_kid, const float *head_b, float *pred,
                                            uint64_t *keys)
{
    const int64_t n = args.n_rows;
    if (wave < (M + 63) / 64) {
        const bool inrow = tid < M;
        const int64_t row = row0 + tid;
        float p = head_b[0];
        if (inrow) {
#pragma unroll
            for (int q = 0; q < C::WN; ++q) p += hpart[q * M + tid];
        }
        const bool ok = inrow && meta_ok[tid] != 0;
        if constexpr (SINK == SINK_PRED || SINK == SINK_TRAIN) {
            if (inrow && row < n) pred[row] = p;
        } else {
            if (inrow && row < n && pred) pred[row] = ok ? p : __builtin_nanf("");
            const bool take = ok && !__builtin_isnan(p);
            uint64_t key = ~0ull;
            if (take) {
                uint32_t u = __float_as_uint(p == 0.0f ? 0.0f : p);
                u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
                key = ((uint64_t)u << 32) | (uint32_t)row;
            }
            // segmented min over runs of equal kernel id within the wave
            // (inclusive scan with segment-head flags), then one atomic
            // per run from its last lane
            const int kid = take ? meta_kid[tid] : -1;
            const int prev = __shfl_up(kid, 1, 64);
            int head = (lane == 0) || (prev != kid);
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint64_t kup = __shfl_up(key, off, 64);
                const int hup = __shfl_up(head, off, 64);
                if (lane >= off && !head) {
                    key = kup < key ? kup : key;
                    head = hup;
                }
            }
            const int next = __shfl_down(kid, 1, 64);
            const bool last = (lane == 63) || (next != kid);
            if (last && kid >= 0 && kid < args.n_k && key != ~0ull)
                atomicMin(reinterpret_cast<unsigned long long *>(keys + kid),
                          (unsigned long long)key);
        }
    }
}

template <int P, int W, int M, int NWAVES, int NSPLIT, int SRC, int SINK>
__global__ __launch_bounds__(NWAVES * 64)
__attribute__((amdgpu_waves_per_eu(tile_waves_per_simd<P, W, M, NWAVES>()))) void
mlp_tiles_kernel(typename KernelArgs<SINK>::type kargs)
{
    static_assert(SINK != SINK_GROUP || SRC == SRC_DESC, "grouped passes rank descriptors");
    const TileArgs &args = base_args(kargs);
    // a grouped pass ranks each of its models as SINK_RANK does; it reads the
    // descriptors from global memory (the staged output weights would have
    // to be reloaded per model)
    constexpr int SK = SINK == SINK_GROUP ? SINK_RANK : SINK;
    constexpr bool VPF = SRC == SRC_DESC && SINK != SINK_GROUP &&
                         tile_vdesc_prefetch<P, W, M, NWAVES>();
    constexpr bool BL = SINK != SINK_GROUP && SINK != SINK_TRAIN &&
                        tile_bias_lds<P, W, M, NWAVES>();
    using C = TileCfg<P, W, M, NWAVES, NSPLIT, VPF, BL>;
    using G = typename C::G;
    constexpr int P0 = FirstP<P>::value;
    using G0 = Geo<P0>;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *xin = lds;                                   // [M][XS]
    unsigned char *act = xin + (size_t)M * C::XS;               // [M][AS]
    float *hpart = reinterpret_cast<float *>(act + C::ACT_BYTES);       // [WN][M]
    int *meta_ok = reinterpret_cast<int *>(hpart + C::WN * M);  // [M]
    int *meta_kid = meta_ok + M;                                // [M]
    unsigned char *vst = lds + C::LDS_BASE;                     // [M][64 B] (VPF)
    float *hw_lds = reinterpret_cast<float *>(vst + C::VST_BYTES);  // [W] (VPF or BL)
    float *bias_lds = hw_lds + (C::HW_BYTES / 4);               // [MAX_LAYERS - 1][W] (BL)

    const int tid0 = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid0 >> 6);
    const int wn = wave % C::WN, wm = wave / C::WN;
    const int nb0 = wn * C::NBW, mb0 = wm * C::MBW;
    const int64_t n = args.n_rows;
    // the training forward covers every row of the saved buffers (zeros past n)
    const int64_t ntiles = SINK == SINK_TRAIN ? args.save_ld / M : (n + M - 1) / M;
    // Per-thread values are re-derived from an opaque copy of the thread
    // index at the top of every tile and layer (opaque_tid): the addresses
    // built from them are then computed where they are used instead of being
    // hoisted out of the tile loop, where they would sit in registers (or
    // spill) through every layer's multiplies.
    auto opaque_tid = [&]() {
        int t = tid0;
        asm volatile("" : "+v"(t));
        return t;
    };
    int tid = tid0, lane = tid0 & 63, half = lane >> 5, col = lane & 31;

    // weight rings of the first layer and of the hidden layers: each call of
    // layer_mma finds its first k-groups already requested, by the call before
    // it (across the epilogue and the barriers, which do not wait for global
    // loads) or, for the first layer, at the end of the input stage. Tiles
    // whose accumulators fill most registers (more than 4 blocks of 32 x 32)
    // request them at the call instead: the ring would spill there.
    constexpr bool XPF = C::NBP * C::MBW <= 4;
    using R0 = typename G0::Vec;
    using RH = typename G::Vec;
    R0 ring0[ring_depth<P0, 32>()][C::NBP];
    RH ringh[ring_depth<P, W>()][C::NBP];

    // Descriptor prefetch: the variant rows of a tile are one contiguous run
    // of M * 64 bytes, copied straight into LDS by direct-to-LDS loads (lane
    // l of a wave writes 16 bytes at the wave's base + 16 l); no registers
    // hold them. The next tile's copy is issued after the last layer's
    // matrix loop; nothing waited on before the next input stage is a vector
    // load issued after it (the output weights are read from LDS), so it
    // completes behind the last epilogue and the output stage.
    auto issue_vdesc = [&](int64_t t) {
        const int64_t r0 = t * M;
        for (int c0 = wave * 64; c0 < M * 4; c0 += C::THREADS) {
            const int c = c0 + lane;
            if (r0 + c / 4 < n)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(args.vdesc + r0 * VD + 2 * c),
                    (__attribute__((address_space(3))) void *)(vst + (size_t)c0 * 16), 16, 0, 0);
        }
    };
    if constexpr (VPF) {
        for (int i = tid; i < W; i += C::THREADS) hw_lds[i] = args.net.head_w[i];
        if ((int64_t)blockIdx.x < ntiles) issue_vdesc(blockIdx.x);
    }
    if constexpr (BL) {
        // read before the first tile's barriers, which order them for every wave
        for (int i = tid; i < W; i += C::THREADS) hw_lds[i] = args.net.head_w[i];
        for (int l = 0; l < args.net.n_hidden; ++l) {
            const float sc = l + 1 < args.net.n_hidden ? args.net.qinv[l] : 1.0f;
            for (int i = tid; i < W; i += C::THREADS) bias_lds[l * W + i] = args.net.b[l][i] * sc;
        }
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row0 = tile * M;
        if constexpr (VPF) __builtin_amdgcn_s_waitcnt(0);  // this tile's rows are in LDS
        __syncthreads();  // previous tile's readers of xin / meta / hpart are done
        tid = opaque_tid();
        lane = tid & 63, half = lane >> 5, col = lane & 31;
        tile_input<C, P, M, SRC, SK>(args, row0, tid, xin, meta_ok, meta_kid, vst);
        // the first layer's weights, requested before the barrier (not across
        // the input stage, whose registers are at their peak)
        if constexpr (XPF)
            ring_load<P0, 32, C::NBP>(reinterpret_cast<const R0 *>(args.net.w[0]), nb0, lane, ring0);
        __syncthreads();

        // one pass of the network per model of a group (one for other sinks),
        // all on the input tile built above
        const int n_models = group_size(kargs);
        for (int t = 0; t < n_models; ++t) {
            const NetView &net = group_net(kargs, t);
            const R0 *w0 = reinterpret_cast<const R0 *>(net.w[0]);
            const bool last_model = t + 1 == n_models;
            if (t > 0) {
                __syncthreads();  // the previous model's readers of act and hpart are done
                if constexpr (XPF) ring_load<P0, 32, C::NBP>(w0, nb0, lane, ring0);
            }

            // ---- layer 0 (32 inputs), then hidden layers 1..n_hidden-1. Each wave
            // covers its n-blocks in NSPLIT passes (smaller accumulators): the
            // outputs of all passes but the last wait packed in registers; the
            // last pass's accumulators cross the barrier after which every wave
            // has read the layer's input, and all outputs then go to LDS in its
            // place.
            for (int l = 0; l < net.n_hidden; ++l) {
                tid = opaque_tid();
                lane = tid & 63, half = lane >> 5, col = lane & 31;
                const bool last = l + 1 == net.n_hidden;
                const float *bias = net.b[l];
                // fp8 layers scale the products before the bias; every other layer
                // starts its accumulators at the bias
                const bool scaled = P == PREC_FP8 && l > 0;
                const float qs = scaled ? net.qscale[l] : 1.0f;
                const float qinv = net.qinv[l];
                typename Held<P>::T held[C::NSPLIT > 1 ? C::NSPLIT - 1 : 1][C::NBP][4][C::MBW];
                float srow[C::MBW];
#pragma unroll
                for (int j = 0; j < C::MBW; ++j) srow[j] = 0.0f;
#pragma unroll
                for (int ps = 0; ps < C::NSPLIT; ++ps) {
                    const int nbp0 = nb0 + ps * C::NBP;
                    const bool final_pass = ps + 1 == C::NSPLIT;
                    v16f acc[C::NBP][C::MBW];
                    const RH *wl = reinterpret_cast<const RH *>(net.w[l]);
                    if constexpr (!XPF) {
                        if (l == 0)
                            ring_load<P0, 32, C::NBP>(w0, nbp0, lane, ring0);
                        else
                            ring_load<P, W, C::NBP>(wl, nbp0, lane, ringh);
                    }
                    if (l == 0)
                        layer_mma<P0, 32, C::NBP, C::MBW>(w0, xin, C::XS, nbp0, mb0, lane, acc, bias,
                                                          ring0);
                    else
                        layer_mma<P, W, C::NBP, C::MBW>(wl, act, C::AS, nbp0, mb0, lane, acc,
                                                        scaled ? nullptr : bias, ringh);
                    // request the next call's first weight groups before the epilogue
                    if (!XPF) {
                    } else if (!final_pass) {
                        if (l == 0)
                            ring_load<P0, 32, C::NBP>(w0, nbp0 + C::NBP, lane, ring0);
                        else
                            ring_load<P, W, C::NBP>(wl, nbp0 + C::NBP, lane, ringh);
                    } else if (!last) {
                        ring_load<P, W, C::NBP>(reinterpret_cast<const RH *>(net.w[l + 1]), nb0, lane,
                                                ringh);
                    }
                    if constexpr (VPF) {
                        if (final_pass && last && last_model && tile + gridDim.x < ntiles)
                            issue_vdesc(tile + gridDim.x);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    // training keeps the last hidden layer's outputs too (copied out below)
                    constexpr bool keep_last = SINK == SINK_TRAIN;
                    if (final_pass && (!last || keep_last)) {
                        if (l > 0) __syncthreads();  // every wave finished reading this layer's input
#pragma unroll
                        for (int hp = 0; hp + 1 < C::NSPLIT; ++hp)
#pragma unroll
                            for (int i = 0; i < C::NBP; ++i)
#pragma unroll
                                for (int j = 0; j < C::MBW; ++j)
#pragma unroll
                                    for (int g = 0; g < 4; ++g) {
                                        const int nn = (nb0 + hp * C::NBP + i) * 32 + 8 * g + 4 * half;
                                        const int m = (mb0 + j) * 32 + col;
                                        store_held<P>(act + (size_t)m * C::AS, nn, held[hp][i][g][j]);
                                    }
                    }
                    // one 32-neuron block at a time: its bias (and output-layer
                    // weight) vectors are loaded together, and the fence keeps the
                    // next block's loads from being hoisted
#pragma unroll
                    for (int i = 0; i < C::NBP; ++i) {
                        v4f bias_r[4], hw_r[4];
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int nn = (nbp0 + i) * 32 + 8 * g + 4 * half;
                            if (scaled)
                                bias_r[g] = BL ? *reinterpret_cast<const v4f *>(bias_lds + l * W + nn)
                                               : *reinterpret_cast<const v4f *>(bias + nn);
                            if (last)
                                hw_r[g] = (VPF || BL) ? *reinterpret_cast<const v4f *>(hw_lds + nn)
                                                      : *reinterpret_cast<const v4f *>(net.head_w + nn);
                        }
#pragma unroll
                        for (int j = 0; j < C::MBW; ++j) {
                            const int m = (mb0 + j) * 32 + col;
                            uint32_t mbits = 0;  // training: ReLU mask of this lane's 16 neurons
#pragma unroll
                            for (int g = 0; g < 4; ++g) {
                                const int nn = (nbp0 + i) * 32 + 8 * g + 4 * half;
                                v4f v;
                                if constexpr (P == PREC_FP8) {
                                    if (!last) {
                                        // the next fp8 layer's input in one step; the
                                        // staged biases are already divided by its scale
                                        v4f a, bq;
#pragma unroll
                                        for (int e = 0; e < 4; ++e) {
                                            a[e] = acc[i][j][4 * g + e];
                                            bq[e] = BL ? bias_r[g][e] : bias_r[g][e] * qinv;
                                        }
                                        const uint32_t q = quant4_fp8(a, scaled, scaled ? qs * qinv : qinv, bq);
                                        const typename Held<P>::T hq = *reinterpret_cast<const typename Held<P>::T *>(&q);
                                        if (final_pass)
                                            store_held<P>(act + (size_t)m * C::AS, nn, hq);
                                        else
                                            held[final_pass ? 0 : ps][i][g][j] = hq;
                                        continue;
                                    }
                                }
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const float z = scaled ? acc[i][j][4 * g + e] * qs + bias_r[g][e]
                                                           : acc[i][j][4 * g + e];
                                    v[e] = z > 0.0f ? z : 0.0f;
                                }
                                if constexpr (SINK == SINK_TRAIN) {
                                    // from the value as stored (non-negative: any
                                    // non-zero bit pattern is positive)
                                    // the stored values are >= 0 (never -0): positive
                                    // exactly when their bit pattern is non-zero, and
                                    // min(bits, 1) is that bit
                                    const typename Held<P>::T hv = pack4<P>(v, qinv);
                                    uint32_t nib;
                                    if constexpr (P == PREC_FP32) {
                                        nib = 0;
#pragma unroll
                                        for (int e = 0; e < 4; ++e)
                                            nib |= min(__float_as_uint(hv[e]), 1u) << e;
                                    } else {
                                        // the four bf16 values as two words, low half first
                                        typedef unsigned v2u_ __attribute__((ext_vector_type(2)));
                                        const v2u_ u = __builtin_bit_cast(v2u_, hv);
                                        nib = min(u[0] & 0xffffu, 1u) | (min(u[0] >> 16, 1u) << 1) |
                                              (min(u[1] & 0xffffu, 1u) << 2) | (min(u[1] >> 16, 1u) << 3);
                                    }
                                    mbits |= nib << (8 * g + 4 * half);
                                }
                                if (last) {
                                    // output layer: fixed order over blocks, groups, elements
#pragma unroll
                                    for (int e = 0; e < 4; ++e) srow[j] += v[e] * hw_r[g][e];
                                }
                                if (!last || keep_last) {
                                    if (final_pass)
                                        store4<P>(act + (size_t)m * C::AS, nn, v, qinv);
                                    else
                                        held[final_pass ? 0 : ps][i][g][j] = pack4<P>(v, qinv);
                                }
                            }
                            if constexpr (SINK == SINK_TRAIN) {
                                // the two lane halves hold the block's other 16 neurons
                                const uint32_t word = mbits | (uint32_t)__shfl_xor((int)mbits, 32, 64);
                                if (!last && args.save_mask != nullptr && half == 0)
                                    args.save_mask[((int64_t)l * (W / 32) + nbp0 + i) * args.save_ld +
                                                   row0 + m] = word;
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                if (!last || SINK == SINK_TRAIN) {
                    __syncthreads();  // next layer (or the copy below) reads the complete activations
                    if constexpr (SINK == SINK_TRAIN)
                        copy_act_transposed<P, W, M, C::THREADS, C::AS>(
                            act,
                            reinterpret_cast<unsigned char *>(args.save_h) +
                                (size_t)l * W * args.save_ld * Geo<P>::EB,
                            args.save_ld, row0, n, tid);
                }
                if (last) {
#pragma unroll
                    for (int j = 0; j < C::MBW; ++j) {
                        float sj = srow[j];
                        sj += __shfl_xor(sj, 32, 64);  // the two lane halves hold different neurons
                        if (half == 0) hpart[wn * M + (mb0 + j) * 32 + col] = sj;
                    }
                }
            }
            __syncthreads();
            tid = opaque_tid();
            lane = tid & 63;
            tile_output<C, M, SK>(args, row0, tid, lane, wave, hpart, meta_ok, meta_kid, net.head_b,
                                  group_pred(kargs, t), group_keys(kargs, t));
        }
    }
}

// Ping-pong schedule of the same pipeline: each wave's rows are split into
// two halves A and B, and every phase runs the matrix loop of one half while
// the epilogue (bias already in the accumulators, ReLU, down-cast, LDS store
// or output-layer dot) of the other half runs beside it:
//   k(0,A) | k(0,B) e(0,A) || k(1,A) e(0,B) || k(1,B) e(1,A) || ... e(L-1,B)
// ("||" a barrier). An epilogue writes rows whose input the other phase's
// matrix loop is not reading, so one barrier per phase suffices, and the two
// waves sharing a SIMD take the two halves of a phase in opposite order, so
// one's epilogue runs while the other's multiplies occupy the matrix core.
// The weights are streamed once per half. Results are bit-identical to
// mlp_tiles_kernel with the same wave count (same per-element arithmetic and
// summation order).
template <int P, int W, int M, int NWAVES, int SRC, int SINK>
__global__ __launch_bounds__(NWAVES * 64)
__attribute__((amdgpu_waves_per_eu(tile_waves_per_simd<P, W, M, NWAVES>()))) void
mlp_pp_kernel(TileArgs args)
{
    static_assert(SINK != SINK_TRAIN, "the training forward uses mlp_tiles_kernel");
    constexpr bool VPF = SRC == SRC_DESC && tile_vdesc_prefetch<P, W, M, NWAVES>();
    using C = TileCfg<P, W, M, NWAVES, 1, VPF>;
    using G = typename C::G;
    static_assert(C::MBW % 2 == 0, "each wave's rows split into two halves");
    constexpr int MH = C::MBW / 2;
    constexpr int NBW = C::NBW;
    constexpr int P0 = FirstP<P>::value;
    using G0 = Geo<P0>;
    using R0 = typename G0::Vec;
    using RH = typename G::Vec;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *xin = lds;                                   // [M][XS]
    unsigned char *act = xin + (size_t)M * C::XS;               // [M][AS]
    float *hpart = reinterpret_cast<float *>(act + C::ACT_BYTES);       // [WN][M]
    int *meta_ok = reinterpret_cast<int *>(hpart + C::WN * M);  // [M]
    int *meta_kid = meta_ok + M;                                // [M]
    unsigned char *vst = lds + C::LDS_BASE;                     // [M][64 B] (VPF)
    float *hw_lds = reinterpret_cast<float *>(vst + C::VST_BYTES);  // [W] (VPF)

    const int tid0 = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid0 >> 6);
    const int wn = wave % C::WN, wm = wave / C::WN;
    const int nb0 = wn * NBW, mb0 = wm * C::MBW;
    // re-derived per tile from an opaque copy (see mlp_tiles_kernel)
    auto opaque_tid = [&]() {
        int t = tid0;
        asm volatile("" : "+v"(t));
        return t;
    };
    int tid = tid0, lane = tid0 & 63, half = lane >> 5, col = lane & 31;
    const NetView &net = args.net;
    const int64_t n = args.n_rows;
    const int64_t ntiles = (n + M - 1) / M;
    // waves w and w + 4 share a SIMD: they take each phase's halves in
    // opposite order
    const bool mma_first = ((wave >> 2) & 1) == 0;
    const R0 *w0 = reinterpret_cast<const R0 *>(net.w[0]);

    auto issue_vdesc = [&](int64_t t) {
        const int64_t r0 = t * M;
        for (int c0 = wave * 64; c0 < M * 4; c0 += C::THREADS) {
            const int c = c0 + lane;
            if (r0 + c / 4 < n)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(args.vdesc + r0 * VD + 2 * c),
                    (__attribute__((address_space(3))) void *)(vst + (size_t)c0 * 16), 16, 0, 0);
        }
    };
    if constexpr (VPF) {
        for (int i = tid; i < W; i += C::THREADS) hw_lds[i] = net.head_w[i];
        if ((int64_t)blockIdx.x < ntiles) issue_vdesc(blockIdx.x);
    }

    // matrix loop of layer l over m-blocks mb .. mb + MH - 1
    auto mma_half = [&](int l, int mb, v16f (&acc)[NBW][MH]) {
        if (l == 0) {
            R0 ring[ring_depth<P0, 32>()][NBW];
            ring_load<P0, 32, NBW>(w0, nb0, lane, ring);
            layer_mma<P0, 32, NBW, MH>(w0, xin, C::XS, nb0, mb, lane, acc, net.b[0], ring);
        } else {
            const RH *wl = reinterpret_cast<const RH *>(net.w[l]);
            RH ring[ring_depth<P, W>()][NBW];
            ring_load<P, W, NBW>(wl, nb0, lane, ring);
            const bool scaled = P == PREC_FP8;
            layer_mma<P, W, NBW, MH>(wl, act, C::AS, nb0, mb, lane, acc,
                                     scaled ? nullptr : net.b[l], ring);
        }
    };
    // epilogue of layer l over m-blocks mb .. mb + MH - 1: next activations
    // to LDS, or for the last layer the output-layer partial dot into srow
    auto epi_half = [&](int l, int mb, v16f (&acc)[NBW][MH], float (&srow)[MH]) {
        const bool last = l + 1 == net.n_hidden;
        const bool scaled = P == PREC_FP8 && l > 0;
        const float qs = scaled ? net.qscale[l] : 1.0f;
        const float qinv = net.qinv[l];
        const float *bias = net.b[l];
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            v4f bias_r[4], hw_r[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int nn = (nb0 + i) * 32 + 8 * g + 4 * half;
                if (scaled) bias_r[g] = *reinterpret_cast<const v4f *>(bias + nn);
                if (last)
                    hw_r[g] = VPF ? *reinterpret_cast<const v4f *>(hw_lds + nn)
                                  : *reinterpret_cast<const v4f *>(net.head_w + nn);
            }
#pragma unroll
            for (int j = 0; j < MH; ++j) {
                const int m = (mb + j) * 32 + col;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int nn = (nb0 + i) * 32 + 8 * g + 4 * half;
                    v4f v;
                    if constexpr (P == PREC_FP8) {
                        if (!last) {  // as in mlp_tiles_kernel: the same bits
                            v4f a, bq;
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                a[e] = acc[i][j][4 * g + e];
                                bq[e] = bias_r[g][e] * qinv;
                            }
                            const uint32_t q = quant4_fp8(a, scaled, scaled ? qs * qinv : qinv, bq);
                            store_held<P>(act + (size_t)m * C::AS, nn, q);
                            continue;
                        }
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float z = scaled ? acc[i][j][4 * g + e] * qs + bias_r[g][e]
                                               : acc[i][j][4 * g + e];
                        v[e] = z > 0.0f ? z : 0.0f;
                    }
                    if (last) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) srow[j] += v[e] * hw_r[g][e];
                    } else {
                        store4<P>(act + (size_t)m * C::AS, nn, v, qinv);
                    }
                }
            }
        }
    };

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row0 = tile * M;
        if constexpr (VPF) __builtin_amdgcn_s_waitcnt(0);  // this tile's rows are in LDS
        __syncthreads();  // previous tile's readers of xin / meta / hpart are done
        tid = opaque_tid();
        lane = tid & 63, half = lane >> 5, col = lane & 31;
        tile_input<C, P, M, SRC, SINK>(args, row0, tid, xin, meta_ok, meta_kid, vst);
        __syncthreads();

        const int mbA = mb0, mbB = mb0 + MH;
        v16f accA[NBW][MH], accB[NBW][MH];
        float srowA[MH], srowB[MH];
#pragma unroll
        for (int j = 0; j < MH; ++j) {
            srowA[j] = 0.0f;
            srowB[j] = 0.0f;
        }
        const int L = net.n_hidden;
        mma_half(0, mbA, accA);
        for (int l = 0; l < L; ++l) {
            const bool last = l + 1 == L;
            // k(l,B) beside e(l,A); e(l,A) overwrites rows A, whose input
            // k(l,A) finished reading before the last barrier
            if (mma_first) {
                mma_half(l, mbB, accB);
                epi_half(l, mbA, accA, srowA);
            } else {
                epi_half(l, mbA, accA, srowA);
                mma_half(l, mbB, accB);
            }
            if constexpr (VPF) {
                if (last && tile + gridDim.x < ntiles) issue_vdesc(tile + gridDim.x);
            }
            if (last) break;
            __syncthreads();  // rows A of layer l are complete
            // k(l+1,A) beside e(l,B)
            if (mma_first) {
                mma_half(l + 1, mbA, accA);
                epi_half(l, mbB, accB, srowB);
            } else {
                epi_half(l, mbB, accB, srowB);
                mma_half(l + 1, mbA, accA);
            }
            __syncthreads();  // rows B of layer l are complete; k(l+1,A) is done with rows A
        }
        epi_half(L - 1, mbB, accB, srowB);
#pragma unroll
        for (int j = 0; j < MH; ++j) {
            float sa = srowA[j], sb = srowB[j];
            sa += __shfl_xor(sa, 32, 64);  // the two lane halves hold different neurons
            sb += __shfl_xor(sb, 32, 64);
            if (half == 0) {
                hpart[wn * M + (mbA + j) * 32 + col] = sa;
                hpart[wn * M + (mbB + j) * 32 + col] = sb;
            }
        }
        __syncthreads();
        tid = opaque_tid();
        lane = tid & 63;
        tile_output<C, M, SINK>(args, row0, tid, lane, wave, hpart, meta_ok, meta_kid, net.head_b,
                                args.pred, args.keys);
    }
}

}  // namespace adv
