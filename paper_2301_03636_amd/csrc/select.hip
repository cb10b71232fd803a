// Integer and selection kernels: standalone feature extraction, the Z-score
// fit, and the per-kernel argmin on given predictions. All of them are
// bandwidth-bound and use no matrix cores.
#include <algorithm>

#include <cstdlib>
#include <string>

#include "features.h"
#include "wave_select.h"

namespace adv {

// ---------------------------------------------------------------------------
// Feature extraction: one thread per variant. A workgroup stages its 256
// feature rows (64 KiB) in LDS so the int64 stores leave as contiguous
// 16-byte chunks per lane (fully coalesced) instead of 256-byte strided rows.
constexpr int FZ_THREADS = 256;

__global__ __launch_bounds__(FZ_THREADS) void featurize_kernel(
    const int64_t *__restrict__ kdesc, const int64_t *__restrict__ vdesc, int64_t n_k,
    int64_t n_v, int64_t *__restrict__ feat, uint8_t *__restrict__ invalid)
{
    __shared__ int64_t stage[FZ_THREADS * NFEAT];
    const int64_t row0 = (int64_t)blockIdx.x * FZ_THREADS;
    const int t = threadIdx.x;
    const int64_t row = row0 + t;
    if (row < n_v) {
        Feat f;
        bool ok = featurize_one(kdesc, vdesc + row * VD, n_k, f);
        if (invalid) invalid[row] = ok ? 0 : 1;
        // rotate the column by the row so neighbouring threads hit distinct banks
#pragma unroll
        for (int j = 0; j < NFEAT; ++j) stage[t * NFEAT + ((j + t) & (NFEAT - 1))] = (int64_t)f.f[j];
    }
    __syncthreads();
    const int64_t rows = min((int64_t)FZ_THREADS, n_v - row0);
    // 2 int64 per lane per store: chunk c covers row c/16, columns 2*(c%16)..+1
    longlong2 *out = reinterpret_cast<longlong2 *>(feat + row0 * NFEAT);
    const int chunks = (int)rows * (NFEAT / 2);
    for (int c = t; c < chunks; c += FZ_THREADS) {
        const int r = c >> 4, j = (c & 15) * 2;
        longlong2 v;
        v.x = stage[r * NFEAT + ((j + r) & (NFEAT - 1))];
        v.y = stage[r * NFEAT + ((j + 1 + r) & (NFEAT - 1))];
        out[c] = v;
    }
}

// ---------------------------------------------------------------------------
// Z-score fit in float64 with a fixed reduction order (deterministic): each
// workgroup owns a contiguous block of rows; 8 row-lanes x 32 features per
// workgroup; per-workgroup partials are combined in workgroup order.
constexpr int ZS_THREADS = 256;
constexpr int ZS_ROWLANES = ZS_THREADS / NFEAT;

__global__ __launch_bounds__(ZS_THREADS) void zscore_partial_kernel(
    const int64_t *__restrict__ feat, int64_t n, int64_t rows_per_block,
    const double *__restrict__ mean, double *__restrict__ part_sum,
    int64_t *__restrict__ part_min, int64_t *__restrict__ part_max)
{
    __shared__ double s_sum[ZS_THREADS];
    __shared__ int64_t s_min[ZS_THREADS], s_max[ZS_THREADS];
    const int j = threadIdx.x & (NFEAT - 1), lane_row = threadIdx.x / NFEAT;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    double s = 0.0;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t r = r0 + lane_row; r < r1; r += ZS_ROWLANES) {
        const int64_t f = feat[r * NFEAT + j];
        const double l = log2((double)f + 1.0);
        if (mean) {
            const double d = l - mean[j];
            s += d * d;
        } else {
            s += l;
        }
        lo = f < lo ? f : lo;
        hi = f > hi ? f : hi;
    }
    s_sum[threadIdx.x] = s;
    s_min[threadIdx.x] = lo;
    s_max[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x < NFEAT) {
        double a = 0.0;
        int64_t mn = INT64_MAX, mx = INT64_MIN;
        for (int q = 0; q < ZS_ROWLANES; ++q) {
            a += s_sum[q * NFEAT + j];
            mn = min(mn, s_min[q * NFEAT + j]);
            mx = max(mx, s_max[q * NFEAT + j]);
        }
        part_sum[blockIdx.x * NFEAT + j] = a;
        if (part_min) {
            part_min[blockIdx.x * NFEAT + j] = mn;
            part_max[blockIdx.x * NFEAT + j] = mx;
        }
    }
}

// One thread per feature: combine the partials in order. Pass 1 writes the
// mean (or the constant's logarithm), pass 2 the population deviation.
__global__ void zscore_final_kernel(const double *__restrict__ part_sum,
                                    const int64_t *__restrict__ part_min,
                                    const int64_t *__restrict__ part_max, int n_blocks, int64_t n,
                                    int pass, double *__restrict__ mu, double *__restrict__ sigma,
                                    int *__restrict__ constant)
{
    const int j = threadIdx.x;
    if (j >= NFEAT) return;
    double a = 0.0;
    for (int b = 0; b < n_blocks; ++b) a += part_sum[b * NFEAT + j];
    if (pass == 1) {
        int64_t mn = INT64_MAX, mx = INT64_MIN;
        for (int b = 0; b < n_blocks; ++b) {
            mn = min(mn, part_min[b * NFEAT + j]);
            mx = max(mx, part_max[b * NFEAT + j]);
        }
        constant[j] = (mn == mx);
        mu[j] = (mn == mx) ? log2((double)mn + 1.0) : a / (double)n;
    } else {
        const double sd = sqrt(a / (double)n);
        sigma[j] = (constant[j] || !(sd > 0.0)) ? 1.0 : sd;
    }
}

// ---------------------------------------------------------------------------
// Segmented argmin on predictions: one wave per kernel segment, keys and
// wave-wide exchanges from wave_select.h.

// Loads in flight per lane in the selection kernels' scans: a segment of up
// to 64 * SEL_UNROLL = 1024 variants is read in one round trip (the loads of
// a pass are all issued before the first compare), so a wave's time is one
// latency of its offsets and one of its predictions rather than a chain.
constexpr int SEL_UNROLL = 16;

constexpr int AM_WAVES = 4;

// The predictions pred[base + 64 u] (u < SEL_UNROLL) of one pass, NaN past hi.
__device__ __forceinline__ void load_pass(const float *__restrict__ pred, int64_t base, int64_t hi,
                                          float (&p)[SEL_UNROLL])
{
#pragma unroll
    for (int u = 0; u < SEL_UNROLL; ++u) {
        const int64_t i = base + 64 * u;
        p[u] = i < hi ? pred[i] : __builtin_nanf("");
    }
    // keep every load of the pass ahead of the compares that use them
    __builtin_amdgcn_sched_barrier(0);
}

__global__ __launch_bounds__(AM_WAVES * 64) void argmin_preds_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets, int64_t n_k,
    int64_t n_v, int64_t *__restrict__ best)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves_total = (int64_t)gridDim.x * AM_WAVES;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t k = (int64_t)blockIdx.x * AM_WAVES + wave; k < n_k; k += nwaves_total) {
        // clamp to the prediction array so malformed offsets cannot read out of bounds
        const int64_t lo = max((int64_t)0, min(offsets[k], n_v));
        const int64_t hi = max(lo, min(offsets[k + 1], n_v));
        uint64_t key = ~0ull;
        for (int64_t base = lo + lane; base < hi; base += 64 * SEL_UNROLL) {
            float p[SEL_UNROLL];
            load_pass(pred, base, hi, p);
#pragma unroll
            for (int u = 0; u < SEL_UNROLL; ++u) {
                if (!__builtin_isnan(p[u])) {
                    const uint64_t q = pred_key(p[u], (uint32_t)(base + 64 * u));
                    key = q < key ? q : key;
                }
            }
        }
        key = wave_min_u64(key);
        if (lane == 0) best[k] = key == ~0ull ? -1 : (int64_t)(key & 0xffffffffull);
    }
}


// A lane's sorted list of the K smallest keys it has seen (compile-time
// indices only): a key enters only if it beats the current K-th.
template <int K>
__device__ __forceinline__ void list_insert(uint64_t (&top)[K], uint64_t x)
{
    if (x >= top[K - 1]) return;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const uint64_t t = top[q];
        const bool less = x < t;
        top[q] = less ? x : t;
        x = less ? t : x;
    }
}

// N rounds of a wave-wide minimum over the lists' heads pop the wave's N
// smallest keys in ascending order (keys are unique, so exactly one lane
// pops each); lane r gets the r-th, ~0 past the last key. N <= K, the same
// in every lane; every lane must be active.
template <int K>
__device__ __forceinline__ uint64_t list_pop(uint64_t (&top)[K], int N, int lane)
{
    uint64_t mine = ~0ull;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        if (r >= N) break;
        const uint64_t v = wave_min_u64(top[0]);
        if (v == ~0ull) break;  // fewer than N keys
        if (lane == r) mine = v;
        if (top[0] == v) {
#pragma unroll
            for (int q = 0; q + 1 < K; ++q) top[q] = top[q + 1];
            top[K - 1] = ~0ull;
        }
    }
    return mine;
}

// The last k in [0, n_k) with offsets[k] <= c0 (offsets non-decreasing,
// offsets[0] = 0 <= c0): rounds of 64 offsets sampled across the remaining
// range, one load and a ballot each. Uniform over the wave; every lane must
// be active. With offsets that break the contract the result is some k in
// range.
__device__ __forceinline__ int64_t segment_of(const int64_t *__restrict__ offsets, int64_t n_k,
                                              int64_t c0, int lane)
{
    int64_t a = 0, b = n_k - 1;
    while (b > a) {
        const int64_t span = b - a + 1;
        const int64_t kj = span <= 64 ? a + lane : a + (int64_t)lane * span / 64;
        const bool ok = kj <= b && offsets[kj] <= c0;
        const uint64_t m = __ballot(ok);
        if (m == 0) break;  // only for offsets[a] > c0: not a valid offsets array
        const int j = 63 - __builtin_clzll(m);
        const int64_t ka = span <= 64 ? a + j : a + (int64_t)j * span / 64;
        if (span <= 64) {
            a = ka;
            break;
        }
        const int64_t kb = j == 63 ? b : a + (int64_t)(j + 1) * span / 64 - 1;
        a = ka;
        b = max(ka, kb);
    }
    return a;
}

// Long segments (on average AM_LONG variants or more per kernel, where one
// wave per segment leaves most of the chip idle): the variants are cut into
// chunks of AM_CHUNK, one wave each. A wave finds the segment holding its
// chunk's first variant (segment_of), walks the segments its chunk overlaps, and folds each one's minimum key
// into keys[k] with a 64-bit atomic minimum (keys start at ~0; the key holds
// the index, so the result does not depend on the order of the atomics).
// Every index is clamped, so offsets that break the contract (not
// non-decreasing) give wrong picks but no access out of bounds.
constexpr int64_t AM_CHUNK = 4096;
constexpr int64_t AM_LONG = 16384;

__global__ __launch_bounds__(AM_WAVES * 64) void argmin_chunks_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets, int64_t n_k,
    int64_t n_v, unsigned long long *__restrict__ keys)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t c0 = ((int64_t)blockIdx.x * AM_WAVES + wave) * AM_CHUNK;
    if (c0 >= n_v) return;
    const int64_t c1 = min(c0 + AM_CHUNK, n_v);
    const int64_t a = segment_of(offsets, n_k, c0, lane);
    int64_t pos = c0;
    for (int64_t k = a; k < n_k && pos < c1; ++k) {
        const int64_t hi = min(max(offsets[k + 1], pos), c1);
        uint64_t key = ~0ull;
        for (int64_t base = pos + lane; base < hi; base += 64 * SEL_UNROLL) {
            float p[SEL_UNROLL];
            load_pass(pred, base, hi, p);
#pragma unroll
            for (int u = 0; u < SEL_UNROLL; ++u) {
                if (!__builtin_isnan(p[u])) {
                    const uint64_t q = pred_key(p[u], (uint32_t)(base + 64 * u));
                    key = q < key ? q : key;
                }
            }
        }
        key = wave_min_u64(key);
        if (lane == 0 && key != ~0ull) atomicMin(keys + k, (unsigned long long)key);
        pos = hi;
    }
}

__global__ void argmin_keys_init_kernel(unsigned long long *keys, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = ~0ull;
}

// key -> variant index (its low 32 bits), -1 where no variant was eligible
__global__ void argmin_keys_final_kernel(int64_t *best, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint64_t k = (uint64_t)best[i];
        best[i] = k == ~0ull ? -1 : (int64_t)(k & 0xffffffffull);
    }
}

// The top-N list of the prediction flow (section 3: the predicted runtimes
// are sorted and the N best variants kept). One wave per kernel segment, in a
// grid-stride loop over kernels. Lane r writes rank r: the variant index and
// its prediction, or -1 and NaN past the end of the eligible variants.
//
// Lists of 8 or more (K >= 8) take two launches. The first (TOPN_FAST)
// holds only the threshold path, in few registers, and marks each segment it
// leaves undone with -2 in the first slot of its list; the second
// (TOPN_MARKED) runs the per-lane lists on the marked segments. Shorter lists
// take one launch (TOPN_ALL) of the per-lane lists.
//
// A segment of at most 64 * SEL_UNROLL variants (one load pass) takes the
// threshold path (threshold_select: a bound on the N-th smallest key from
// one wave sort, then at most 64 candidates gathered and sorted). Every
// other segment (longer ones, more than 64 candidates): each lane keeps the
// K smallest keys it has seen (a sorted list held in registers, compile-time
// indices only, entered only by keys that beat its current K-th), then N
// rounds of a wave-wide minimum pop the segment's best keys in ascending
// order (keys are unique, so exactly one lane pops each).
enum { TOPN_ALL = 0, TOPN_FAST = 1, TOPN_MARKED = 2 };

template <int K, int MODE>
__global__ __launch_bounds__(AM_WAVES * 64) void topn_preds_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets, int64_t n_k,
    int64_t n_v, int N, int64_t *__restrict__ idx_out, float *__restrict__ val_out)
{
    __shared__ uint64_t cand_lds[AM_WAVES][64];
    const int lane = threadIdx.x & 63;
    const int64_t nwaves_total = (int64_t)gridDim.x * AM_WAVES;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t k = (int64_t)blockIdx.x * AM_WAVES + wave; k < n_k; k += nwaves_total) {
        if constexpr (MODE == TOPN_MARKED) {
            if (idx_out[k * N] != -2) continue;  // done by the threshold path
        }
        const int64_t lo = max((int64_t)0, min(offsets[k], n_v));
        const int64_t hi = max(lo, min(offsets[k + 1], n_v));
        if constexpr (MODE == TOPN_FAST) {
            if (hi - lo <= 64 * SEL_UNROLL) {  // the same for every lane
                float p[SEL_UNROLL];
                load_pass(pred, lo + lane, hi, p);
                uint64_t x[SEL_UNROLL];
#pragma unroll
                for (int u = 0; u < SEL_UNROLL; ++u)
                    x[u] = __builtin_isnan(p[u]) ? ~0ull
                                                 : pred_key(p[u], (uint32_t)(lo + lane + 64 * u));
                uint64_t v;
                if (threshold_select(x, N, lane, cand_lds[wave], v)) {
                    if (lane < N) {
                        const int64_t s_ = k * N + lane;
                        const bool some = v != ~0ull;
                        const int64_t mine = some ? (int64_t)(v & 0xffffffffull) : -1;
                        idx_out[s_] = mine;
                        if (val_out) {
                            // a zero key may stand for -0: read the stored value
                            float pv = some ? key_pred(v) : __builtin_nanf("");
                            if (some && pv == 0.0f) pv = pred[mine];
                            val_out[s_] = pv;
                        }
                    }
                    continue;
                }
            }
            if (lane == 0) idx_out[k * N] = -2;  // left to the per-lane lists
            continue;
        }
        uint64_t top[K];
#pragma unroll
        for (int q = 0; q < K; ++q) top[q] = ~0ull;
        for (int64_t base = lo + lane; base < hi; base += 64 * SEL_UNROLL) {
            float p[SEL_UNROLL];
            load_pass(pred, base, hi, p);
#pragma unroll
            for (int u = 0; u < SEL_UNROLL; ++u)
                if (!__builtin_isnan(p[u])) list_insert(top, pred_key(p[u], (uint32_t)(base + 64 * u)));
        }
        const uint64_t v = list_pop(top, N, lane);
        const int64_t mine = v == ~0ull ? -1 : (int64_t)(v & 0xffffffffull);
        if (lane < N) {
            const int64_t slot = k * N + lane;
            idx_out[slot] = mine;
            if (val_out) val_out[slot] = mine >= 0 ? pred[mine] : __builtin_nanf("");
        }
    }
}

// Top-N on long segments (AM_LONG variants or more per kernel on average):
// chunks of AM_CHUNK variants, one wave each, find their first segment as
// the chunked argmin does; for every segment k a chunk c overlaps, the
// overlap's N best keys (per-lane lists, then N pops) go to list c + k of a
// scratch array of (chunks + n_k) lists of N keys (a later segment only
// overlaps later chunks, so the lists of different overlaps never share a
// slot, and segment k's chunks own the consecutive lists c_first + k ..
// c_last + k). A second launch, one wave per segment, takes the N best keys
// of its lists the same way and writes the segment's top-N list.
template <int K>
__global__ __launch_bounds__(AM_WAVES * 64) void topn_chunks_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets, int64_t n_k,
    int64_t n_v, int N, uint64_t *__restrict__ lists)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t c = (int64_t)blockIdx.x * AM_WAVES + wave;
    const int64_t c0 = c * AM_CHUNK;
    if (c0 >= n_v) return;
    const int64_t c1 = min(c0 + AM_CHUNK, n_v);
    int64_t pos = c0;
    for (int64_t k = segment_of(offsets, n_k, c0, lane); k < n_k && pos < c1; ++k) {
        const int64_t hi = min(max(offsets[k + 1], pos), c1);
        if (hi == pos) continue;
        uint64_t top[K];
#pragma unroll
        for (int q = 0; q < K; ++q) top[q] = ~0ull;
        for (int64_t base = pos + lane; base < hi; base += 64 * SEL_UNROLL) {
            float p[SEL_UNROLL];
            load_pass(pred, base, hi, p);
#pragma unroll
            for (int u = 0; u < SEL_UNROLL; ++u)
                if (!__builtin_isnan(p[u])) list_insert(top, pred_key(p[u], (uint32_t)(base + 64 * u)));
        }
        const uint64_t v = list_pop(top, N, lane);
        if (lane < N) lists[(c + k) * N + lane] = v;
        pos = hi;
    }
}

template <int K>
__global__ __launch_bounds__(AM_WAVES * 64) void topn_merge_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets, int64_t n_k,
    int64_t n_v, int N, const uint64_t *__restrict__ lists, int64_t *__restrict__ idx_out,
    float *__restrict__ val_out)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves_total = (int64_t)gridDim.x * AM_WAVES;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t k = (int64_t)blockIdx.x * AM_WAVES + wave; k < n_k; k += nwaves_total) {
        const int64_t lo = max((int64_t)0, min(offsets[k], n_v));
        const int64_t hi = max(lo, min(offsets[k + 1], n_v));
        uint64_t top[K];
#pragma unroll
        for (int q = 0; q < K; ++q) top[q] = ~0ull;
        if (hi > lo) {
            const int64_t first = (lo / AM_CHUNK + k) * N, last = ((hi - 1) / AM_CHUNK + k + 1) * N;
            for (int64_t i = first + lane; i < last; i += 64) list_insert(top, lists[i]);
        }
        const uint64_t v = list_pop(top, N, lane);
        const int64_t mine = v == ~0ull ? -1 : (int64_t)(v & 0xffffffffull);
        if (lane < N) {
            const int64_t slot = k * N + lane;
            idx_out[slot] = mine;
            if (val_out) val_out[slot] = mine >= 0 ? pred[mine] : __builtin_nanf("");
        }
    }
}

template <int K>
static void launch_topn(const float *pred, const int64_t *offsets, int64_t n_k, int64_t n_v,
                        int N, int64_t *idx_out, float *val_out, uint64_t *lists, hipStream_t s)
{
    if (lists) {
        const int64_t chunks = (n_v + AM_CHUNK - 1) / AM_CHUNK;
        hipLaunchKernelGGL((topn_chunks_kernel<K>), dim3((unsigned)((chunks + AM_WAVES - 1) / AM_WAVES)),
                           dim3(AM_WAVES * 64), 0, s, pred, offsets, n_k, n_v, N, lists);
        const int64_t blocks = std::min<int64_t>((n_k + AM_WAVES - 1) / AM_WAVES, 1 << 20);
        hipLaunchKernelGGL((topn_merge_kernel<K>), dim3((unsigned)blocks), dim3(AM_WAVES * 64), 0, s,
                           pred, offsets, n_k, n_v, N, (const uint64_t *)lists, idx_out, val_out);
        return;
    }
    const int64_t blocks = std::min<int64_t>((n_k + AM_WAVES - 1) / AM_WAVES, 1 << 20);
    if constexpr (K >= 8) {
        hipLaunchKernelGGL((topn_preds_kernel<K, TOPN_FAST>), dim3((unsigned)blocks),
                           dim3(AM_WAVES * 64), 0, s, pred, offsets, n_k, n_v, N, idx_out, val_out);
        hipLaunchKernelGGL((topn_preds_kernel<K, TOPN_MARKED>), dim3((unsigned)blocks),
                           dim3(AM_WAVES * 64), 0, s, pred, offsets, n_k, n_v, N, idx_out, val_out);
    } else {
        hipLaunchKernelGGL((topn_preds_kernel<K, TOPN_ALL>), dim3((unsigned)blocks),
                           dim3(AM_WAVES * 64), 0, s, pred, offsets, n_k, n_v, N, idx_out, val_out);
    }
}

// Long segments on average take the chunked form, with its lists in a
// stream-ordered scratch allocation freed after the merge.
int launch_topn_preds(const float *pred, const int64_t *offsets, int64_t n_k, int64_t n_v,
                      int N, int64_t *idx_out, float *val_out, hipStream_t s)
{
    uint64_t *lists = nullptr;
    if (n_v >= AM_LONG * n_k) {
        const int64_t chunks = (n_v + AM_CHUNK - 1) / AM_CHUNK;
        ADV_HIP(hipMallocAsync((void **)&lists, sizeof(uint64_t) * (size_t)(chunks + n_k) * N, s));
    }
    if (N <= 1) launch_topn<1>(pred, offsets, n_k, n_v, N, idx_out, val_out, lists, s);
    else if (N <= 2) launch_topn<2>(pred, offsets, n_k, n_v, N, idx_out, val_out, lists, s);
    else if (N <= 4) launch_topn<4>(pred, offsets, n_k, n_v, N, idx_out, val_out, lists, s);
    else if (N <= 8) launch_topn<8>(pred, offsets, n_k, n_v, N, idx_out, val_out, lists, s);
    else if (N <= 16) launch_topn<16>(pred, offsets, n_k, n_v, N, idx_out, val_out, lists, s);
    else launch_topn<32>(pred, offsets, n_k, n_v, N, idx_out, val_out, lists, s);
    const hipError_t le = hipGetLastError();
    const hipError_t fe = lists ? hipFreeAsync(lists, s) : hipSuccess;
    if (le != hipSuccess) return hip_fail(le, "topn_preds_kernel");
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    return ADVISOR_OK;
}

// The kernel segments are well formed when offsets[0] = 0, offsets[n_k] =
// n_v and offsets[i] <= offsets[i + 1]; first_bad gets the lowest index
// whose entry breaks that (a 64-bit vector atomic min, starting at ~0).
__global__ void offsets_check_kernel(const int64_t *__restrict__ off, int64_t n_k, int64_t n_v,
                                     unsigned long long *__restrict__ first_bad)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n_k; i += stride) {
        const int64_t v = off[i];
        const bool bad = (i == 0 && v != 0) || (i == n_k && v != n_v) || (i < n_k && v > off[i + 1]);
        if (bad) atomicMin(first_bad, (unsigned long long)i);
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v) { *p = v; }

// Opt-in checking of the segments before a ranking call: the environment
// variable ADVISOR_DEBUG_OFFSETS set to a non-empty value other than "0"
// (read at every call; skipped while the stream is being captured).
bool debug_offsets(hipStream_t s)
{
    const char *e = getenv("ADVISOR_DEBUG_OFFSETS");
    return e && e[0] && !(e[0] == '0' && e[1] == 0) && !stream_capturing(s);
}

}  // namespace adv

using namespace adv;

extern "C" int advisor_validate_offsets(const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                                        int64_t *first_bad, void *stream)
{
    clear_error();
    if (first_bad) *first_bad = -1;
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (!offsets) return fail(ADVISOR_EINVAL, "advisor_validate_offsets: null offsets");
    hipStream_t s = as_stream(stream);
    unsigned long long *d = nullptr;
    ADV_HIP(hipMalloc((void **)&d, sizeof(unsigned long long)));
    unsigned long long h = ~0ull;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(1), 0, s, d, ~0ull);
    const int64_t blocks = std::min<int64_t>((n_kernels + 1 + 255) / 256, 4096);
    hipLaunchKernelGGL(offsets_check_kernel, dim3((unsigned)blocks), dim3(256), 0, s, offsets,
                       n_kernels, n_variants, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "offsets check");
    if (h == ~0ull) return ADVISOR_OK;
    if (first_bad) *first_bad = (int64_t)h;
    return fail(ADVISOR_ESHAPE, "offsets are not a segmentation of the variants: first bad entry " +
                                    std::to_string((long long)h) +
                                    " (need offsets[0] = 0, non-decreasing, offsets[n_kernels] = n_variants)");
}

extern "C" int advisor_featurize(const int64_t *kdesc, const int64_t *vdesc, int64_t n_kernels,
                                 int64_t n_variants, int64_t *feat_out, uint8_t *invalid_out,
                                 void *stream)
{
    clear_error();
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants == 0) return ADVISOR_OK;
    if (!vdesc || !feat_out || (n_kernels > 0 && !kdesc))
        return fail(ADVISOR_EINVAL, "advisor_featurize: null pointer");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    const int64_t blocks = (n_variants + FZ_THREADS - 1) / FZ_THREADS;
    hipLaunchKernelGGL(featurize_kernel, dim3((unsigned)blocks), dim3(FZ_THREADS), 0,
                       as_stream(stream), kdesc, vdesc, n_kernels, n_variants, feat_out,
                       invalid_out);
    ADV_LAUNCHED("featurize_kernel");
    return ADVISOR_OK;
}

extern "C" int advisor_zscore_fit(const int64_t *feat, int64_t n, double *mu_out,
                                  double *sigma_out, void *stream)
{
    clear_error();
    if (n < 1) return fail(ADVISOR_ESHAPE, "advisor_zscore_fit: n must be >= 1");
    if (!feat || !mu_out || !sigma_out) return fail(ADVISOR_EINVAL, "advisor_zscore_fit: null pointer");
    hipStream_t s = as_stream(stream);
    const int n_blocks = (int)std::min<int64_t>(256, (n + 255) / 256);
    const int64_t rows_per_block = (n + n_blocks - 1) / n_blocks;
    const size_t bytes = (size_t)n_blocks * NFEAT * (sizeof(double) + 2 * sizeof(int64_t)) +
                         NFEAT * sizeof(int);
    void *ws = nullptr;
    ADV_HIP(hipMallocAsync(&ws, bytes, s));
    double *psum = (double *)ws;
    int64_t *pmin = (int64_t *)(psum + n_blocks * NFEAT);
    int64_t *pmax = pmin + n_blocks * NFEAT;
    int *cflag = (int *)(pmax + n_blocks * NFEAT);
    hipLaunchKernelGGL(zscore_partial_kernel, dim3(n_blocks), dim3(ZS_THREADS), 0, s, feat, n,
                       rows_per_block, (const double *)nullptr, psum, pmin, pmax);
    hipLaunchKernelGGL(zscore_final_kernel, dim3(1), dim3(64), 0, s, psum, pmin, pmax, n_blocks,
                       n, 1, mu_out, sigma_out, cflag);
    hipLaunchKernelGGL(zscore_partial_kernel, dim3(n_blocks), dim3(ZS_THREADS), 0, s, feat, n,
                       rows_per_block, (const double *)mu_out, psum, (int64_t *)nullptr,
                       (int64_t *)nullptr);
    hipLaunchKernelGGL(zscore_final_kernel, dim3(1), dim3(64), 0, s, psum, pmin, pmax, n_blocks,
                       n, 2, mu_out, sigma_out, cflag);
    hipError_t le = hipGetLastError();
    hipError_t fe = hipFreeAsync(ws, s);
    if (le != hipSuccess) return hip_fail(le, "zscore kernels");
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    return ADVISOR_OK;
}

extern "C" int advisor_rank_preds(const float *pred, const int64_t *offsets, int64_t n_kernels,
                                  int64_t n_variants, int64_t *best_out, void *stream)
{
    clear_error();
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!offsets || !best_out || (n_variants > 0 && !pred))
        return fail(ADVISOR_EINVAL, "advisor_rank_preds: null pointer");
    if (debug_offsets(as_stream(stream))) {
        if (int rc = advisor_validate_offsets(offsets, n_kernels, n_variants, nullptr, stream)) return rc;
    }
    hipStream_t s = as_stream(stream);
    if (n_variants >= AM_LONG * n_kernels) {
        // long segments: chunks of variants, per-kernel keys in best_out
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(best_out);
        const unsigned kb = (unsigned)((n_kernels + 255) / 256);
        hipLaunchKernelGGL(argmin_keys_init_kernel, dim3(kb), dim3(256), 0, s, keys, n_kernels);
        const int64_t waves = (n_variants + AM_CHUNK - 1) / AM_CHUNK;
        hipLaunchKernelGGL(argmin_chunks_kernel, dim3((unsigned)((waves + AM_WAVES - 1) / AM_WAVES)),
                           dim3(AM_WAVES * 64), 0, s, pred, offsets, n_kernels, n_variants, keys);
        hipLaunchKernelGGL(argmin_keys_final_kernel, dim3(kb), dim3(256), 0, s, best_out, n_kernels);
        ADV_LAUNCHED("argmin_chunks_kernel");
        return ADVISOR_OK;
    }
    const int64_t blocks = std::min<int64_t>((n_kernels + AM_WAVES - 1) / AM_WAVES, 1 << 20);
    hipLaunchKernelGGL(argmin_preds_kernel, dim3((unsigned)blocks), dim3(AM_WAVES * 64), 0,
                       s, pred, offsets, n_kernels, n_variants, best_out);
    ADV_LAUNCHED("argmin_preds_kernel");
    return ADVISOR_OK;
}

extern "C" int advisor_topn_preds(const float *pred, const int64_t *offsets, int64_t n_kernels,
                                  int64_t n_variants, int top_n, int64_t *idx_out, float *val_out,
                                  void *stream)
{
    clear_error();
    if (top_n < 1 || top_n > ADVISOR_MAX_TOP_N)
        return fail(ADVISOR_EINVAL, "top_n must be in [1, 32]");
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels >= ((int64_t)1 << 62) / ADVISOR_MAX_TOP_N)
        return fail(ADVISOR_ESHAPE, "n_kernels too large");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!offsets || !idx_out || (n_variants > 0 && !pred))
        return fail(ADVISOR_EINVAL, "advisor_topn_preds: null pointer");
    hipStream_t s = as_stream(stream);
    if (debug_offsets(s)) {
        if (int rc = advisor_validate_offsets(offsets, n_kernels, n_variants, nullptr, stream)) return rc;
    }
    return launch_topn_preds(pred, offsets, n_kernels, n_variants, top_n, idx_out, val_out, s);
}
