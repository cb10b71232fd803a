// Multi-stage ranking: a fast low-precision model ranks every variant, each
// kernel's K best variants by its predictions go on to a second, more
// precise model, whose K' best go on to a third, and so on; the last model's
// argmin over its candidates is the answer. Near-ties that low-precision
// rounding could order either way are thereby decided as the last model
// decides them, at the cost of its predictions for a few candidates per
// kernel. It is the argmin of section 3's prediction flow (N = 1) over
// candidate sets chosen by the same network in lower precisions.
// The file also holds the prediction flow with a top-N list (the fused pass,
// then the segmented top-N on its predictions), which shares the workspace.
#include <algorithm>

#include "internal.h"
#include "wave_select.h"

namespace adv {

// A model's workspace for the multi-stage and top-N calls: one device arena,
// grown on demand (synchronous allocation).
struct RankWs {
    unsigned char *base = nullptr;
    size_t bytes = 0;
};

void free_refine_ws(advisor_model *m)
{
    RankWs *w = reinterpret_cast<RankWs *>(m->refine_ws);
    if (!w) return;
    if (w->base) (void)hipFree(w->base);
    delete w;
    m->refine_ws = nullptr;
}

static int ensure_arena(advisor_model *m, size_t bytes, unsigned char **out)
{
    RankWs *w = reinterpret_cast<RankWs *>(m->refine_ws);
    if (!w) {
        w = new (std::nothrow) RankWs();
        if (!w) return fail(ADVISOR_ENOMEM, "host allocation");
        m->refine_ws = w;
    }
    if (bytes > w->bytes) {
        if (w->base) (void)hipFree(w->base);
        w->base = nullptr;
        w->bytes = 0;
        ADV_HIP(hipMalloc((void **)&w->base, bytes));
        w->bytes = bytes;
    }
    *out = w->base;
    return ADVISOR_OK;
}

CascadeLayout cascade_layout(int64_t n_v, int64_t n_k, const int *keep, int n_stages,
                                    bool own_pred)
{
    CascadeLayout L;
    size_t at = 0;
    auto take = [&](size_t b) {
        const size_t o = at;
        at += (b + 255) & ~(size_t)255;
        return o;
    };
    if (own_pred) L.pred = take(sizeof(float) * (size_t)n_v);
    for (int s = 0; s + 1 < n_stages; ++s) {
        const size_t rows = (size_t)n_k * keep[s];
        L.cand[s] = take(8 * rows);
        L.vd[s] = take(8 * rows * VD);
        L.off[s] = take(8 * ((size_t)n_k + 1));
        if (s + 2 < n_stages) L.cpred[s] = take(4 * rows);
    }
    L.best = take(8 * (size_t)n_k);
    L.total = at;
    return L;
}

constexpr int RF_WAVES = 4;
constexpr int RF_UNROLL = 16;

// One wave per kernel segment of a workload's predictions: the K smallest
// keys (prediction, row; pred_key) of its non-NaN predictions, written as
// candidate variant indices in ascending order, padded with -1. Lists of 8
// or more over a segment of at most 64 * RF_UNROLL rows take the threshold
// path (threshold_select: a bound on the K-th smallest key from one wave
// sort, then at most 64 candidates gathered and sorted, and the best K
// sorted again by row); other segments, and threshold paths with more than
// 64 candidates, keep a sorted list of each lane's own K best, then K rounds
// of a wave-wide minimum pop the overall best. Lists of 8 or more take two
// launches: the first (TK_FAST, few registers) holds only the threshold path
// and marks each kernel it leaves undone with -2 in its first candidate
// slot; the second (TK_MARKED) runs the per-lane lists on the marked
// kernels. Shorter lists take one launch (TK_ALL) of the lists, which was
// measured faster for them. A row's
// variant index is map[row] for a compact workload (map = the previous
// stage's candidates, ascending within each kernel, so row order is variant
// order and ties still go to the lowest variant index), else the row itself.
// The candidates' descriptor rows are gathered from the original vdesc with
// kernel id k (padding rows get kernel id -1: never eligible).
enum { TK_ALL = 0, TK_FAST = 1, TK_MARKED = 2 };

template <int K, int MODE>
__global__ __launch_bounds__(RF_WAVES * 64) void topk_gather_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets,
    const int64_t *__restrict__ map, const int64_t *__restrict__ vdesc, int64_t n_k,
    int64_t n_rows, int64_t *__restrict__ cand, int64_t *__restrict__ vdesc_c,
    int64_t *__restrict__ off_c)
{
    __shared__ uint64_t cand_lds[RF_WAVES][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t k = (int64_t)blockIdx.x * RF_WAVES + wave;
    if (k > n_k) return;
    if constexpr (MODE == TK_MARKED) {
        if (k == n_k || cand[k * K] != -2) return;  // done by the threshold path
    }
    if (k == n_k) {  // the last offset
        if (lane == 0) off_c[n_k] = n_k * K;
        return;
    }
    const int64_t lo = max((int64_t)0, min(offsets[k], n_rows));
    const int64_t hi = max(lo, min(offsets[k + 1], n_rows));
    // candidate `slot` of this kernel: the variant of `row` (INT64_MAX: none)
    // and its descriptor row, with kernel id k (-1 for padding)
    auto emit = [&](int64_t row, int slot) {
        const int64_t dst_row = k * K + slot;
        int64_t var = -1;
        if (row != INT64_MAX) var = map ? map[row] : row;
        cand[dst_row] = var;
        const int64_t *src = vdesc + (var >= 0 ? var : 0) * VD;
        int64_t *dst = vdesc_c + dst_row * VD;
#pragma unroll
        for (int c = 0; c < VD; ++c) dst[c] = var >= 0 ? (c == 0 ? k : src[c]) : (c == 0 ? -1 : 0);
    };
    if constexpr (MODE == TK_FAST) {
        // 16-byte copies of descriptor rows where both ends allow them
        const bool wide = ((reinterpret_cast<uintptr_t>(vdesc) | reinterpret_cast<uintptr_t>(vdesc_c)) & 15) == 0;
        if (hi - lo <= 64 * RF_UNROLL) {  // the same for every lane
            uint64_t x[RF_UNROLL];
#pragma unroll
            for (int u = 0; u < RF_UNROLL; ++u) {
                const int64_t i = lo + lane + 64 * u;
                const float pv = i < hi ? pred[i] : __builtin_nanf("");
                x[u] = __builtin_isnan(pv) ? ~0ull : pred_key(pv, (uint32_t)i);
            }
            uint64_t v;
            if (threshold_select(x, K, lane, cand_lds[wave], v)) {
                // rows are below 2^32 - 1 (the variant count is below 2^32),
                // so the all-ones row of padding sorts last; lanes 0..K-1
                // end in ascending row order
                const uint32_t r32 = lane < K && v != ~0ull ? (uint32_t)v : ~0u;
                const uint32_t row = bitonic_from<2, K>(r32, lane);
                int64_t var = -1;
                if (lane < K && row != ~0u) var = map ? map[row] : (int64_t)row;
                if (lane < K) cand[k * K + lane] = var;
                // the K descriptor rows are one contiguous block of the
                // output: LPC lanes copy each row, CPL columns apiece
                constexpr int LPC = 64 / K < VD ? 64 / K : VD, CPL = VD / LPC;
                static_assert(VD % LPC == 0, "a row splits evenly over its lanes");
                const int c = min(lane / LPC, K - 1), part = lane % LPC;
                const bool copies = lane < K * LPC;
                const uint32_t vlo = (uint32_t)__shfl((int)(uint32_t)var, c, 64);
                const uint32_t vhi = (uint32_t)__shfl((int)(uint32_t)((uint64_t)var >> 32), c, 64);
                const int64_t vc = (int64_t)(((uint64_t)vhi << 32) | vlo);
                const int64_t *src = vdesc + (vc >= 0 ? vc : 0) * VD + part * CPL;
                int64_t *dst = vdesc_c + (k * K + c) * VD + part * CPL;
                int64_t col[CPL];
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int cc = part * CPL + q;
                    col[q] = cc == 0 ? (vc >= 0 ? k : -1) : 0;
                }
                typedef long long v2ll_ __attribute__((ext_vector_type(2)));
                if constexpr (CPL % 2 == 0) {
                    if (wide && copies) {
#pragma unroll
                        for (int q = 0; q < CPL; q += 2) {
                            v2ll_ w = vc >= 0 ? *reinterpret_cast<const v2ll_ *>(src + q) : v2ll_{0, 0};
                            if (part * CPL + q == 0) w[0] = col[0];
                            *reinterpret_cast<v2ll_ *>(dst + q) = w;
                        }
                    }
                }
                if ((CPL % 2 != 0 || !wide) && copies) {
#pragma unroll
                    for (int q = 0; q < CPL; ++q)
                        dst[q] = vc >= 0 && part * CPL + q != 0 ? src[q] : col[q];
                }
                if (lane == 0) off_c[k] = k * K;
                return;
            }
        }
        if (lane == 0) {
            cand[k * K] = -2;  // left to the per-lane lists
            off_c[k] = k * K;
        }
        return;
    }
    uint64_t top[K];
#pragma unroll
    for (int q = 0; q < K; ++q) top[q] = ~0ull;
    // RF_UNROLL loads per lane in flight per pass (a segment of up to
    // 64 * RF_UNROLL variants in one round trip), then their insertions
    for (int64_t base = lo + lane; base < hi; base += 64 * RF_UNROLL) {
        float pv[RF_UNROLL];
#pragma unroll
        for (int u = 0; u < RF_UNROLL; ++u) {
            const int64_t i = base + 64 * u;
            pv[u] = i < hi ? pred[i] : __builtin_nanf("");
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < RF_UNROLL; ++u) {
            if (__builtin_isnan(pv[u])) continue;
            uint64_t x = pred_key(pv[u], (uint32_t)(base + 64 * u));
            if (x >= top[K - 1]) continue;
            // insertion into the sorted list (compile-time indices only)
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const uint64_t t = top[q];
                const bool less = x < t;
                top[q] = less ? x : t;
                x = less ? t : x;
            }
        }
    }
    // K rounds: the wave-wide minimum of the lanes' heads (the same value in
    // every lane, kept scalar), popped from the lane that holds it
    int64_t crow[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        uint64_t v = top[0];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const uint64_t o = __shfl_xor(v, off, 64);
            v = o < v ? o : v;
        }
        const uint32_t vlo = __builtin_amdgcn_readfirstlane((uint32_t)v);
        const uint32_t vhi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
        v = ((uint64_t)vhi << 32) | vlo;
        crow[r] = v == ~0ull ? INT64_MAX : (int64_t)vlo;
        if (v != ~0ull && top[0] == v) {  // keys are unique (they hold the row)
#pragma unroll
            for (int q = 0; q + 1 < K; ++q) top[q] = top[q + 1];
            top[K - 1] = ~0ull;
        }
    }
    // lane r < K takes the r-th popped row and writes it to the slot of its
    // rank in ascending row order (padding, INT64_MAX, sorts last)
    if (lane < K) {
        int64_t mine = INT64_MAX;
#pragma unroll
        for (int r = 0; r < K; ++r)
            if (lane == r) mine = crow[r];
        int slot = 0;
#pragma unroll
        for (int r = 0; r < K; ++r) slot += (crow[r] < mine || (crow[r] == mine && r < lane)) ? 1 : 0;
        emit(mine, slot);
    }
    if (lane == 0) off_c[k] = k * K;
}

// best[k] = the candidate the last stage chose (its variant index), or -1
__global__ void refine_map_kernel(const int64_t *__restrict__ best_c,
                                  const int64_t *__restrict__ cand, int64_t n_k,
                                  int64_t *__restrict__ best)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_k) {
        const int64_t b = best_c[k];
        best[k] = b >= 0 ? cand[b] : -1;
    }
}

static int launch_topk(int K, const float *pred, const int64_t *offsets, const int64_t *map,
                       const int64_t *vdesc, int64_t n_k, int64_t n_rows, int64_t *cand,
                       int64_t *vdesc_c, int64_t *off_c, hipStream_t s)
{
    const unsigned blocks = (unsigned)((n_k + 1 + RF_WAVES - 1) / RF_WAVES);
#define ADV_TK1(KK, MODE)                                                                        \
    hipLaunchKernelGGL((topk_gather_kernel<KK, MODE>), dim3(blocks), dim3(RF_WAVES * 64), 0, s, \
                       pred, offsets, map, vdesc, n_k, n_rows, cand, vdesc_c, off_c);
#define ADV_TK(KK)                       \
    case KK:                             \
        if constexpr (KK >= 8) {         \
            ADV_TK1(KK, TK_FAST)         \
            ADV_TK1(KK, TK_MARKED)       \
        } else {                         \
            ADV_TK1(KK, TK_ALL)          \
        }                                \
        break;
    switch (K) {
        ADV_TK(1) ADV_TK(2) ADV_TK(4) ADV_TK(8) ADV_TK(16) ADV_TK(32)
    default: return fail(ADVISOR_EINVAL, "candidates per kernel must be 1, 2, 4, 8, 16 or 32");
    }
#undef ADV_TK
#undef ADV_TK1
    ADV_LAUNCHED("topk_gather_kernel");
    return ADVISOR_OK;
}

// Argument checks shared by the multi-stage entry points.
int cascade_check(const advisor_model *const *models, const int *keep, int n_stages,
                         const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                         int64_t n_kernels, int64_t n_variants, const int64_t *best_out)
{
    if (n_stages < 1 || n_stages > CS_MAX_STAGES) return fail(ADVISOR_EINVAL, "1 to 4 stages");
    if (n_stages > 1 && !keep) return fail(ADVISOR_EINVAL, "null keep");
    for (int s = 0; s + 1 < n_stages; ++s) {
        const int K = keep[s];
        if (K != 1 && K != 2 && K != 4 && K != 8 && K != 16 && K != 32)
            return fail(ADVISOR_EINVAL, "candidates per kernel must be 1, 2, 4, 8, 16 or 32");
        if (s > 0 && K > keep[s - 1])
            return fail(ADVISOR_EINVAL, "a stage keeps no more candidates than the one before");
    }
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels >= ((int64_t)1 << 31) / CS_MAX_K)
        return fail(ADVISOR_ESHAPE, "n_kernels * 32 must be < 2^31");
    if (!models) return fail(ADVISOR_EINVAL, "null models");
    for (int s = 0; s < n_stages; ++s) {
        if (!models[s]) return fail(ADVISOR_EINVAL, "null model");
        if (models[s]->device != models[0]->device)
            return fail(ADVISOR_EINVAL, "the models live on different devices");
    }
    if (n_kernels > 0 && (!kdesc || !offsets || !best_out || (n_variants > 0 && !vdesc)))
        return fail(ADVISOR_EINVAL, "null pointer");
    return ADVISOR_OK;
}

// The stages, on a workspace of at least cascade_layout(...).total bytes.
int cascade_run(const advisor_model *const *models, const int *keep, int n_stages,
                       const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                       int64_t n_k, int64_t n_v, int64_t *best_out, float *pred_out,
                       unsigned char *ws, hipStream_t s, bool may_check_offsets)
{
    const CascadeLayout L = cascade_layout(n_v, n_k, keep, n_stages, pred_out == nullptr);
    float *pred = pred_out ? pred_out : reinterpret_cast<float *>(ws + L.pred);
    // first stage: every variant (its argmin is the answer only with one stage)
    int rc = rank_core(models[0], kdesc, vdesc, offsets, n_k, n_v, best_out,
                       n_stages > 1 ? pred : pred_out, s, may_check_offsets);
    if (rc || n_stages == 1 || n_v == 0) return rc;  // no variant: every kernel is -1 already
    const float *P = pred;
    const int64_t *offP = offsets;
    const int64_t *mapP = nullptr;
    int64_t rowsP = n_v;
    int64_t *best_c = reinterpret_cast<int64_t *>(ws + L.best);
    for (int st = 0; st + 1 < n_stages; ++st) {
        const int K = keep[st];
        int64_t *cand = reinterpret_cast<int64_t *>(ws + L.cand[st]);
        int64_t *vd_c = reinterpret_cast<int64_t *>(ws + L.vd[st]);
        int64_t *off_c = reinterpret_cast<int64_t *>(ws + L.off[st]);
        rc = launch_topk(K, P, offP, mapP, vdesc, n_k, rowsP, cand, vd_c, off_c, s);
        if (rc) return rc;
        const bool last = st + 2 == n_stages;
        float *cp = last ? nullptr : reinterpret_cast<float *>(ws + L.cpred[st]);
        rc = rank_core(models[st + 1], kdesc, vd_c, off_c, n_k, n_k * K, best_c, cp, s, false);
        if (rc) return rc;
        if (last) {
            hipLaunchKernelGGL(refine_map_kernel, dim3((unsigned)((n_k + 255) / 256)), dim3(256),
                               0, s, best_c, cand, n_k, best_out);
            ADV_LAUNCHED("refine_map_kernel");
        }
        P = cp;
        offP = off_c;
        mapP = cand;
        rowsP = n_k * K;
    }
    return ADVISOR_OK;
}

}  // namespace adv

using namespace adv;

extern "C" int advisor_rank_cascade(advisor_model *const *models, const int *keep, int n_stages,
                                    const int64_t *kdesc, const int64_t *vdesc,
                                    const int64_t *offsets, int64_t n_kernels,
                                    int64_t n_variants, int64_t *best_out, float *pred_out,
                                    void *stream)
{
    clear_error();
    int rc = cascade_check(models, keep, n_stages, kdesc, vdesc, offsets, n_kernels, n_variants,
                           best_out);
    if (rc || n_kernels == 0) return rc;
    unsigned char *ws = nullptr;
    if (n_stages > 1) {
        const CascadeLayout L = cascade_layout(n_variants, n_kernels, keep, n_stages,
                                               pred_out == nullptr);
        rc = ensure_arena(models[0], L.total, &ws);
        if (rc) return rc;
    }
    return cascade_run(models, keep, n_stages, kdesc, vdesc, offsets, n_kernels, n_variants,
                       best_out, pred_out, ws, as_stream(stream), true);
}

extern "C" int advisor_rank_refined(advisor_model *model, const advisor_model *refine,
                                    const int64_t *kdesc, const int64_t *vdesc,
                                    const int64_t *offsets, int64_t n_kernels,
                                    int64_t n_variants, int top_k, int64_t *best_out,
                                    float *pred_out, void *stream)
{
    clear_error();
    if (!model || !refine) return fail(ADVISOR_EINVAL, "advisor_rank_refined: null model");
    if (top_k != 1 && top_k != 2 && top_k != 4 && top_k != 8 && top_k != 16)
        return fail(ADVISOR_EINVAL, "top_k must be 1, 2, 4, 8 or 16");
    advisor_model *const models[2] = {model, const_cast<advisor_model *>(refine)};
    const int keep[1] = {top_k};
    return advisor_rank_cascade(models, keep, 2, kdesc, vdesc, offsets, n_kernels, n_variants,
                                best_out, pred_out, stream);
}

extern "C" int advisor_rank_topn(advisor_model *model, const int64_t *kdesc, const int64_t *vdesc,
                                 const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                                 int top_n, int64_t *idx_out, float *val_out, float *pred_out,
                                 void *stream)
{
    clear_error();
    if (!model) return fail(ADVISOR_EINVAL, "advisor_rank_topn: null model");
    if (top_n < 1 || top_n > ADVISOR_MAX_TOP_N)
        return fail(ADVISOR_EINVAL, "top_n must be in [1, 32]");
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels >= (int64_t)1 << 31) return fail(ADVISOR_ESHAPE, "n_kernels must be < 2^31");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!kdesc || !offsets || !idx_out || (n_variants > 0 && !vdesc))
        return fail(ADVISOR_EINVAL, "advisor_rank_topn: null pointer");
    hipStream_t s = as_stream(stream);
    // workspace: the predictions (unless the caller keeps them), then the
    // fused pass's argmin, which is not used
    const size_t pbytes = pred_out ? 0 : ((sizeof(float) * (size_t)n_variants + 255) & ~(size_t)255);
    unsigned char *ws = nullptr;
    int rc = ensure_arena(model, pbytes + 8 * (size_t)n_kernels, &ws);
    if (rc) return rc;
    float *pred = pred_out ? pred_out : reinterpret_cast<float *>(ws);
    rc = advisor_rank(model, kdesc, vdesc, offsets, n_kernels, n_variants,
                      reinterpret_cast<int64_t *>(ws + pbytes), pred, s);
    if (rc) return rc;
    return launch_topn_preds(pred, offsets, n_kernels, n_variants, top_n, idx_out, val_out, s);
}
