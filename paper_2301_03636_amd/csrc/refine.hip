// Precision-refined ranking: a low-precision model ranks every variant, then
// each kernel's K best variants by its predictions are ranked again by a
// second (higher-precision) model, so near-ties that low-precision rounding
// could order either way are decided as the second model decides them. The
// argmin of section 3's prediction flow (N = 1) over a candidate set chosen
// by the same network in another precision.
// The file also holds the prediction flow with a top-N list (the fused pass,
// then the segmented top-N on its predictions), which shares the workspace.
#include <algorithm>

#include "internal.h"

namespace adv {

constexpr int RF_MAX_K = 16;

struct RefineWs {
    int64_t n_v = 0, n_k = 0;
    int k = 0;
    float *pred = nullptr;      // [n_v] first-pass predictions
    int64_t *cand = nullptr;    // [n_k * K] candidate variant indices, ascending, -1 padded
    int64_t *vdesc_c = nullptr; // [n_k * K][8] candidate descriptors
    int64_t *off_c = nullptr;   // [n_k + 1] = k * K
    int64_t *best_c = nullptr;  // [n_k] second-pass winners (index into the candidates)
};

void free_refine_ws(advisor_model *m)
{
    RefineWs *w = reinterpret_cast<RefineWs *>(m->refine_ws);
    if (!w) return;
    void *ptrs[] = {w->pred, w->cand, w->vdesc_c, w->off_c, w->best_c};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete w;
    m->refine_ws = nullptr;
}

static int ensure_refine_ws(advisor_model *m, int64_t n_v, int64_t n_k, int k)
{
    RefineWs *w = reinterpret_cast<RefineWs *>(m->refine_ws);
    if (!w) {
        w = new (std::nothrow) RefineWs();
        if (!w) return fail(ADVISOR_ENOMEM, "host allocation");
        m->refine_ws = w;
    }
    if (n_v > w->n_v) {
        if (w->pred) (void)hipFree(w->pred);
        w->pred = nullptr;
        w->n_v = 0;
        ADV_HIP(hipMalloc((void **)&w->pred, sizeof(float) * n_v));
        w->n_v = n_v;
    }
    if (n_k > w->n_k || k > w->k) {
        const int64_t nk = std::max(n_k, w->n_k);
        const int kk = std::max(k, w->k);
        for (void **p : {(void **)&w->cand, (void **)&w->vdesc_c, (void **)&w->off_c, (void **)&w->best_c})
            if (*p) { (void)hipFree(*p); *p = nullptr; }
        w->n_k = 0;
        w->k = 0;
        ADV_HIP(hipMalloc((void **)&w->cand, sizeof(int64_t) * nk * kk));
        ADV_HIP(hipMalloc((void **)&w->vdesc_c, sizeof(int64_t) * nk * kk * VD));
        ADV_HIP(hipMalloc((void **)&w->off_c, sizeof(int64_t) * (nk + 1)));
        ADV_HIP(hipMalloc((void **)&w->best_c, sizeof(int64_t) * nk));
        w->n_k = nk;
        w->k = kk;
    }
    return ADVISOR_OK;
}

// order-preserving key of (prediction, index): smaller prediction first,
// then lower index; -0 equals +0
__device__ __forceinline__ uint64_t rf_key(float p, uint32_t idx)
{
    uint32_t u = __float_as_uint(p == 0.0f ? 0.0f : p);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | idx;
}

constexpr int RF_WAVES = 4;

// One wave per kernel segment: the K smallest keys of its non-NaN
// predictions (each lane keeps a sorted list of its own K best, then K rounds
// of a wave-wide minimum pop the overall best), written as candidate indices
// in ascending index order, padded with -1; the candidates' descriptors are
// gathered with kernel id k (padding rows get kernel id -1: invalid).
template <int K>
__global__ __launch_bounds__(RF_WAVES * 64) void topk_gather_kernel(
    const float *__restrict__ pred, const int64_t *__restrict__ offsets,
    const int64_t *__restrict__ vdesc, int64_t n_k, int64_t n_v, int64_t *__restrict__ cand,
    int64_t *__restrict__ vdesc_c, int64_t *__restrict__ off_c)
{
    const int lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * RF_WAVES + (threadIdx.x >> 6);
    if (k > n_k) return;
    if (k == n_k) {  // the last offset
        if (lane == 0) off_c[n_k] = n_k * K;
        return;
    }
    const int64_t lo = max((int64_t)0, min(offsets[k], n_v));
    const int64_t hi = max(lo, min(offsets[k + 1], n_v));
    uint64_t top[K];
#pragma unroll
    for (int q = 0; q < K; ++q) top[q] = ~0ull;
    for (int64_t i = lo + lane; i < hi; i += 64) {
        const float p = pred[i];
        if (__builtin_isnan(p)) continue;
        uint64_t x = rf_key(p, (uint32_t)i);
        // insertion into the sorted list (compile-time indices only)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const uint64_t t = top[q];
            const bool less = x < t;
            top[q] = less ? x : t;
            x = less ? t : x;
        }
    }
    // K rounds: the wave-wide minimum of the lanes' heads, popped from its lane
    uint64_t chosen[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        uint64_t v = top[0];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const uint64_t o = __shfl_xor(v, off, 64);
            v = o < v ? o : v;
        }
        chosen[r] = v;
        if (v != ~0ull && top[0] == v) {  // keys are unique (they hold the index)
#pragma unroll
            for (int q = 0; q + 1 < K; ++q) top[q] = top[q + 1];
            top[K - 1] = ~0ull;
        }
    }
    // candidate indices in ascending order (padding ~0 sorts last)
    int64_t idx[K];
#pragma unroll
    for (int r = 0; r < K; ++r) idx[r] = chosen[r] == ~0ull ? INT64_MAX : (int64_t)(chosen[r] & 0xffffffffull);
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b + 1 < K - a; ++b) {
            const int64_t x = idx[b], y = idx[b + 1];
            idx[b] = x < y ? x : y;
            idx[b + 1] = x < y ? y : x;
        }
    // lane s < K writes slot s; lanes K .. write nothing
    int64_t mine = INT64_MAX;
#pragma unroll
    for (int r = 0; r < K; ++r)
        if (lane == r) mine = idx[r];
    if (lane < K) {
        const int64_t slot = k * K + lane;
        const bool has = mine != INT64_MAX;
        cand[slot] = has ? mine : -1;
        const int64_t *src = vdesc + (has ? mine : 0) * VD;
        int64_t *dst = vdesc_c + slot * VD;
#pragma unroll
        for (int c = 0; c < VD; ++c) dst[c] = has ? (c == 0 ? k : src[c]) : (c == 0 ? -1 : 0);
    }
    if (lane == 0) off_c[k] = k * K;
}

// best[k] = the candidate the second pass chose (its variant index), or -1
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

template <int K>
static void launch_topk(const float *pred, const int64_t *offsets, const int64_t *vdesc,
                        int64_t n_k, int64_t n_v, RefineWs *w, hipStream_t s)
{
    const unsigned blocks = (unsigned)((n_k + 1 + RF_WAVES - 1) / RF_WAVES);
    hipLaunchKernelGGL(topk_gather_kernel<K>, dim3(blocks), dim3(RF_WAVES * 64), 0, s, pred,
                       offsets, vdesc, n_k, n_v, w->cand, w->vdesc_c, w->off_c);
}

}  // namespace adv

using namespace adv;

extern "C" int advisor_rank_refined(advisor_model *model, const advisor_model *refine,
                                    const int64_t *kdesc, const int64_t *vdesc,
                                    const int64_t *offsets, int64_t n_kernels,
                                    int64_t n_variants, int top_k, int64_t *best_out,
                                    float *pred_out, void *stream)
{
    clear_error();
    if (!model || !refine) return fail(ADVISOR_EINVAL, "advisor_rank_refined: null model");
    if (model->device != refine->device)
        return fail(ADVISOR_EINVAL, "the two models live on different devices");
    if (top_k != 1 && top_k != 2 && top_k != 4 && top_k != 8 && top_k != 16)
        return fail(ADVISOR_EINVAL, "top_k must be 1, 2, 4, 8 or 16");
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels >= ((int64_t)1 << 31) / RF_MAX_K)
        return fail(ADVISOR_ESHAPE, "n_kernels * top_k must be < 2^31");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!kdesc || !offsets || !best_out || (n_variants > 0 && !vdesc))
        return fail(ADVISOR_EINVAL, "advisor_rank_refined: null pointer");
    hipStream_t s = as_stream(stream);
    int rc = ensure_refine_ws(model, n_variants, n_kernels, top_k);
    if (rc) return rc;
    RefineWs *w = reinterpret_cast<RefineWs *>(model->refine_ws);
    float *pred = pred_out ? pred_out : w->pred;
    // first pass: every variant, low precision (its argmin is not used)
    rc = advisor_rank(model, kdesc, vdesc, offsets, n_kernels, n_variants, best_out, pred, s);
    if (rc) return rc;
    if (n_variants == 0) return ADVISOR_OK;  // every kernel is -1 already
    switch (top_k) {
    case 1: launch_topk<1>(pred, offsets, vdesc, n_kernels, n_variants, w, s); break;
    case 2: launch_topk<2>(pred, offsets, vdesc, n_kernels, n_variants, w, s); break;
    case 4: launch_topk<4>(pred, offsets, vdesc, n_kernels, n_variants, w, s); break;
    case 8: launch_topk<8>(pred, offsets, vdesc, n_kernels, n_variants, w, s); break;
    default: launch_topk<16>(pred, offsets, vdesc, n_kernels, n_variants, w, s); break;
    }
    ADV_LAUNCHED("topk_gather_kernel");
    // second pass: the candidates, ranked by the refining model
    rc = advisor_rank(refine, kdesc, w->vdesc_c, w->off_c, n_kernels, n_kernels * top_k,
                      w->best_c, nullptr, s);
    if (rc) return rc;
    hipLaunchKernelGGL(refine_map_kernel, dim3((unsigned)((n_kernels + 255) / 256)), dim3(256), 0,
                       s, w->best_c, w->cand, n_kernels, best_out);
    ADV_LAUNCHED("refine_map_kernel");
    return ADVISOR_OK;
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
    int rc = ensure_refine_ws(model, pred_out ? 0 : n_variants, n_kernels, 1);
    if (rc) return rc;
    RefineWs *w = reinterpret_cast<RefineWs *>(model->refine_ws);
    float *pred = pred_out ? pred_out : w->pred;
    // the fused pass; its argmin lands in the workspace and is not used
    rc = advisor_rank(model, kdesc, vdesc, offsets, n_kernels, n_variants, w->best_c, pred, s);
    if (rc) return rc;
    return launch_topn_preds(pred, offsets, n_kernels, n_variants, top_n, idx_out, val_out, s);
}
