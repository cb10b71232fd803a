// Launch side of the fused tile pipeline: tile shapes per (precision,
// width), kernel instances, the argmin-key set-up and read-out kernels, and
// the advisor_predict / advisor_rank entry points.
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "mlp_tile.h"

namespace adv {

// Event pairs around tile-kernel launches while profiling is enabled.
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;

static void prof_clear_locked()
{
    for (auto &e : g_prof_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    g_prof_events.clear();
}

// Tile shapes. Shape 0 is the default of each (precision, width): rows per
// tile M as large as LDS allows (activations [M][W] plus the input tile),
// 8 waves (two per SIMD, 256 registers each) except the 1024-wide fp8 tile
// (one wave per SIMD and its 512 registers), and NS passes over each wave's
// neurons for the 1024-wide tiles and the 512-wide bf16 and fp8 tiles. Shape 1 halves the rows with 8 waves.
// Shape 2 halves the rows (or quarters them for 1024 bf16 and 512 fp32
// neurons) and the waves, so two workgroups share each CU by LDS and by
// registers: one's input stage, epilogues and barriers overlap the other's
// matrix work, at the price of more weight traffic from L2 (and, for bf16
// and fp8 layers of 512 or more neurons, two or four passes over the
// activations to stay within 256 registers). Shapes with the
// same wave count give bit-identical predictions; the autotuner picks one per
// model.
template <int P, int W, int V> struct TileShape;
template <int P, int W> struct TileShape<P, W, 0> {
    static constexpr bool exists = true;
    static constexpr bool PP = false;
    // bf16x3 tiles hold activations of fp32 size: the fp32 rows per tile
    static constexpr int M = (P == PREC_FP32 || P == PREC_X3)
                                 ? (W <= 256 ? 128 : (W == 512 ? 64 : 32))
                                 : (P == PREC_BF16 ? (W <= 512 ? 128 : 64) : 128);
    static constexpr int NW = (W == 1024 && P == PREC_FP8) ? 4 : 8;
    // two passes at 512 wide in bf16 and fp8 (a wave's 128 x 64 accumulators
    // in one pass spill: 36 B per lane in bf16, 296 in fp8), except for the
    // training forward, whose copy-out registers spill more with two
    static constexpr int NS = W == 1024 ? (P == PREC_FP8 ? 4 : (P == PREC_BF16 ? 2 : 1))
                                        : ((W == 512 && (P == PREC_BF16 || P == PREC_FP8)) ? 2 : 1);
    static constexpr int NS_TRAIN = W == 1024 ? NS : 1;
};
template <int P, int W> struct TileShape<P, W, 1> {
    static constexpr bool PP = false;
    static constexpr bool exists = (P == PREC_FP32 && W == 256) ||
                                   (P == PREC_BF16 && (W == 256 || W == 512 || W == 1024)) ||
                                   (P == PREC_FP8 && (W == 512 || W == 1024));
    static constexpr int M = (P == PREC_BF16 && W == 1024) ? 32 : 64;
    static constexpr int NW = 8;
    static constexpr int NS = (P == PREC_FP8 && W == 1024) ? 2 : 1;
};
template <int P, int W> struct TileShape<P, W, 2> {
    static constexpr bool PP = false;
    static constexpr bool exists = (P == PREC_FP32 && (W == 256 || W == 512)) ||
                                   (P == PREC_BF16 && (W == 256 || W == 512 || W == 1024)) ||
                                   (P == PREC_FP8 && W == 512);
    static constexpr int M = ((P == PREC_BF16 && W == 1024) || (P == PREC_FP32 && W == 512)) ? 32 : 64;
    static constexpr int NW = 4;
    static constexpr int NS = P == PREC_FP32 ? 1 : ((P == PREC_FP8 && W == 1024) ? 4 : (W >= 512 ? 2 : 1));
};
// Shape 3 is the ping-pong schedule (mlp_pp_kernel) on the rows and waves
// of shape 0 (of shape 1 for 1024-wide fp8 layers, whose shape 0 has four
// waves), where each wave holds an even number of 32-row blocks; it gives
// the same bits as that shape.
template <int P, int W> struct TileShape<P, W, 3> {
    static constexpr bool PP = true;
    static constexpr bool exists = (P == PREC_FP32 && (W == 256 || W == 512)) ||
                                   (P == PREC_BF16 && (W == 256 || W == 512 || W == 1024)) ||
                                   (P == PREC_FP8 && (W == 512 || W == 1024));
    using Base = TileShape<P, W, (P == PREC_FP8 && W == 1024) ? 1 : 0>;
    static constexpr int M = Base::M;
    static constexpr int NW = Base::NW;
    static constexpr int NS = 1;
};
constexpr int N_TILE_SHAPES = 4;

// (a grouped pass runs shape 3's rows and waves on mlp_tiles_kernel: the
// same bits as the ping-pong kernel)
// Passes over a wave's neurons as a kernel with this sink runs the shape
// (only shape 0 runs the training forward).
template <class S, int SINK> constexpr int shape_passes()
{
    if constexpr (SINK == SINK_TRAIN) return S::NS_TRAIN;
    else return S::NS;
}

template <class S, int P, int W, int SRC, int SINK, bool PP = S::PP && SINK != SINK_GROUP>
struct TileKernel {
    static constexpr auto kern = mlp_tiles_kernel<P, W, S::M, S::NW, shape_passes<S, SINK>(), SRC, SINK>;
};
template <class S, int P, int W, int SRC, int SINK> struct TileKernel<S, P, W, SRC, SINK, true> {
    static constexpr auto kern = mlp_pp_kernel<P, W, S::M, S::NW, SRC, SINK>;
};

__global__ void keys_init_kernel(uint64_t *keys, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = ~0ull;
}

// argmin key -> global variant index (low 32 bits), -1 if no variant won
__global__ void keys_final_kernel(int64_t *best, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint64_t k = (uint64_t)best[i];
        best[i] = k == ~0ull ? -1 : (int64_t)(k & 0xffffffffull);
    }
}

template <int P, int W, int V, int SRC, int SINK>
struct TileLaunch {
    using S = TileShape<P, W, V>;
    static constexpr int M = S::M;
    static constexpr int NW = S::NW;
    static constexpr int NS = shape_passes<S, SINK>();
    using C = TileCfg<P, W, M, NW, NS,
                      SRC == SRC_DESC && SINK != SINK_GROUP && tile_vdesc_prefetch<P, W, M, NW>(),
                      SINK != SINK_GROUP && SINK != SINK_TRAIN && !S::PP &&
                          tile_bias_lds<P, W, M, NW>()>;
    static constexpr auto kern = TileKernel<S, P, W, SRC, SINK>::kern;
    static inline std::once_flag once;
    static inline int blocks_per_cu = 1;
    static inline hipError_t setup_err = hipSuccess;
    // dynamic-LDS limit and occupancy, once per process
    static int setup()
    {
        std::call_once(once, [] {
            setup_err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)C::LDS);
            if (setup_err == hipSuccess) {
                int nb = 0;
                setup_err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &nb, reinterpret_cast<const void *>(kern), C::THREADS, C::LDS);
                blocks_per_cu = nb > 0 ? nb : 1;
            }
        });
        return setup_err == hipSuccess ? ADVISOR_OK : hip_fail(setup_err, "tile kernel set-up");
    }
};

template <int P, int W, int V, int SRC, int SINK>
int launch_tiles(const typename KernelArgs<SINK>::type &kargs, hipStream_t s)
{
    using TL = TileLaunch<P, W, V, SRC, SINK>;
    using C = typename TL::C;
    int rc = TL::setup();
    if (rc) return rc;
    const TileArgs &args = base_args(kargs);
    const int64_t ntiles = SINK == SINK_TRAIN ? args.save_ld / TL::M
                                              : (args.n_rows + TL::M - 1) / TL::M;
    const int64_t grid = std::min<int64_t>(ntiles, (int64_t)device_cus() * TL::blocks_per_cu);
    if (grid <= 0) return ADVISOR_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        if (g_prof_on && !stream_capturing(s)) {
            ADV_HIP(hipEventCreate(&e0));
            ADV_HIP(hipEventCreate(&e1));
            ADV_HIP(hipEventRecord(e0, s));
        }
    }
    hipLaunchKernelGGL(TL::kern, dim3((unsigned)grid), dim3(C::THREADS), C::LDS, s, kargs);
    ADV_LAUNCHED("mlp_tiles_kernel");
    if (e0) {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        ADV_HIP(hipEventRecord(e1, s));
        g_prof_events.emplace_back(e0, e1);
    }
    return ADVISOR_OK;
}

bool tile_shape_exists(int precision, int W, int V)
{
    if (V == 0) return true;
    if (V < 1 || V >= N_TILE_SHAPES) return false;
#define ADV_E(P, WW)                                                                   \
    if (precision == P && W == WW)                                                     \
        return V == 1 ? TileShape<P, WW, 1>::exists                                    \
                      : (V == 2 ? TileShape<P, WW, 2>::exists : TileShape<P, WW, 3>::exists);
#define ADV_EW(P) ADV_E(P, 64) ADV_E(P, 128) ADV_E(P, 256) ADV_E(P, 512) ADV_E(P, 1024)
    ADV_EW(PREC_FP32)
    ADV_EW(PREC_BF16)
    ADV_EW(PREC_FP8)
    ADV_EW(PREC_X3)
#undef ADV_EW
#undef ADV_E
    return false;
}

int prepare_model_kernels(int precision, int tile_w)
{
#define ADV_P(P, WW)                                                                   \
    if (precision == P && tile_w == WW) {                                              \
        int rc = TileLaunch<P, WW, 0, SRC_DESC, SINK_RANK>::setup();                   \
        if (!rc) rc = TileLaunch<P, WW, 0, SRC_FEAT, SINK_PRED>::setup();              \
        if constexpr (P == PREC_FP32 || P == PREC_BF16)                                \
            if (!rc) rc = TileLaunch<P, WW, 0, SRC_FEAT, SINK_TRAIN>::setup();         \
        if constexpr (TileShape<P, WW, 1>::exists) {                                   \
            if (!rc) rc = TileLaunch<P, WW, 1, SRC_DESC, SINK_RANK>::setup();          \
            if (!rc) rc = TileLaunch<P, WW, 1, SRC_FEAT, SINK_PRED>::setup();          \
        }                                                                              \
        if constexpr (TileShape<P, WW, 2>::exists) {                                   \
            if (!rc) rc = TileLaunch<P, WW, 2, SRC_DESC, SINK_RANK>::setup();          \
            if (!rc) rc = TileLaunch<P, WW, 2, SRC_FEAT, SINK_PRED>::setup();          \
        }                                                                              \
        if constexpr (TileShape<P, WW, 3>::exists) {                                   \
            if (!rc) rc = TileLaunch<P, WW, 3, SRC_DESC, SINK_RANK>::setup();          \
            if (!rc) rc = TileLaunch<P, WW, 3, SRC_FEAT, SINK_PRED>::setup();          \
        }                                                                              \
        return rc;                                                                     \
    }
#define ADV_PW(P) ADV_P(P, 64) ADV_P(P, 128) ADV_P(P, 256) ADV_P(P, 512) ADV_P(P, 1024)
    ADV_PW(PREC_FP32)
    ADV_PW(PREC_BF16)
    ADV_PW(PREC_FP8)
    ADV_PW(PREC_X3)
#undef ADV_PW
#undef ADV_P
    return fail(ADVISOR_EUNSUPPORTED, "no tile kernel for this precision and width");
}

template <int SRC, int SINK>
int dispatch_tiles(int precision, int W, int variant, const typename KernelArgs<SINK>::type &a,
                   hipStream_t s)
{
#define ADV_CASE(P, WW)                                                          \
    if (precision == P && W == WW) {                                             \
        if constexpr (TileShape<P, WW, 1>::exists)                               \
            if (variant == 1) return launch_tiles<P, WW, 1, SRC, SINK>(a, s);    \
        if constexpr (TileShape<P, WW, 2>::exists)                               \
            if (variant == 2) return launch_tiles<P, WW, 2, SRC, SINK>(a, s);    \
        if constexpr (TileShape<P, WW, 3>::exists && SINK != SINK_GROUP)         \
            if (variant == 3) return launch_tiles<P, WW, 3, SRC, SINK>(a, s);    \
        return launch_tiles<P, WW, 0, SRC, SINK>(a, s);                          \
    }
#define ADV_WIDTHS(P) ADV_CASE(P, 64) ADV_CASE(P, 128) ADV_CASE(P, 256) ADV_CASE(P, 512) ADV_CASE(P, 1024)
    ADV_WIDTHS(PREC_FP32)
    ADV_WIDTHS(PREC_BF16)
    ADV_WIDTHS(PREC_FP8)
    ADV_WIDTHS(PREC_X3)
#undef ADV_WIDTHS
#undef ADV_CASE
    return fail(ADVISOR_EUNSUPPORTED, "no tile kernel for this precision and width");
}

// Training forward: predictions plus the transposed activations the
// backward pass reads (fp32 and bf16 models).
int launch_train_forward(const advisor_model *m, const TileArgs &a0, hipStream_t s);

NetView net_view(const advisor_model *m)
{
    NetView v{};
    for (int l = 0; l < m->n_hidden; ++l) {
        v.w[l] = m->wpack[l];
        v.b[l] = m->bias + (size_t)l * m->tile_w;
        v.qscale[l] = m->qscale[l];
        v.qinv[l] = m->qinv[l];
    }
    v.head_w = m->head;
    v.head_b = m->head + m->tile_w;
    v.mu = m->mu;
    v.sigma = m->sigma;
    v.n_hidden = m->n_hidden;
    return v;
}

int check_model_ready(const advisor_model *m)
{
    if (!m) return fail(ADVISOR_EINVAL, "null model");
    if (m->precision == PREC_FP8 && !m->fp8_calibrated)
        return fail(ADVISOR_EINVAL, "fp8 model used before advisor_model_calibrate_fp8");
    int dev = -1;
    ADV_HIP(hipGetDevice(&dev));
    if (dev != m->device) return fail(ADVISOR_EINVAL, "model lives on another device");
    return ADVISOR_OK;
}

int launch_train_forward(const advisor_model *m, const TileArgs &a0, hipStream_t s)
{
    TileArgs a = a0;
    a.net = net_view(m);
#define ADV_T(P, WW) \
    if (m->precision == P && m->tile_w == WW) return launch_tiles<P, WW, 0, SRC_FEAT, SINK_TRAIN>(a, s);
    ADV_T(PREC_FP32, 64) ADV_T(PREC_FP32, 128) ADV_T(PREC_FP32, 256) ADV_T(PREC_FP32, 512)
    ADV_T(PREC_FP32, 1024) ADV_T(PREC_BF16, 64) ADV_T(PREC_BF16, 128) ADV_T(PREC_BF16, 256)
    ADV_T(PREC_BF16, 512) ADV_T(PREC_BF16, 1024)
#undef ADV_T
    return fail(ADVISOR_EUNSUPPORTED, "training needs an fp32 or bf16 model");
}

}  // namespace adv

using namespace adv;

extern "C" int advisor_predict(const advisor_model *model, const int64_t *feat, int64_t n,
                               float *pred_out, void *stream)
{
    clear_error();
    int rc = check_model_ready(model);
    if (rc) return rc;
    if (n < 0) return fail(ADVISOR_ESHAPE, "negative row count");
    if (n == 0) return ADVISOR_OK;
    if (!feat || !pred_out) return fail(ADVISOR_EINVAL, "advisor_predict: null pointer");
    if (n >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "row count must be < 2^32");
    TileArgs a{};
    a.feat = feat;
    a.n_rows = n;
    a.net = net_view(model);
    a.pred = pred_out;
    return dispatch_tiles<SRC_FEAT, SINK_PRED>(model->precision, model->tile_w,
                                               model->tile_variant, a, as_stream(stream));
}

namespace adv {

int rank_core(const advisor_model *model, const int64_t *kdesc, const int64_t *vdesc,
              const int64_t *offsets, int64_t n_kernels, int64_t n_variants, int64_t *best_out,
              float *pred_out, hipStream_t s, bool may_check_offsets)
{
    int rc = check_model_ready(model);
    if (rc) return rc;
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels >= (int64_t)1 << 31) return fail(ADVISOR_ESHAPE, "n_kernels must be < 2^31");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!kdesc || !offsets || !best_out || (n_variants > 0 && !vdesc))
        return fail(ADVISOR_EINVAL, "advisor_rank: null pointer");
    if (may_check_offsets && debug_offsets(s)) {
        if (int rc2 = advisor_validate_offsets(offsets, n_kernels, n_variants, nullptr, s)) return rc2;
    }
    const unsigned kb = (unsigned)((n_kernels + 255) / 256);
    hipLaunchKernelGGL(keys_init_kernel, dim3(kb), dim3(256), 0, s,
                       reinterpret_cast<uint64_t *>(best_out), n_kernels);
    ADV_LAUNCHED("keys_init_kernel");
    if (n_variants > 0) {
        TileArgs a{};
        a.kdesc = kdesc;
        a.vdesc = vdesc;
        a.offsets = offsets;
        a.n_k = n_kernels;
        a.n_rows = n_variants;
        a.net = net_view(model);
        a.pred = pred_out;
        a.keys = reinterpret_cast<uint64_t *>(best_out);
        rc = dispatch_tiles<SRC_DESC, SINK_RANK>(model->precision, model->tile_w,
                                                 model->tile_variant, a, s);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(keys_final_kernel, dim3(kb), dim3(256), 0, s, best_out, n_kernels);
    ADV_LAUNCHED("keys_final_kernel");
    return ADVISOR_OK;
}

}  // namespace adv

extern "C" int advisor_rank(const advisor_model *model, const int64_t *kdesc,
                            const int64_t *vdesc, const int64_t *offsets, int64_t n_kernels,
                            int64_t n_variants, int64_t *best_out, float *pred_out, void *stream)
{
    clear_error();
    return rank_core(model, kdesc, vdesc, offsets, n_kernels, n_variants, best_out, pred_out,
                     as_stream(stream), true);
}

namespace adv {

// The tile shape a grouped pass runs a model on: its own, except that the
// ping-pong shape runs as the shape it schedules (the same bits).
static int group_variant(const advisor_model *m)
{
    if (m->tile_variant != 3) return m->tile_variant;
    return (m->precision == PREC_FP8 && m->tile_w == 1024) ? 1 : 0;
}

// Whether two models can share a grouped pass: one kernel instance (precision,
// tile width, tile shape) and one input tile (identical Z-score statistics).
static bool groupable(const advisor_model *a, const advisor_model *b)
{
    if (a->precision != b->precision || a->tile_w != b->tile_w) return false;
    if (group_variant(a) != group_variant(b)) return false;
    if (!a->h_stats || !b->h_stats) return false;
    return std::memcmp(a->h_mu, b->h_mu, sizeof(a->h_mu)) == 0 &&
           std::memcmp(a->h_sigma, b->h_sigma, sizeof(a->h_sigma)) == 0;
}

// One grouped pass: the input tile of each tile is built once (with the
// shared statistics) and every model's network runs on it; model i's keys
// go to best_out row idx[i].
static int rank_group(const advisor_model *const *models, const int *idx, int n_group,
                      const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                      int64_t n_kernels, int64_t n_variants, int64_t *best_out, float *pred_out,
                      hipStream_t s)
{
    const advisor_model *m0 = models[idx[0]];
    const unsigned kb = (unsigned)((n_kernels + 255) / 256);
    GroupArgs g{};
    g.base.kdesc = kdesc;
    g.base.vdesc = vdesc;
    g.base.offsets = offsets;
    g.base.n_k = n_kernels;
    g.base.n_rows = n_variants;
    g.base.net = net_view(m0);
    g.n_models = n_group;
    for (int i = 0; i < n_group; ++i) {
        int64_t *row = best_out + (int64_t)idx[i] * n_kernels;
        hipLaunchKernelGGL(keys_init_kernel, dim3(kb), dim3(256), 0, s,
                           reinterpret_cast<uint64_t *>(row), n_kernels);
        g.nets[i] = net_view(models[idx[i]]);
        g.keys[i] = reinterpret_cast<uint64_t *>(row);
        g.pred[i] = pred_out ? pred_out + (int64_t)idx[i] * n_variants : nullptr;
    }
    ADV_LAUNCHED("keys_init_kernel");
    if (n_variants > 0) {
        int rc = dispatch_tiles<SRC_DESC, SINK_GROUP>(m0->precision, m0->tile_w, group_variant(m0),
                                                      g, s);
        if (rc) return rc;
    }
    for (int i = 0; i < n_group; ++i)
        hipLaunchKernelGGL(keys_final_kernel, dim3(kb), dim3(256), 0, s,
                           best_out + (int64_t)idx[i] * n_kernels, n_kernels);
    ADV_LAUNCHED("keys_final_kernel");
    return ADVISOR_OK;
}

}  // namespace adv

extern "C" int advisor_rank_multi(const advisor_model *const *models, int n_models,
                                  const int64_t *kdesc, const int64_t *vdesc,
                                  const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                                  int64_t *best_out, float *pred_out, void *stream)
{
    clear_error();
    if (n_models < 1 || !models) return fail(ADVISOR_EINVAL, "need at least one model");
    for (int t = 0; t < n_models; ++t) {
        if (int rc = check_model_ready(models[t])) return rc;
        if (models[t]->device != models[0]->device)
            return fail(ADVISOR_EINVAL, "the models live on different devices");
    }
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (n_kernels >= (int64_t)1 << 31) return fail(ADVISOR_ESHAPE, "n_kernels must be < 2^31");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!best_out) return fail(ADVISOR_EINVAL, "advisor_rank_multi: null best_out");
    if (!kdesc || !offsets || (n_variants > 0 && !vdesc))
        return fail(ADVISOR_EINVAL, "advisor_rank_multi: null pointer");
    hipStream_t s = as_stream(stream);
    if (debug_offsets(s)) {
        if (int rc = advisor_validate_offsets(offsets, n_kernels, n_variants, nullptr, stream))
            return rc;
    }
    // models that share a kernel instance and their statistics run in one
    // grouped pass (at most GROUP_MAX each); the others alone
    std::vector<char> done((size_t)n_models, 0);
    std::vector<int> idx;
    for (int t0 = 0; t0 < n_models; ++t0) {
        if (done[t0]) continue;
        idx.assign(1, t0);
        done[t0] = 1;
        for (int t1 = t0 + 1; t1 < n_models && (int)idx.size() < GROUP_MAX; ++t1)
            if (!done[t1] && groupable(models[t0], models[t1])) {
                idx.push_back(t1);
                done[t1] = 1;
            }
        int rc = idx.size() > 1
                     ? rank_group(models, idx.data(), (int)idx.size(), kdesc, vdesc, offsets,
                                  n_kernels, n_variants, best_out, pred_out, s)
                     : rank_core(models[t0], kdesc, vdesc, offsets, n_kernels, n_variants,
                                 best_out + (int64_t)t0 * n_kernels,
                                 pred_out ? pred_out + (int64_t)t0 * n_variants : nullptr, s,
                                 false);
        if (rc) return rc;
    }
    return ADVISOR_OK;
}

extern "C" int advisor_profile_enable(int on)
{
    clear_error();
    std::lock_guard<std::mutex> lock(g_prof_mu);
    prof_clear_locked();
    g_prof_on = on != 0;
    return ADVISOR_OK;
}

extern "C" int advisor_profile_read_each(double *ms_out, int64_t cap, int64_t *launches)
{
    clear_error();
    if (cap < 0) return fail(ADVISOR_EINVAL, "negative capacity");
    std::lock_guard<std::mutex> lock(g_prof_mu);
    int64_t i = 0;
    for (auto &e : g_prof_events) {
        ADV_HIP(hipEventSynchronize(e.second));
        float ms = 0.0f;
        ADV_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        if (ms_out && i < cap) ms_out[i] = ms;
        ++i;
    }
    if (launches) *launches = (int64_t)g_prof_events.size();
    prof_clear_locked();
    return ADVISOR_OK;
}

extern "C" int advisor_profile_read(int64_t *launches, double *total_ms)
{
    clear_error();
    std::lock_guard<std::mutex> lock(g_prof_mu);
    double sum = 0.0;
    for (auto &e : g_prof_events) {
        ADV_HIP(hipEventSynchronize(e.second));
        float ms = 0.0f;
        ADV_HIP(hipEventElapsedTime(&ms, e.first, e.second));
        sum += ms;
    }
    if (launches) *launches = (int64_t)g_prof_events.size();
    if (total_ms) *total_ms = sum;
    prof_clear_locked();
    return ADVISOR_OK;
}
