/*
 * libadvisor: batched evaluation and training of the OpenMP Advisor's
 * machine-learned cost model (Mishra et al., arXiv 2301.03636) on one
 * AMD Instinct MI355X (gfx950).
 *
 * The paper's prediction mode (sections 3 and 4) generates the offloading
 * variants of a kernel, predicts each variant's runtime with a trained
 * multi-layer perceptron (section 5.3) and returns the best ones; its
 * training mode fits that perceptron to measured (variant, runtime) pairs.
 * This library does both for many kernels at once: every variant's static
 * descriptor becomes 32 integer features, a fully-connected ReLU network
 * predicts its log-runtime, and a segmented argmin picks each kernel's
 * predicted-fastest variant.
 *
 * Conventions shared by every entry point:
 *  - Buffers named "device" are HIP device allocations owned by the caller
 *    (rows are C-contiguous); buffers named "host" are ordinary host memory.
 *  - "stream" is a hipStream_t passed as void* (NULL: the null stream).
 *    Work on device buffers is enqueued on it and returns before it runs;
 *    argument and shape errors are detected on the host and returned
 *    synchronously, before anything is enqueued.
 *  - Return value: ADVISOR_OK (0) or a negative ADVISOR_E* code; the text of
 *    the last error of the calling thread is advisor_last_error().
 *  - Descriptor layout (int64, row-major):
 *      kdesc [n_kernels, 16]: D, N0..N3, A, E, s0..s3, fpi, req0..req3
 *        D loop-nest depth (1..4), N_i trip counts (1 for i >= D), A arrays
 *        (0..4) of E bytes per element (1..64), s_a 1 for a stride-N walk,
 *        fpi flops per innermost iteration, req_a the data class found by
 *        the data analysis of section 4.1.2 (0 alloc, 1 to, 2 from, 3 tofrom)
 *      vdesc [n_variants, 8]: kernel_id, p, T, H, m0..m3
 *        p the parallel structure c + 8 x + 64 d + 512 s (section 4.1.3):
 *        the parallel-for directive at loop x with collapse c, teams
 *        distribute with collapse d, schedule s (0 static, 1 dynamic,
 *        2 guided); x = d = s = 0 is the combined teams-distribute-parallel-
 *        for with collapse c, so p = c there. T teams, H threads per team,
 *        m_a the map clause of array a (same codes as req_a)
 *      offsets [n_kernels + 1]: variants of kernel k are rows
 *        offsets[k] .. offsets[k+1]-1; offsets[0] = 0, offsets[n_kernels] =
 *        n_variants, non-decreasing (empty segments allowed).
 *  - n_variants must stay below 2^32 and n_kernels below 2^31.
 */
#ifndef ADVISOR_H
#define ADVISOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum advisor_status {
    ADVISOR_OK = 0,
    ADVISOR_EINVAL = -1,       /* null pointer, bad enum, bad scalar argument */
    ADVISOR_ESHAPE = -2,       /* sizes inconsistent or outside the supported range */
    ADVISOR_EHIP = -3,         /* a HIP runtime call failed (text in advisor_last_error) */
    ADVISOR_ENOMEM = -4,       /* device or host allocation failed */
    ADVISOR_EUNSUPPORTED = -5  /* network shape or precision not built into the library */
};

enum advisor_precision {
    ADVISOR_FP32 = 0,      /* fp32 weights and activations, fp32 matrix cores */
    ADVISOR_BF16 = 1,      /* bf16 weights and activations, fp32 accumulation */
    ADVISOR_FP8_E4M3 = 2,  /* OCP e4m3 hidden layers with per-tensor scales, first layer bf16 */
    ADVISOR_BF16X3 = 3     /* fp32 weights and activations as bf16 pairs (high part, rounded
                              remainder), three bf16 matrix-core products per product
                              (hi*hi + hi*lo + lo*hi), fp32 accumulation: close to fp32
                              (each product within about 2^-16 relative) at bf16 matrix-core
                              speed; inference only (no training entry points) */
};

#define ADVISOR_NFEAT 32
#define ADVISOR_KD_COLS 16
#define ADVISOR_VD_COLS 8
#define ADVISOR_MAX_LAYERS 9   /* hidden layers + output layer */
#define ADVISOR_MAX_WIDTH 1024
#define ADVISOR_MAX_TOP_N 32     /* longest top-N list of advisor_topn_preds / advisor_rank_topn */
#define ADVISOR_MAX_LOOPS 4      /* collapsible loops per kernel the variant generator handles */
#define ADVISOR_VARIANT_COLS 6   /* columns of a generated variant row */
#define ADVISOR_MAX_STAGES 4     /* models of one advisor_rank_cascade call */

typedef struct advisor_model advisor_model;  /* opaque; owned by the library */

/* Text of the calling thread's last error ("" if none). Owned by the library,
 * valid until the thread's next call. */
const char *advisor_last_error(void);

/* Library version string. */
const char *advisor_version(void);

/*
 * Create a cost model: the multi-layer perceptron of section 5.3 (ReLU hidden
 * layers, a linear single-output layer predicting ln(runtime in us)).
 * widths (host) [n_widths]: 32, h_1, ..., h_L, 1 with 1 <= h_i <= 1024 and
 * 2 <= n_widths <= ADVISOR_MAX_LAYERS + 1. precision: enum advisor_precision
 * (ADVISOR_FP8_E4M3 also needs advisor_model_calibrate_fp8 before use).
 * The model is allocated on the current HIP device; parameters start at 0,
 * mu at 0 and sigma at 1. *out receives the handle (NULL on error).
 */
int advisor_model_create(const int32_t *widths, int n_widths, int precision,
                         advisor_model **out);

/* Free a model and every device buffer it owns. NULL is ignored. */
void advisor_model_destroy(advisor_model *model);

/* Number of parameters: sum over layers of out*in + out. */
int64_t advisor_model_param_count(const advisor_model *model);

/*
 * Load parameters and the Z-score statistics (section 5.3 standardizes the
 * data; here x_j = (log2(1 + f_j) - mu_j) / sigma_j).
 * w_master (host, float) [param_count]: per layer l, W_l as [out, in]
 * row-major followed by b_l [out]. mu, sigma (host, double) [32]; sigma > 0.
 * Copies synchronously, rebuilds the packed compute copies, resets Adam state
 * (m = v = 0, step 0) and any FP8 calibration.
 */
int advisor_model_set_params(advisor_model *model, const float *w_master,
                             const double *mu, const double *sigma);

/* Copy the fp32 master parameters (host, float [param_count]) and, if not
 * NULL, mu and sigma (host, double [32]) out of the model. Synchronous. */
int advisor_model_get_params(const advisor_model *model, float *w_master, double *mu,
                             double *sigma);

/* Copy the Adam state out (host: m, v float [param_count], step) or load it
 * in (advisor_model_set_adam); either array pointer may be NULL to skip it.
 * Synchronous. Used for checkpoint and resume of training. */
int advisor_model_get_adam(const advisor_model *model, float *m, float *v, int64_t *step);
int advisor_model_set_adam(advisor_model *model, const float *m, const float *v, int64_t step);

/*
 * Static activation scales of an ADVISOR_FP8_E4M3 model (required before it
 * predicts or ranks; cleared by advisor_model_set_params). Runs the model in
 * bf16 on feat (device, int64 [n, 32], a calibration sample of variants,
 * 1 <= n < 2^32) and sets each hidden layer's input scale to
 * amax(activation) / 448, the e4m3 maximum; weights were quantized per
 * tensor with amax(|W_l|) / 448 when the parameters were loaded. Conversion
 * is round-to-nearest-even with saturation to +-448. Synchronizes the stream;
 * allocates temporary device memory.
 */
int advisor_model_calibrate_fp8(advisor_model *model, const int64_t *feat, int64_t n,
                                void *stream);

/* Per-layer fp8 scales (host, float [n_hidden] each): weight scale of each
 * hidden layer, and the input-activation scale of each hidden layer (1 for
 * the bf16 first layer). */
int advisor_model_get_fp8_scales(const advisor_model *model, float *wscale, float *ascale);

/*
 * Feature extraction (the Feature Extraction step of the training and
 * prediction flows, section 3; the paper does not list its features, this
 * library defines 32). For each variant i (device inputs kdesc, vdesc as in
 * the header comment), writes feat_out[i, 0..31] (device, int64) and, if
 * invalid_out (device, uint8 [n_variants]) is not NULL, invalid_out[i] = 1
 * for an invalid variant (its feature row is all zero) and 0 otherwise.
 * A variant is invalid when its kernel_id is outside [0, n_kernels), its
 * kernel's D, N_i, A, E, s_a, req_a or fpi is out of range, T < 1, H < 1,
 * its parallel structure is not one of section 4.1.3 (p < 0 or s > 2; at
 * x = 0: d != 0 or c outside 1..D; at x >= 1: x >= D, d outside 1..x or c
 * outside 1..D-x), or a map clause m_a does not carry the data its class
 * req_a needs (to needs to/tofrom, from needs from/tofrom, tofrom needs
 * tofrom). Integer arithmetic is unsigned 64-bit modulo 2^64, exact while
 * trip-count products times 64 stay below 2^63.
 * Features: 0 D, 1-4 N0..N3, 5 I = prod N_i, 6 loops collapsed into parallel
 * work, 7 Pc parallel iterations, 8 R = I / Pc serial iterations per
 * parallel one, 9 T, 10 H, 11 TH = T*H, 12 busy threads, 13 waves rounds of
 * parallel work per thread, 14 waves*R, 15 waves*TH - Pc, 16 A, 17 E,
 * 18 S = E*I, 19-22 arrays mapped to / from / tofrom / alloc,
 * 23 h2d = S*(n_to + n_tofrom), 24 d2h = S*(n_from + n_tofrom),
 * 25 h2d + d2h, 26 ns = number of strided arrays, 27 S*A,
 * 28 S*(A - ns) + (64/E)*S*ns, 29 fpi*I, 30 fpi, 31 S*n_alloc.
 * At x = 0 (combined directive over loops 0..c-1): feature 6 = c,
 * Pc = prod_{i<c} N_i, busy = min(TH, Pc), waves = ceil(Pc/TH). At x >= 1
 * (teams over loops 0..d-1: Pt = prod_{i<d} N_i; a team's threads over loops
 * x..x+c-1: Pf = prod_{x<=i<x+c} N_i): feature 6 = d + c, Pc = Pt*Pf,
 * busy = min(T, Pt)*min(H, Pf), waves = ceil(Pt/T)*ceil(Pf/H). The schedule
 * enters no feature: the paper's printed predictions come in groups of
 * identical values, as variants differing only in such a choice would.
 */
int advisor_featurize(const int64_t *kdesc, const int64_t *vdesc, int64_t n_kernels,
                      int64_t n_variants, int64_t *feat_out, uint8_t *invalid_out, void *stream);

/*
 * Fit the Z-score statistics (section 5.3) on a calibration sample:
 * feat (device, int64 [n, 32]) -> mu_out, sigma_out (device, double [32]):
 * mean and population deviation of log2(1 + f_j), accumulated in float64;
 * a feature with a single value over the sample gets mu = log2(1 + value)
 * and sigma = 1. n >= 1. The result can be copied into a model with
 * advisor_model_set_params or advisor_model_set_zscore.
 */
int advisor_zscore_fit(const int64_t *feat, int64_t n, double *mu_out, double *sigma_out,
                       void *stream);

/* Replace the model's Z-score statistics (device, double [32] each). */
int advisor_model_set_zscore(advisor_model *model, const double *mu, const double *sigma,
                             void *stream);

/*
 * Predict ln(runtime in us) of every row (section 5.3's network applied to
 * the standardized features): feat (device, int64 [n, 32]) ->
 * pred_out (device, float [n]). Every row is treated as valid.
 */
int advisor_predict(const advisor_model *model, const int64_t *feat, int64_t n,
                    float *pred_out, void *stream);

/*
 * The prediction flow of section 3 for many kernels at once, in one fused
 * pass: featurize -> standardize -> network -> per-kernel argmin (the paper
 * sorts predictions and keeps the best N; this is N = 1).
 * best_out (device, int64 [n_kernels]) receives, for each kernel k, the
 * global index of the variant in [offsets[k], offsets[k+1]) with the lowest
 * prediction, the lowest index among equal predictions (-0 equals +0), or -1
 * if the segment has no eligible variant. A variant is eligible when it is
 * valid (see advisor_featurize) and its kernel_id equals k. pred_out (device,
 * float [n_variants], may be NULL) receives every prediction, NaN for
 * ineligible variants, identical bit for bit to advisor_predict on the same
 * features. best_out doubles as scratch during the call.
 */
int advisor_rank(const advisor_model *model, const int64_t *kdesc, const int64_t *vdesc,
                 const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                 int64_t *best_out, float *pred_out, void *stream);

/*
 * Multi-target prediction (section 3 trains one model per cluster and GPU
 * architecture): the same variants ranked by n_models models, each a fused
 * pass as advisor_rank. best_out (device, int64 [n_models, n_kernels],
 * row-major) receives target t's winners in row t; pred_out (device, float
 * [n_models, n_variants], may be NULL) its predictions. Models may differ
 * in widths and precision; all must live on the current device. Each row
 * equals advisor_rank with that model, bit for bit. Models that share the
 * precision, the padded hidden width, the tile shape and the Z-score
 * statistics (set from identical host values by advisor_model_set_params;
 * the statistics describe the variants' features, which do not depend on
 * the target) are evaluated in grouped passes of up to 8 models: each tile's
 * descriptors are read, featurized and standardized once and every model's
 * network runs on that input. Other models get a pass of their own.
 */
int advisor_rank_multi(const advisor_model *const *models, int n_models, const int64_t *kdesc,
                       const int64_t *vdesc, const int64_t *offsets, int64_t n_kernels,
                       int64_t n_variants, int64_t *best_out, float *pred_out, void *stream);

/*
 * Precision-refined ranking (the prediction flow of section 3, N = 1, with
 * the argmin decided in two precisions). `model` (any precision) ranks every
 * variant as advisor_rank does; then, per kernel, its top_k variants by
 * `model`'s predictions (lowest index first on ties; NaN and ineligible
 * variants never enter) are ranked again by `refine`, and best_out[k]
 * receives the one `refine` predicts fastest (lowest variant index on ties),
 * or -1 if the kernel has no eligible variant. When `refine`'s own argmin of
 * the kernel is among those candidates, the result equals advisor_rank with
 * `refine`; a bf16 or fp8 first pass with an fp32 `refine` of the same
 * weights resolves near-ties as fp32 does at the cost of top_k fp32
 * predictions per kernel. top_k in {1, 2, 4, 8, 16}; n_kernels * 16 < 2^31.
 * Arguments as for advisor_rank; pred_out (may be NULL) receives `model`'s
 * predictions. The two models must live on the current device. `model` owns
 * a workspace that grows on demand (synchronous allocation); calls on one
 * model must not overlap.
 */
int advisor_rank_refined(advisor_model *model, const advisor_model *refine,
                         const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                         int64_t n_kernels, int64_t n_variants, int top_k, int64_t *best_out,
                         float *pred_out, void *stream);

/*
 * Multi-stage ranking (the prediction flow of section 3, N = 1, with the
 * argmin decided by the most precise of several models of one network, for
 * example fp8, then bf16, then fp32 copies of the same weights). models[0]
 * ranks every variant as advisor_rank does; for s = 0 .. n_stages - 2, each
 * kernel's keep[s] best candidates by models[s]'s predictions (lowest
 * variant index first on ties; NaN and ineligible variants never enter)
 * are ranked again by models[s + 1], which passes on its own keep[s + 1]
 * best of them; best_out[k] receives the variant the last model predicts
 * fastest among its candidates (lowest variant index on ties), or -1 if the
 * kernel has no eligible variant. Whenever the last model's own argmin of a
 * kernel survives every earlier cut, the result equals advisor_rank with
 * the last model. 1 <= n_stages <= ADVISOR_MAX_STAGES; keep (host,
 * int [n_stages - 1], may be NULL for one stage) values in {1, 2, 4, 8, 16,
 * 32}, non-increasing; n_kernels * 32 < 2^31. Arguments as for
 * advisor_rank; pred_out (may be NULL) receives models[0]'s predictions. All
 * models must live on the current device. models[0] owns a workspace that
 * grows on demand (synchronous allocation; at most 4 n_variants bytes for
 * the first-stage predictions when pred_out is NULL, plus about
 * 80 n_kernels * keep[s] bytes per cut); calls sharing models[0] must not
 * overlap. advisor_rank_refined(model, refine, ..., top_k, ...) is this call
 * with models {model, refine} and keep {top_k}.
 */
int advisor_rank_cascade(advisor_model *const *models, const int *keep, int n_stages,
                         const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                         int64_t n_kernels, int64_t n_variants, int64_t *best_out,
                         float *pred_out, void *stream);

/*
 * advisor_rank_cascade for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. Same arguments, results and argument checks as
 * advisor_rank_cascade (bit-identical picks and predictions), but the
 * stages' workspace (each cut's candidate lists, their gathered descriptor
 * rows and offsets, middle stages' predictions, the last stage's winners;
 * plus 4 n_variants bytes for the first stage's predictions when pred_out
 * is NULL) lives in one library-owned static device array of
 * ADVISOR_NOALLOC_SCRATCH_BYTES bytes per GPU, held from the first call on
 * that GPU until the process ends. The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine) and skips the opt-in offsets check
 * (ADVISOR_DEBUG_OFFSETS), which allocates. A call whose workspace would
 * exceed the array returns ADVISOR_ESHAPE with the sizes in the error text;
 * cut s takes 72 bytes per candidate (76 when another cut follows) for its
 * n_kernels * keep[s] candidates, plus 8 (n_kernels + 1) bytes (the
 * 32768-kernel workload with keep {32, 4} and pred_out given takes 85 MiB).
 * The models must live on the current device. Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (other streams,
 * other threads) race and their picks are undefined; calls ordered on one
 * stream are safe. One-stage calls use no workspace.
 */
#define ADVISOR_NOALLOC_SCRATCH_BYTES (96u << 20)
int advisor_rank_cascade_noalloc(advisor_model *const *models, const int *keep, int n_stages,
                                 const int64_t *kdesc, const int64_t *vdesc,
                                 const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                                 int64_t *best_out, float *pred_out, void *stream);

/*
 * The per-kernel argmin alone (the selection step of section 3, N = 1) on
 * given predictions: pred (device, float [n_variants]), offsets (device,
 * int64 [n_kernels + 1]) -> best_out (device, int64 [n_kernels]), with the
 * tie, signed-zero and empty-segment rules of advisor_rank; NaN never wins.
 * n_variants is offsets[n_kernels], passed for the size check.
 */
int advisor_rank_preds(const float *pred, const int64_t *offsets, int64_t n_kernels,
                       int64_t n_variants, int64_t *best_out, void *stream);

/*
 * The top-N list of the prediction flow (section 3: predicted runtimes are
 * sorted and the N best variants recommended) on given predictions.
 * pred (device, float [n_variants]) and offsets (device, int64
 * [n_kernels + 1]) as for advisor_rank_preds; 1 <= top_n <= 32.
 * idx_out (device, int64 [n_kernels, top_n], row-major) receives, for each
 * kernel k, its variants in ascending order of prediction, the lower index
 * first among equal predictions (-0 equals +0), NaN predictions left out;
 * past the last eligible variant the row holds -1. idx_out[k, 0] is
 * advisor_rank_preds' best[k]. val_out (device, float [n_kernels, top_n],
 * may be NULL) receives the matching predictions, NaN where idx_out is -1.
 */
int advisor_topn_preds(const float *pred, const int64_t *offsets, int64_t n_kernels,
                       int64_t n_variants, int top_n, int64_t *idx_out, float *val_out,
                       void *stream);

/*
 * The prediction flow of section 3 with its top-N list: advisor_rank's fused
 * pass writing every prediction, then advisor_topn_preds on them. idx_out
 * and val_out as for advisor_topn_preds (eligibility as for advisor_rank:
 * invalid variants and those whose kernel_id is not k have NaN predictions
 * and never enter); idx_out[k, 0] equals advisor_rank's best_out[k].
 * pred_out (device, float [n_variants], may be NULL) receives every
 * prediction; when it is NULL the model's workspace holds them (it grows on
 * demand with a synchronous allocation, so calls on one model must not
 * overlap). Limits as for advisor_rank and advisor_topn_preds.
 */
int advisor_rank_topn(advisor_model *model, const int64_t *kdesc, const int64_t *vdesc,
                      const int64_t *offsets, int64_t n_kernels, int64_t n_variants, int top_n,
                      int64_t *idx_out, float *val_out, float *pred_out, void *stream);

/*
 * Data analysis (section 4.1.2). Access bits of a variable a kernel may use
 * (OR of ADVISOR_ACC_*), and the map classes they give (ADVISOR_MAP_*; the
 * first four are the data classes of the kernel descriptor's req columns):
 *   alloc   - first assigned within the kernel and not needed after it;
 *   to      - assigned before and only read within;
 *   from    - updated within and accessed after, not assigned before;
 *   tofrom  - assigned before, updated within and accessed after;
 *   private - declared within the kernel;
 *   none    - neither read nor written within.
 * Patterns those definitions leave open: read within but never modified is
 * to (assigned before or not); assigned before, read and updated within but
 * not needed after is to; assigned before, only written within and not
 * needed after is alloc.
 *
 * advisor_classify_maps: access (device, uint8 [n_vars]) and nbytes
 * (device, int64 [n_vars], each variable's mapped extent in bytes), grouped
 * per kernel by var_offsets (device, int64 [n_kernels + 1]); writes
 * class_out (device, uint8 [n_vars]) and per kernel enter_bytes (to and
 * tofrom bytes, sent by the enter-data directive), exit_bytes (from and
 * tofrom bytes, returned by the exit-data directive) and naive_bytes (twice
 * the bytes of every alloc/to/from/tofrom variable: the code that maps
 * everything to and from the GPU), each device int64 [n_kernels]. Any
 * output may be NULL. Offsets are clamped to [0, n_vars]. Sums wrap modulo
 * 2^64.
 */
enum { ADVISOR_ACC_BEFORE = 1, ADVISOR_ACC_READ = 2, ADVISOR_ACC_WRITE = 4,
       ADVISOR_ACC_AFTER = 8, ADVISOR_ACC_LOCAL = 16 };
enum { ADVISOR_MAP_ALLOC = 0, ADVISOR_MAP_TO = 1, ADVISOR_MAP_FROM = 2, ADVISOR_MAP_TOFROM = 3,
       ADVISOR_MAP_PRIVATE = 4, ADVISOR_MAP_NONE = 5 };
int advisor_classify_maps(const uint8_t *access, const int64_t *nbytes, const int64_t *var_offsets,
                          int64_t n_kernels, int64_t n_vars, uint8_t *class_out,
                          int64_t *enter_bytes, int64_t *exit_bytes, int64_t *naive_bytes,
                          void *stream);

/*
 * Variant generation (section 4.1.3). For a kernel with n collapsible loops
 * (1 <= n <= 4; any other value gives the kernel no variants) loop 0 is
 * distributed over the teams and the parallel-for directive is placed
 * either at loop 0, merged into one combined directive with collapse c in
 * 1..n, or at loop x (1 <= x < n) with teams distribute collapsing d in
 * 1..x loops and parallel for collapsing c in 1..n-x; every placement takes
 * each allowed schedule and both data-transfer options. With all three
 * schedules that is n^3 + 5n variants (6, 18, 42, 84 for n = 1..4).
 *
 * advisor_count_variants: n_loops (device, int64 [n_kernels]) ->
 * offsets_out (device, int64 [n_kernels + 1]): offsets_out[0] = 0 and
 * offsets_out[k+1] - offsets_out[k] = kernel k's variant count.
 * sched_mask (1..7) selects schedules: bit 0 static, bit 1 dynamic, bit 2
 * guided (compilers without dynamic or guided scheduling on the GPU take
 * 1). n_kernels < 2^31. Allocates and frees a small scratch buffer in
 * stream order.
 *
 * advisor_enumerate_variants: with those offsets and n_variants =
 * offsets[n_kernels], writes variants_out (device, int64 [n_variants, 6],
 * row-major): [kernel, x, d, c, schedule (0 static, 1 dynamic, 2 guided),
 * data option (0, 1)], d = 0 for the combined directive at x = 0. Within a
 * kernel the rows run over placements (x ascending; at x = 0 c ascending,
 * then d, c ascending), then allowed schedules ascending, then the data
 * option. Writes stay inside [0, n_variants) rows whatever the offsets;
 * rows past a kernel's own count (offsets not from advisor_count_variants)
 * hold -1.
 */
int advisor_count_variants(const int64_t *n_loops, int64_t n_kernels, int sched_mask,
                           int64_t *offsets_out, void *stream);
int advisor_enumerate_variants(const int64_t *n_loops, const int64_t *offsets, int64_t n_kernels,
                               int64_t n_variants, int sched_mask, int64_t *variants_out,
                               void *stream);

/*
 * Generated variants as the cost model's descriptors, so that they go
 * through featurize -> network -> per-kernel selection (section 3's
 * prediction flow over section 4.1.3's variants). variants (device, int64
 * [n_variants, 6], rows of advisor_enumerate_variants) -> vdesc_out
 * (device, int64 [n_variants, 8]): [kernel, c + 8 x + 64 d + 512 schedule,
 * teams, threads, m0, m1, m2, m3]. The generated directives carry no
 * num_teams or thread_limit clause, so teams and threads (>= 1) are the
 * launch the target runtime makes by default, stated by the caller. Data
 * option 0 maps each array with the class kdesc records for it (the data
 * analysis of section 4.1.2), option 1 maps every array tofrom (the
 * untransformed code); arrays past the kernel's count get 0. A row whose
 * kernel id is outside [0, n_kernels) (the -1 padding of a mismatched
 * enumeration) keeps that id and is an invalid variant for advisor_featurize
 * and advisor_rank. Variants that differ only in schedule get identical
 * features (the schedule enters no feature; see advisor_featurize).
 */
int advisor_lower_variants(const int64_t *kdesc, const int64_t *variants, int64_t n_kernels,
                           int64_t n_variants, int64_t teams, int64_t threads, int64_t *vdesc_out,
                           void *stream);

/*
 * Training (section 5.3: the network is fit to measured runtimes with a
 * squared-error loss; here Adam on the MSE, eq. RMSE squared). Only fp32 and
 * bf16 models train (bf16: bf16 operands, fp32 accumulation, fp32 master
 * weights). Calls on one model must not overlap: the model owns a workspace
 * that grows (synchronous hipMalloc) to the largest batch seen.
 *
 * advisor_mlp_saved_bytes: size of the buffer advisor_mlp_forward fills for a
 * batch of n rows (the transposed inputs and hidden activations and the
 * hidden layers' ReLU masks; its layout is the library's), or -1.
 *
 * advisor_mlp_backward stages dy in the model's workspace (a copy of n
 * floats on the stream) before its kernels read it.
 */
int64_t advisor_mlp_saved_bytes(const advisor_model *model, int64_t n);

/* Forward pass for training: feat (device, int64 [n, 32]) -> y_out (device,
 * float [n]) and saved (device, advisor_mlp_saved_bytes(model, n) bytes,
 * caller-owned, read by advisor_mlp_backward). 1 <= n < 2^32. */
int advisor_mlp_forward(advisor_model *model, const int64_t *feat, int64_t n, float *y_out,
                        void *saved, void *stream);

/* Backward pass: dy (device, float [n]) = dLoss/dy_hat for the rows of the
 * forward call that filled `saved`; writes grads_out (device, float
 * [param_count], the master layout: dW_l [out, in], db_l per layer) by the
 * chain rule (ReLU derivative 0 at 0). Weights must be unchanged since the
 * forward call. */
int advisor_mlp_backward(advisor_model *model, const float *dy, const void *saved, int64_t n,
                         float *grads_out, void *stream);

/* One full training step on a batch: forward, float64 MSE loss
 * L = (1/n) sum (y_hat - y)^2 with y (device, double [n], ln runtime in us),
 * backward, float64 gradient 2-norm, and one Adam step (Kingma and Ba; t
 * counts from 1, no weight decay) on the fp32 master weights, after which the
 * compute copies are rebuilt. loss_out, gnorm_out (device, double [1]) may be
 * NULL. 0 < lr, 0 <= beta1, beta2 < 1, eps >= 0. */
int advisor_train_step(advisor_model *model, const int64_t *feat, const double *y, int64_t n,
                       float lr, float beta1, float beta2, float eps, double *loss_out,
                       double *gnorm_out, void *stream);

/* Losses of advisor_train_step_rmsprop. */
enum { ADVISOR_LOSS_MSE = 0, ADVISOR_LOSS_RMSE = 1 };

/* One training step with the optimizer section 5.3 selects: RMSprop
 * (Hinton's lecture notes) with weight decay as an L2 term of the gradient,
 *   g' = g + weight_decay * w,  v <- alpha v + (1 - alpha) g'^2,
 *   w <- w - lr g' / (sqrt(v) + eps),
 * on every fp32 master parameter (biases included), then the compute copies
 * are rebuilt. loss selects the loss being minimized: ADVISOR_LOSS_MSE
 * (1/n) sum (y_hat - y)^2, or ADVISOR_LOSS_RMSE, its square root (eq. rmse;
 * its gradient is the MSE gradient / (2 RMSE), 0 when the RMSE is 0).
 * loss_out (device, double [1], may be NULL) receives that loss in float64;
 * gnorm_out (device, double [1], may be NULL) the float64 2-norm of its
 * gradient (without the weight-decay term), which advisor_model_grads then
 * returns. The running average v is the model's second-moment buffer, the
 * one advisor_model_get_adam / set_adam read and write as Adam's v (Adam's
 * first moment and step count are left untouched). lr is read at every
 * call; advisor_step_lr gives section 5.3's schedule for it. 0 < lr,
 * 0 <= alpha < 1, eps >= 0, weight_decay >= 0. Other arguments and limits as for advisor_train_step. */
int advisor_train_step_rmsprop(advisor_model *model, const int64_t *feat, const double *y,
                               int64_t n, float lr, float alpha, float eps, float weight_decay,
                               int loss, double *loss_out, double *gnorm_out, void *stream);

/* The stepped learning rate of section 5.3 for epoch `epoch` (counted from
 * 0): lr0 * gamma^floor(epoch / every) (the paper: lr0 = 0.01, gamma = 0.1,
 * every = 30). A host computation, no device work; returns NaN (and sets the
 * error text) when epoch < 0, every < 1, lr0 <= 0 or gamma is outside (0, 1]. */
double advisor_step_lr(int64_t epoch, double lr0, double gamma, int64_t every);

/* Replace the fp32 master weights from a device buffer (float [param_count])
 * and rebuild the compute copies; for optimizers that run outside the
 * library. Adam state is left as it is. */
int advisor_model_load_params(advisor_model *model, const float *w_master, void *stream);

/* Copy the gradient of the last advisor_train_step (device, float
 * [param_count]) into grads_out (device). */
int advisor_model_grads(const advisor_model *model, float *grads_out, void *stream);

/*
 * Tile-shape autotuner. The fused kernel is built in up to four tile shapes
 * per (precision, width) (rows per tile, waves, passes); advisor_autotune
 * times each on the given ranking workload (2 warm-up calls, then `reps`
 * timed advisor_rank calls on the stream, device buffers as for
 * advisor_rank), keeps the fastest for this model's advisor_rank and
 * advisor_predict, and records it in a JSON cache keyed by (GPU
 * architecture, precision, widths): the file named by the environment
 * variable ADVISOR_TUNE_CACHE (an empty value disables the cache), else
 * $HOME/.cache/libadvisor/tune.json; advisor_model_create reads it.
 * times_ms (host, double [max_variants]) receives each shape's mean
 * milliseconds (-1 where a shape is not built); *chosen (may be NULL) the
 * chosen shape. Synchronizes the stream and allocates a temporary buffer.
 * Shapes with the same number of waves give bit-identical predictions;
 * otherwise only the order of the output layer's fp32 sum differs. Shapes:
 * 0 largest row tile, 1 half the rows, 2 two workgroups per CU, 3 ping-pong
 * schedule. ADVISOR_BF16X3 models are built in shape 0 only.
 */
int advisor_autotune(advisor_model *model, const int64_t *kdesc, const int64_t *vdesc,
                     const int64_t *offsets, int64_t n_kernels, int64_t n_variants, int reps,
                     double *times_ms, int max_variants, int *chosen, void *stream);
int advisor_model_set_tile_variant(advisor_model *model, int variant);
int advisor_model_get_tile_variant(const advisor_model *model);

/*
 * Captured plans: one advisor_rank or advisor_train_step call with fixed
 * arguments recorded into a HIP graph, replayed by advisor_plan_launch on
 * any stream with the same effect as repeating the call (the same kernels,
 * bit-identical results). The buffers named at creation must stay allocated
 * and their contents are read at replay time. advisor_train_plan_create
 * reserves the training workspace for n rows and rebuilds the transposed
 * weights before capturing; it does not run a step. A plan belongs to the
 * device current at creation. Replays of one plan must not overlap, and the
 * model must not be destroyed while a plan of it exists.
 */
typedef struct advisor_plan advisor_plan;
int advisor_rank_plan_create(const advisor_model *model, const int64_t *kdesc,
                             const int64_t *vdesc, const int64_t *offsets, int64_t n_kernels,
                             int64_t n_variants, int64_t *best_out, float *pred_out,
                             advisor_plan **out);
int advisor_train_plan_create(advisor_model *model, const int64_t *feat, const double *y,
                              int64_t n, float lr, float beta1, float beta2, float eps,
                              double *loss_out, double *gnorm_out, advisor_plan **out);
/* advisor_train_step_rmsprop captured the same way; lr is fixed in the plan,
 * so a stepped schedule takes one plan per learning rate. */
int advisor_train_plan_create_rmsprop(advisor_model *model, const int64_t *feat, const double *y,
                                      int64_t n, float lr, float alpha, float eps,
                                      float weight_decay, int loss, double *loss_out,
                                      double *gnorm_out, advisor_plan **out);
/* One RMSprop step of each of n_models (1..64) distinct models, each on its
 * own batch (feats[t], ys[t], ns[t] rows), captured as one plan (the steps
 * one after another in a single branch): section 3's one model per cluster
 * and architecture, trained with one launch per step of all.
 * loss_out and gnorm_out (device, double [n_models], may be NULL) receive
 * model t's loss and gradient norm at index t. Each replay equals
 * advisor_train_step_rmsprop on every model. */
int advisor_train_plan_create_rmsprop_multi(advisor_model *const *models,
                                            const int64_t *const *feats, const double *const *ys,
                                            const int64_t *ns, int n_models, float lr, float alpha,
                                            float eps, float weight_decay, int loss,
                                            double *loss_out, double *gnorm_out,
                                            advisor_plan **out);
int advisor_plan_launch(advisor_plan *plan, void *stream);
/* Waits for the plan's device to finish all queued work (so no launch of the
 * plan is still pending), then frees the plan. */
void advisor_plan_destroy(advisor_plan *plan);

/*
 * Checks that offsets (device, int64 [n_kernels + 1]) segments n_variants
 * variants: offsets[0] = 0, non-decreasing, offsets[n_kernels] = n_variants
 * (section 4.1.1 files every variant under one kernel). Returns ADVISOR_OK,
 * or ADVISOR_ESHAPE with *first_bad (host, may be NULL; -1 when valid) set to
 * the lowest offending index. Synchronizes the stream and allocates 8 bytes.
 * The ranking calls never read outside their arrays on malformed offsets
 * (they clamp), but their results are then meaningless; setting the
 * environment variable ADVISOR_DEBUG_OFFSETS=1 makes advisor_rank,
 * advisor_rank_preds and advisor_rank_refined run this check first (not
 * while the stream is being captured) and fail with its status.
 */
int advisor_validate_offsets(const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                             int64_t *first_bad, void *stream);

/*
 * Measurement aid (not part of the method): while enabled, every launch of
 * the fused tile kernel (advisor_rank, advisor_predict) is bracketed by a
 * pair of HIP events recorded on the caller's stream. advisor_profile_read
 * waits for the recorded events, returns the number of bracketed launches
 * and their summed duration in milliseconds (either pointer may be NULL),
 * and forgets them. Enabling or disabling also forgets them. Not thread-safe
 * against concurrent calls that launch the tile kernel.
 */
int advisor_profile_enable(int on);
int advisor_profile_read(int64_t *launches, double *total_ms);
/*
 * advisor_profile_read with every bracketed launch's own duration: ms_out
 * (host, double [cap], may be NULL) receives the first min(cap, launches)
 * durations in milliseconds in launch order (a multi-stage call launches
 * the tile kernel once per stage); *launches (may be NULL) the number of
 * bracketed launches. Waits for the recorded events and forgets them;
 * EINVAL if cap < 0.
 */
int advisor_profile_read_each(double *ms_out, int64_t cap, int64_t *launches);

/*
 * Measurement aid (not part of the method): the sustained matrix-core rate
 * of the current device for `precision` (ADVISOR_FP32: 32x32x2 fp32,
 * ADVISOR_BF16: 32x32x16 bf16, ADVISOR_FP8_E4M3: 32x32x64 e4m3, the ops the
 * tile kernels issue). workgroups_per_cu (1..8) workgroups of 4 waves per
 * compute unit each run `iters` (1..2^24) rounds of 8 independent ops on
 * register operands; the timed launch follows a short warm-up one on
 * `stream`. *tflops_out receives dense TFLOP/s. Allocates a small buffer,
 * synchronizes the stream, EINVAL on bad arguments.
 */
int advisor_mfma_peak(int precision, int64_t iters, int workgroups_per_cu, double *tflops_out,
                      void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ADVISOR_H */
