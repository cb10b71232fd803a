// Internal declarations of libadvisor (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/advisor.h"

struct advisor_model;

namespace adv {

constexpr int NFEAT = ADVISOR_NFEAT;
constexpr int KD = ADVISOR_KD_COLS;
constexpr int VD = ADVISOR_VD_COLS;
constexpr int MAX_LAYERS = ADVISOR_MAX_LAYERS;

// Error reporting: a thread-local message plus the status code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
void clear_error();

#define ADV_HIP(call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::adv::hip_fail(e_, #call); \
    } while (0)

#define ADV_LAUNCHED(what)                                  \
    do {                                                    \
        hipError_t e_ = hipGetLastError();                  \
        if (e_ != hipSuccess) return ::adv::hip_fail(e_, what); \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Number of compute units of the current device (cached per device).
int device_cus();

// Training workspace release (train.hip).
void free_train_ws(advisor_model *m);
void free_refine_ws(advisor_model *m);

// One-time launch set-up (dynamic LDS limits, occupancy) of every kernel a
// model of this precision and tile width uses, so that later calls can be
// captured into a graph (mlp.hip, train.hip).
int prepare_model_kernels(int precision, int tile_w);
int prepare_train_kernels(int precision, int tile_w);

// True while `s` is being captured into a graph.
bool stream_capturing(hipStream_t s);

// Whether the ranking calls check their offsets first (select.hip).
bool debug_offsets(hipStream_t s);
// segmented top-N on predictions (arguments checked by the caller)
int launch_topn_preds(const float *pred, const int64_t *offsets, int64_t n_k, int64_t n_v, int N,
                      int64_t *idx_out, float *val_out, hipStream_t s);

// advisor_rank without clearing the error text; the opt-in offsets check
// (which allocates) runs only when may_check_offsets is set (mlp.hip).
int rank_core(const advisor_model *model, const int64_t *kdesc, const int64_t *vdesc,
              const int64_t *offsets, int64_t n_kernels, int64_t n_variants, int64_t *best_out,
              float *pred_out, hipStream_t s, bool may_check_offsets);

// Multi-stage ranking (refine.hip): argument checks, workspace layout and
// the stages on a given workspace.
constexpr int CS_MAX_STAGES = ADVISOR_MAX_STAGES;
constexpr int CS_MAX_K = 32;
// Byte offsets of a cascade's buffers inside its workspace (each part
// 256-byte aligned). Stage s < n_stages - 1 hands on keep[s] candidates per
// kernel: their variant indices (ascending, -1 padded), their descriptor
// rows (kernel id k, or -1 for padding, which makes the row ineligible) and
// the segment offsets k * keep[s] of that compact workload; a middle stage
// also writes its predictions of the previous compact workload.
struct CascadeLayout {
    size_t pred = 0;                    // float [n_v] first-stage predictions (caller gave none)
    size_t cand[CS_MAX_STAGES] = {};    // int64 [n_k * keep_s]
    size_t vd[CS_MAX_STAGES] = {};      // int64 [n_k * keep_s][8]
    size_t off[CS_MAX_STAGES] = {};     // int64 [n_k + 1]
    size_t cpred[CS_MAX_STAGES] = {};   // float [n_k * keep_s] (stages with a successor)
    size_t best = 0;                    // int64 [n_k] winners inside the last compact workload
    size_t total = 0;
};

CascadeLayout cascade_layout(int64_t n_v, int64_t n_k, const int *keep, int n_stages,
                             bool own_pred);
int cascade_check(const advisor_model *const *models, const int *keep, int n_stages,
                  const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                  int64_t n_kernels, int64_t n_variants, const int64_t *best_out);
int cascade_run(const advisor_model *const *models, const int *keep, int n_stages,
                const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets, int64_t n_k,
                int64_t n_v, int64_t *best_out, float *pred_out, unsigned char *ws, hipStream_t s,
                bool may_check_offsets);

// Whether tile shape V is built for this precision and width (mlp.hip).
bool tile_shape_exists(int precision, int W, int V);

// Tile shape recorded by the autotuner for a model of this shape, else 0.
int tuned_variant(const advisor_model *m);

// Kernel-side view of a model's packed parameters.
struct NetView {
    const void *w[MAX_LAYERS];      // packed hidden-layer weights (fragment-major)
    const float *b[MAX_LAYERS];     // hidden-layer biases, zero-padded to the tile width
    const float *head_w;            // output-layer weights, zero-padded
    const float *head_b;            // output-layer bias [1]
    const double *mu;               // Z-score mean [32]
    const double *sigma;            // Z-score deviation [32]
    float qscale[MAX_LAYERS];       // fp8: product of weight and input scales per layer
    float qinv[MAX_LAYERS];         // fp8: 1 / scale of each layer's output activations
    int n_hidden;                   // number of hidden layers (>= 1)
};

}  // namespace adv

struct advisor_model {
    int device = 0;
    int n_widths = 0;
    int widths[ADVISOR_MAX_LAYERS + 1] = {0};
    int precision = 0;
    int tile_w = 0;           // hidden width every layer is padded to (kernel instance)
    int n_hidden = 0;
    int64_t n_params = 0;
    int64_t layer_off[ADVISOR_MAX_LAYERS + 1] = {0};  // offsets of W_l in the master vector
    float *master = nullptr;  // fp32 master parameters [n_params]
    float *adam_m = nullptr;
    float *adam_v = nullptr;
    int64_t *d_step = nullptr;  // Adam step counter, on the device so a captured step replays
    double *mu = nullptr;     // [32]
    double *sigma = nullptr;  // [32]
    void *wpack[ADVISOR_MAX_LAYERS] = {nullptr};
    size_t wpack_bytes[ADVISOR_MAX_LAYERS] = {0};
    float *bias = nullptr;    // [n_hidden, tile_w]
    float *head = nullptr;    // [tile_w + 1]: head weights then head bias
    int64_t *d_layer_off = nullptr;  // device copy of layer_off
    int *d_widths = nullptr;         // device copy of widths
    float wscale[ADVISOR_MAX_LAYERS] = {0};  // fp8: per-tensor weight scale amax/448
    float ascale[ADVISOR_MAX_LAYERS] = {0};  // fp8: scale of each layer's input activations
    float qscale[ADVISOR_MAX_LAYERS] = {0};  // fp8: wscale * ascale (dequantization)
    float qinv[ADVISOR_MAX_LAYERS] = {0};    // fp8: 1 / ascale of the next layer
    bool fp8_calibrated = false;
    void *train_ws = nullptr;  // training workspace (train.hip), grown on demand
    void *refine_ws = nullptr; // refined-ranking workspace (refine.hip), grown on demand
    int tile_variant = 0;      // tile shape used by rank/predict (autotuned)
    // host copies of the Z-score statistics when they were last set from
    // host values (advisor_model_set_params, or the defaults 0 and 1);
    // h_stats is false after advisor_model_set_zscore (device values)
    double h_mu[ADVISOR_NFEAT] = {0};
    double h_sigma[ADVISOR_NFEAT] = {0};
    bool h_stats = false;
    bool wt_valid = false;     // transposed packs (backward) match the master weights
};
