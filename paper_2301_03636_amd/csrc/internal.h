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
    bool wt_valid = false;     // transposed packs (backward) match the master weights
};
