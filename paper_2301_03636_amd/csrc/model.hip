// Model object of libadvisor: creation, parameter upload and packing into
// the matrix-core layouts, Z-score statistics, Adam state, error text.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "mlp_tile.h"

namespace adv {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? ADVISOR_ENOMEM : ADVISOR_EHIP;
}

void clear_error() { g_last_error.clear(); }

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}

int device_cus()
{
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// Elements of layer l's packed weights: [tile_w rows] x [Kp inputs], where
// Kp = 32 for the first layer and tile_w for the others.
static int64_t packed_elems(const advisor_model *m, int l)
{
    const int64_t kp = l == 0 ? NFEAT : m->tile_w;
    return (int64_t)m->tile_w * kp;
}

static int layer_prec(const advisor_model *m, int l)
{
    if (m->precision == PREC_FP32) return PREC_FP32;
    if (m->precision == PREC_BF16) return PREC_BF16;
    if (m->precision == PREC_X3) return PREC_X3;
    return l == 0 ? PREC_BF16 : PREC_FP8;
}

static size_t prec_bytes(int p)
{
    return (p == PREC_FP32 || p == PREC_X3) ? 4 : (p == PREC_BF16 ? 2 : 1);
}

// Scatter one layer's fp32 master weights (zero-padded to tile_w x Kp) into
// the fragment-major packed layout, converted to the layer's precision
// (fp8: divided by the per-tensor weight scale first; bf16x3: the bf16
// rounding of the weight and of its remainder, in their chunk places).
template <int P>
__global__ void pack_layer_kernel(const float *__restrict__ w, int out, int in, int tile_w,
                                  int kp, float inv_scale, void *__restrict__ dst)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)tile_w * kp) return;
    const int n = (int)(idx / kp), k = (int)(idx % kp);
    const float v = (n < out && k < in) ? w[(int64_t)n * in + k] : 0.0f;
    const int64_t at = pack_index<P>(n, k, kp);
    if constexpr (P == PREC_FP32) {
        reinterpret_cast<float *>(dst)[at] = v;
    } else if constexpr (P == PREC_BF16) {
        reinterpret_cast<__bf16 *>(dst)[at] = (__bf16)v;
    } else if constexpr (P == PREC_X3) {
        unsigned char *e = reinterpret_cast<unsigned char *>(dst) + x3_off(at);
        const __bf16 h = (__bf16)v;
        *reinterpret_cast<__bf16 *>(e) = h;
        *reinterpret_cast<__bf16 *>(e + 16) = (__bf16)(v - (float)h);
    } else {
        reinterpret_cast<uint8_t *>(dst)[at] = (uint8_t)f32_to_e4m3(v * inv_scale);
    }
}

// Biases of the hidden layers and the output layer, zero-padded to tile_w.
__global__ void pack_bias_kernel(const float *__restrict__ master, const int64_t *__restrict__ offs,
                                 const int *__restrict__ widths, int n_hidden, int tile_w,
                                 float *__restrict__ bias, float *__restrict__ head)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (n_hidden + 1) * tile_w + 1) return;
    if (i < n_hidden * tile_w) {
        const int l = i / tile_w, n = i % tile_w;
        const int in = widths[l], out = widths[l + 1];
        bias[i] = n < out ? master[offs[l] + (int64_t)out * in + n] : 0.0f;
    } else {
        const int j = i - n_hidden * tile_w;          // head weights then head bias
        const int in = widths[n_hidden];
        const float *hw = master + offs[n_hidden];
        head[j] = j < tile_w ? (j < in ? hw[j] : 0.0f) : hw[in];
    }
}

// Rebuild the packed compute copies from the fp32 master parameters.
int repack(advisor_model *m, hipStream_t s)
{
    for (int l = 0; l < m->n_hidden; ++l) {
        const int p = layer_prec(m, l);
        const int64_t ne = packed_elems(m, l);
        const int kp = l == 0 ? NFEAT : m->tile_w;
        const float *w = m->master + m->layer_off[l];
        const float inv = p == PREC_FP8 ? 1.0f / m->wscale[l] : 1.0f;
        const unsigned blocks = (unsigned)((ne + 255) / 256);
        if (p == PREC_FP32)
            hipLaunchKernelGGL(pack_layer_kernel<PREC_FP32>, dim3(blocks), dim3(256), 0, s, w,
                               m->widths[l + 1], m->widths[l], m->tile_w, kp, inv, m->wpack[l]);
        else if (p == PREC_BF16)
            hipLaunchKernelGGL(pack_layer_kernel<PREC_BF16>, dim3(blocks), dim3(256), 0, s, w,
                               m->widths[l + 1], m->widths[l], m->tile_w, kp, inv, m->wpack[l]);
        else if (p == PREC_X3)
            hipLaunchKernelGGL(pack_layer_kernel<PREC_X3>, dim3(blocks), dim3(256), 0, s, w,
                               m->widths[l + 1], m->widths[l], m->tile_w, kp, inv, m->wpack[l]);
        else
            hipLaunchKernelGGL(pack_layer_kernel<PREC_FP8>, dim3(blocks), dim3(256), 0, s, w,
                               m->widths[l + 1], m->widths[l], m->tile_w, kp, inv, m->wpack[l]);
        ADV_LAUNCHED("pack_layer_kernel");
    }
    const int nb = (m->n_hidden + 1) * m->tile_w + 1;
    hipLaunchKernelGGL(pack_bias_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, m->master,
                       m->d_layer_off, m->d_widths, m->n_hidden, m->tile_w, m->bias, m->head);
    ADV_LAUNCHED("pack_bias_kernel");
    return ADVISOR_OK;
}

}  // namespace adv

using namespace adv;

extern "C" const char *advisor_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *advisor_version(void) { return "libadvisor 0.1 gfx950"; }

extern "C" void advisor_model_destroy(advisor_model *m)
{
    if (!m) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    free_train_ws(m);
    free_refine_ws(m);
    void *ptrs[] = {m->master, m->adam_m, m->adam_v, m->mu, m->sigma, m->bias, m->head,
                    m->d_layer_off, m->d_widths, m->d_step};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < ADVISOR_MAX_LAYERS; ++l)
        if (m->wpack[l]) (void)hipFree(m->wpack[l]);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete m;
}

extern "C" int advisor_model_create(const int32_t *widths, int n_widths, int precision,
                                    advisor_model **out)
{
    clear_error();
    if (!out) return fail(ADVISOR_EINVAL, "advisor_model_create: out is null");
    *out = nullptr;
    if (!widths) return fail(ADVISOR_EINVAL, "advisor_model_create: widths is null");
    if (precision != PREC_FP32 && precision != PREC_BF16 && precision != PREC_FP8 &&
        precision != PREC_X3)
        return fail(ADVISOR_EINVAL, "unknown precision");
    if (n_widths < 3 || n_widths > ADVISOR_MAX_LAYERS + 1)
        return fail(ADVISOR_ESHAPE, "need 32, 1 to 8 hidden widths, then 1");
    if (widths[0] != NFEAT || widths[n_widths - 1] != 1)
        return fail(ADVISOR_ESHAPE, "first width must be 32 and last width 1");
    int wmax = 0;
    for (int i = 1; i + 1 < n_widths; ++i) {
        if (widths[i] < 1 || widths[i] > ADVISOR_MAX_WIDTH)
            return fail(ADVISOR_ESHAPE, "hidden widths must be in 1..1024");
        wmax = widths[i] > wmax ? widths[i] : wmax;
    }
    int tw = 64;
    while (tw < wmax) tw *= 2;
    advisor_model *m = new (std::nothrow) advisor_model();
    if (!m) return fail(ADVISOR_ENOMEM, "host allocation");
    int rc = ADVISOR_OK;
    auto alloc = [&](void **p, size_t bytes) {
        if (rc) return;
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) rc = hip_fail(e, "hipMalloc");
        else if ((e = hipMemset(*p, 0, bytes)) != hipSuccess) rc = hip_fail(e, "hipMemset");
    };
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return fail(ADVISOR_EHIP, "hipGetDevice failed");
    }
    m->n_widths = n_widths;
    for (int i = 0; i < n_widths; ++i) m->widths[i] = widths[i];
    m->precision = precision;
    m->tile_w = tw;
    m->n_hidden = n_widths - 2;
    int64_t off = 0;
    for (int l = 0; l + 1 < n_widths; ++l) {
        m->layer_off[l] = off;
        off += (int64_t)widths[l + 1] * widths[l] + widths[l + 1];
    }
    m->layer_off[n_widths - 1] = off;
    m->n_params = off;
    alloc((void **)&m->master, sizeof(float) * off);
    alloc((void **)&m->adam_m, sizeof(float) * off);
    alloc((void **)&m->adam_v, sizeof(float) * off);
    alloc((void **)&m->d_step, sizeof(int64_t));
    alloc((void **)&m->mu, sizeof(double) * NFEAT);
    alloc((void **)&m->sigma, sizeof(double) * NFEAT);
    alloc((void **)&m->bias, sizeof(float) * m->n_hidden * tw);
    alloc((void **)&m->head, sizeof(float) * (tw + 1));
    alloc((void **)&m->d_layer_off, sizeof(int64_t) * (ADVISOR_MAX_LAYERS + 1));
    alloc((void **)&m->d_widths, sizeof(int) * (ADVISOR_MAX_LAYERS + 1));
    for (int l = 0; l < m->n_hidden; ++l) {
        m->wpack_bytes[l] = (size_t)packed_elems(m, l) * prec_bytes(layer_prec(m, l));
        alloc(&m->wpack[l], m->wpack_bytes[l]);
    }
    if (!rc) {
        std::vector<double> one(NFEAT, 1.0);
        hipError_t e = hipMemcpy(m->sigma, one.data(), sizeof(double) * NFEAT, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(m->d_layer_off, m->layer_off, sizeof(int64_t) * (ADVISOR_MAX_LAYERS + 1),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(m->d_widths, m->widths, sizeof(int) * (ADVISOR_MAX_LAYERS + 1),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy");
    }
    for (int j = 0; j < NFEAT; ++j) {
        m->h_mu[j] = 0.0;
        m->h_sigma[j] = 1.0;
    }
    m->h_stats = true;
    for (int l = 0; l < ADVISOR_MAX_LAYERS; ++l) {
        m->qscale[l] = 1.0f;
        m->qinv[l] = 1.0f;
        m->wscale[l] = 1.0f;
        m->ascale[l] = 1.0f;
    }
    if (!rc) rc = prepare_model_kernels(precision, tw);
    if (!rc) m->tile_variant = tuned_variant(m);
    if (!rc && (precision == PREC_FP32 || precision == PREC_BF16))
        rc = prepare_train_kernels(precision, tw);
    if (rc) {
        advisor_model_destroy(m);
        return rc;
    }
    *out = m;
    return ADVISOR_OK;
}

extern "C" int64_t advisor_model_param_count(const advisor_model *m) { return m ? m->n_params : -1; }

extern "C" int advisor_model_set_params(advisor_model *m, const float *w_master, const double *mu,
                                        const double *sigma)
{
    clear_error();
    if (!m || !w_master || !mu || !sigma) return fail(ADVISOR_EINVAL, "set_params: null pointer");
    for (int j = 0; j < NFEAT; ++j)
        if (!(sigma[j] > 0.0)) return fail(ADVISOR_EINVAL, "sigma must be positive");
    int prev = -1;
    ADV_HIP(hipGetDevice(&prev));
    ADV_HIP(hipSetDevice(m->device));
    // per-tensor fp8 weight scales (amax / 448) from the host copy
    for (int l = 0; l < m->n_hidden; ++l) {
        float amax = 0.0f;
        const int64_t nw = (int64_t)m->widths[l + 1] * m->widths[l];
        for (int64_t i = 0; i < nw; ++i) amax = fmaxf(amax, fabsf(w_master[m->layer_off[l] + i]));
        m->wscale[l] = amax > 0.0f ? amax / 448.0f : 1.0f;
    }
    hipError_t e = hipMemcpy(m->master, w_master, sizeof(float) * m->n_params, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->mu, mu, sizeof(double) * NFEAT, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->sigma, sigma, sizeof(double) * NFEAT, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->adam_m, 0, sizeof(float) * m->n_params);
    if (e == hipSuccess) e = hipMemset(m->adam_v, 0, sizeof(float) * m->n_params);
    if (e == hipSuccess) e = hipMemset(m->d_step, 0, sizeof(int64_t));
    if (e != hipSuccess) {
        (void)hipSetDevice(prev);
        return hip_fail(e, "set_params copy");
    }
    for (int j = 0; j < NFEAT; ++j) {
        m->h_mu[j] = mu[j];
        m->h_sigma[j] = sigma[j];
    }
    m->h_stats = true;
    m->fp8_calibrated = false;
    m->wt_valid = false;
    int rc = repack(m, nullptr);
    if (!rc) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "repack");
    }
    (void)hipSetDevice(prev);
    return rc;
}

extern "C" int advisor_model_get_params(const advisor_model *m, float *w_master, double *mu,
                                        double *sigma)
{
    clear_error();
    if (!m || !w_master) return fail(ADVISOR_EINVAL, "get_params: null pointer");
    ADV_HIP(hipDeviceSynchronize());
    ADV_HIP(hipMemcpy(w_master, m->master, sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    if (mu) ADV_HIP(hipMemcpy(mu, m->mu, sizeof(double) * NFEAT, hipMemcpyDeviceToHost));
    if (sigma) ADV_HIP(hipMemcpy(sigma, m->sigma, sizeof(double) * NFEAT, hipMemcpyDeviceToHost));
    return ADVISOR_OK;
}

extern "C" int advisor_model_set_zscore(advisor_model *m, const double *mu, const double *sigma,
                                        void *stream)
{
    clear_error();
    if (!m || !mu || !sigma) return fail(ADVISOR_EINVAL, "set_zscore: null pointer");
    hipStream_t s = as_stream(stream);
    m->h_stats = false;  // device values: no host copy to compare
    ADV_HIP(hipMemcpyAsync(m->mu, mu, sizeof(double) * NFEAT, hipMemcpyDeviceToDevice, s));
    ADV_HIP(hipMemcpyAsync(m->sigma, sigma, sizeof(double) * NFEAT, hipMemcpyDeviceToDevice, s));
    return ADVISOR_OK;
}

extern "C" int advisor_model_get_adam(const advisor_model *m, float *am, float *av, int64_t *step)
{
    clear_error();
    if (!m) return fail(ADVISOR_EINVAL, "get_adam: null model");
    ADV_HIP(hipDeviceSynchronize());
    if (am) ADV_HIP(hipMemcpy(am, m->adam_m, sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    if (av) ADV_HIP(hipMemcpy(av, m->adam_v, sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    if (step) ADV_HIP(hipMemcpy(step, m->d_step, sizeof(int64_t), hipMemcpyDeviceToHost));
    return ADVISOR_OK;
}

extern "C" int advisor_model_set_adam(advisor_model *m, const float *am, const float *av,
                                      int64_t step)
{
    clear_error();
    if (!m) return fail(ADVISOR_EINVAL, "set_adam: null model");
    if (step < 0) return fail(ADVISOR_EINVAL, "set_adam: negative step");
    ADV_HIP(hipDeviceSynchronize());
    if (am) ADV_HIP(hipMemcpy(m->adam_m, am, sizeof(float) * m->n_params, hipMemcpyHostToDevice));
    if (av) ADV_HIP(hipMemcpy(m->adam_v, av, sizeof(float) * m->n_params, hipMemcpyHostToDevice));
    ADV_HIP(hipMemcpy(m->d_step, &step, sizeof(int64_t), hipMemcpyHostToDevice));
    return ADVISOR_OK;
}
