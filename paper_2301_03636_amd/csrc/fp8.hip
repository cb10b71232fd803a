// FP8 (OCP e4m3) inference support: static per-tensor activation scales
// calibrated on a sample of features. Weights are quantized per tensor with
// scale amax(|W_l|) / 448 when parameters are loaded; here each hidden
// layer's input activations get scale amax(h) / 448 from a bf16 forward pass
// over the calibration sample, so no scale depends on the tile a row lands in.
#include <math.h>
#include <string.h>

#include <vector>

#include "mlp_tile.h"

namespace adv {

int repack(advisor_model *m, hipStream_t s);                                  // model.hip
int launch_train_forward(const advisor_model *m, const TileArgs &a, hipStream_t s);  // mlp.hip

__global__ void fill_u32_kernel(uint32_t *p, int n, uint32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// amax of a non-negative bf16 array (ReLU outputs): the float bits of
// non-negative values order like unsigned integers, so an atomic max on them
// is exact and independent of the order of the updates.
__global__ void amax_bf16_kernel(const __bf16 *__restrict__ v, int64_t n, uint32_t *__restrict__ out)
{
    float mx = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = fabsf((float)v[i]);
        mx = x > mx ? x : mx;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(mx));
}

}  // namespace adv

using namespace adv;

extern "C" int advisor_model_calibrate_fp8(advisor_model *m, const int64_t *feat, int64_t n,
                                           void *stream)
{
    clear_error();
    if (!m || !feat) return fail(ADVISOR_EINVAL, "calibrate_fp8: null pointer");
    if (m->precision != PREC_FP8) return fail(ADVISOR_EINVAL, "calibrate_fp8 needs an fp8 model");
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    hipStream_t s = as_stream(stream);
    // bf16 shadow of the model
    advisor_model *b = nullptr;
    int rc = advisor_model_create(m->widths, m->n_widths, PREC_BF16, &b);
    if (rc) return rc;
    hipError_t e0 = hipDeviceSynchronize();  // creation initialized b on the null stream
    if (e0 != hipSuccess) {
        advisor_model_destroy(b);
        return hip_fail(e0, "calibrate_fp8 set-up");
    }
    void *saved = nullptr;
    float *y = nullptr;
    uint32_t *amax = nullptr;
    std::vector<uint32_t> host(ADVISOR_MAX_LAYERS, 0);
    const int64_t ld = ((n + 255) / 256) * 256;
    const size_t eb = 2;
    const size_t saved_bytes = (size_t)(NFEAT + (int64_t)b->n_hidden * b->tile_w) * ld * eb;
    hipError_t e = hipMemcpyAsync(b->master, m->master, sizeof(float) * m->n_params,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->mu, m->mu, sizeof(double) * NFEAT, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->sigma, m->sigma, sizeof(double) * NFEAT, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMalloc(&saved, saved_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&y, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&amax, sizeof(uint32_t) * ADVISOR_MAX_LAYERS);
    if (e != hipSuccess) rc = hip_fail(e, "calibrate_fp8 set-up");
    if (!rc) rc = repack(b, s);
    if (!rc) {
        TileArgs a{};
        a.feat = feat;
        a.n_rows = n;
        a.pred = y;
        a.save_ld = ld;
        a.save_x = saved;
        a.save_h = reinterpret_cast<unsigned char *>(saved) + (size_t)NFEAT * ld * eb;
        rc = launch_train_forward(b, a, s);
    }
    if (!rc) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, amax, ADVISOR_MAX_LAYERS, 0u);
        for (int l = 0; l < m->n_hidden; ++l) {
            const __bf16 *h = reinterpret_cast<const __bf16 *>(
                reinterpret_cast<unsigned char *>(saved) + (size_t)NFEAT * ld * eb +
                (size_t)l * b->tile_w * ld * eb);
            hipLaunchKernelGGL(amax_bf16_kernel, dim3(1024), dim3(256), 0, s, h,
                               (int64_t)b->tile_w * ld, amax + l);
        }
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(host.data(), amax, sizeof(uint32_t) * ADVISOR_MAX_LAYERS,
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "calibrate_fp8 reduction");
    }
    if (!rc) {
        // layer l >= 1 reads h_{l-1}: its input scale; layer l-1 writes with 1/scale
        for (int l = 0; l < ADVISOR_MAX_LAYERS; ++l) {
            m->ascale[l] = 1.0f;
            m->qscale[l] = 1.0f;
            m->qinv[l] = 1.0f;
        }
        for (int l = 1; l < m->n_hidden; ++l) {
            float am;
            uint32_t bits = host[l - 1];
            memcpy(&am, &bits, sizeof(am));
            m->ascale[l] = (am > 0.0f && isfinite(am)) ? am / 448.0f : 1.0f;
            m->qscale[l] = m->wscale[l] * m->ascale[l];
            m->qinv[l - 1] = 1.0f / m->ascale[l];
        }
        m->fp8_calibrated = true;
    }
    if (saved) (void)hipFree(saved);
    if (y) (void)hipFree(y);
    if (amax) (void)hipFree(amax);
    advisor_model_destroy(b);
    return rc;
}

extern "C" int advisor_model_get_fp8_scales(const advisor_model *m, float *wscale, float *ascale)
{
    clear_error();
    if (!m || !wscale || !ascale) return fail(ADVISOR_EINVAL, "get_fp8_scales: null pointer");
    for (int l = 0; l < m->n_hidden; ++l) {
        wscale[l] = m->wscale[l];
        ascale[l] = m->ascale[l];
    }
    return ADVISOR_OK;
}
