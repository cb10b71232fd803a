// Attainable matrix-core rate of the device, a measurement aid beside the
// published peaks the roofline figures use (not a step of the method). Every
// wave issues a long run of independent matrix-core ops of the same shapes
// the tile kernels use, on register operands with no memory traffic in the
// loop, so the kernel's duration gives the sustained rate under full load,
// with whatever clock the chip holds under it.
#include <algorithm>

#include "mlp_tile.h"

namespace adv {

namespace {

constexpr int PK_THREADS = 256;  // 4 waves: one per SIMD per workgroup
constexpr int PK_CHAINS = 8;     // independent accumulators per wave

template <int P> struct PeakOp;
template <> struct PeakOp<PREC_FP32> {
    using A = float;
    static constexpr double flops = 2.0 * 32 * 32 * 2;
    __device__ static A make(int lane) { return 1.0f + 1e-3f * (float)(lane & 7); }
};
template <> struct PeakOp<PREC_BF16> {
    using A = v8bf;
    static constexpr double flops = 2.0 * 32 * 32 * 16;
    __device__ static A make(int lane)
    {
        A a;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = (__bf16)(0.5f + 0.0625f * (float)((lane + e) & 7));
        return a;
    }
};
template <> struct PeakOp<PREC_FP8> {
    using A = v8i;
    static constexpr double flops = 2.0 * 32 * 32 * 64;
    __device__ static A make(int lane)
    {
        // e4m3 bytes 0x30..0x37: 0.25 .. 0.4375, finite and non-zero
        A a;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned b = 0x30u + (unsigned)((lane + e) & 7);
            a[e] = (int)(b | (b << 8) | (b << 16) | (b << 24));
        }
        return a;
    }
};

template <int P>
__global__ __launch_bounds__(PK_THREADS) void mfma_peak_kernel(int64_t iters, float *__restrict__ out)
{
    using Op = PeakOp<P>;
    const int lane = threadIdx.x & 63;
    const typename Op::A a = Op::make(lane), b = Op::make(lane + 3);
    v16f acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = v16f{0};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) acc[c] = mma(a, b, acc[c]);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[c][r];
    out[(int64_t)blockIdx.x * PK_THREADS + threadIdx.x] = s;
}

}  // namespace

}  // namespace adv

using namespace adv;

extern "C" int advisor_mfma_peak(int precision, int64_t iters, int workgroups_per_cu,
                                 double *tflops_out, void *stream)
{
    clear_error();
    if (!tflops_out) return fail(ADVISOR_EINVAL, "tflops_out is null");
    if (precision != ADVISOR_FP32 && precision != ADVISOR_BF16 && precision != ADVISOR_FP8_E4M3)
        return fail(ADVISOR_EINVAL, "unknown precision");
    if (iters < 1 || iters > (int64_t)1 << 24)
        return fail(ADVISOR_EINVAL, "iters must be in [1, 2^24]");
    if (workgroups_per_cu < 1 || workgroups_per_cu > 8)
        return fail(ADVISOR_EINVAL, "workgroups_per_cu must be in [1, 8]");
    hipStream_t s = as_stream(stream);
    const int grid = device_cus() * workgroups_per_cu;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ADVISOR_OK;
    auto check = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == ADVISOR_OK) rc = hip_fail(e, what);
        return rc == ADVISOR_OK;
    };
    if (check(hipMalloc((void **)&out, sizeof(float) * (size_t)grid * PK_THREADS), "hipMalloc") &&
        check(hipEventCreate(&e0), "hipEventCreate") && check(hipEventCreate(&e1), "hipEventCreate")) {
        auto launch = [&](int64_t n) {
            if (precision == ADVISOR_FP32)
                hipLaunchKernelGGL(mfma_peak_kernel<PREC_FP32>, dim3(grid), dim3(PK_THREADS), 0, s, n, out);
            else if (precision == ADVISOR_BF16)
                hipLaunchKernelGGL(mfma_peak_kernel<PREC_BF16>, dim3(grid), dim3(PK_THREADS), 0, s, n, out);
            else
                hipLaunchKernelGGL(mfma_peak_kernel<PREC_FP8>, dim3(grid), dim3(PK_THREADS), 0, s, n, out);
            return check(hipGetLastError(), "mfma_peak_kernel");
        };
        // a short warm-up launch, then the timed one
        if (launch(std::max<int64_t>(1, iters / 16)) && check(hipEventRecord(e0, s), "hipEventRecord") &&
            launch(iters) && check(hipEventRecord(e1, s), "hipEventRecord") &&
            check(hipEventSynchronize(e1), "hipEventSynchronize")) {
            float ms = 0.0f;
            if (check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) {
                double flops = 0.0;
                if (precision == ADVISOR_FP32) flops = PeakOp<PREC_FP32>::flops;
                else if (precision == ADVISOR_BF16) flops = PeakOp<PREC_BF16>::flops;
                else flops = PeakOp<PREC_FP8>::flops;
                const double total = flops * PK_CHAINS * (double)iters * (double)grid * (PK_THREADS / 64);
                *tflops_out = total / ((double)ms * 1e-3) / 1e12;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    return rc;
}
