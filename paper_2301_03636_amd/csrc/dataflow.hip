// Data analysis (section 4.1.2): every variable a kernel touches gets a map
// class from what happens to it before, during and after the kernel, and each
// kernel gets the bytes its enter-data and exit-data directives move, beside
// the bytes of mapping every variable to and from the GPU. Integer work on a
// few bytes per variable, bound by memory: one thread per kernel.
#include <algorithm>

#include "internal.h"

namespace adv {

namespace {

constexpr int DF_THREADS = 256;

// class of one variable from its access bits (the codes of ADVISOR_MAP_*)
__device__ __forceinline__ int map_class(unsigned bits)
{
    const bool before = bits & ADVISOR_ACC_BEFORE, rd = bits & ADVISOR_ACC_READ;
    const bool wr = bits & ADVISOR_ACC_WRITE, after = bits & ADVISOR_ACC_AFTER;
    if (bits & ADVISOR_ACC_LOCAL) return ADVISOR_MAP_PRIVATE;
    if (!rd && !wr) return ADVISOR_MAP_NONE;
    if (!wr) return ADVISOR_MAP_TO;
    if (after) return before ? ADVISOR_MAP_TOFROM : ADVISOR_MAP_FROM;
    return (before && rd) ? ADVISOR_MAP_TO : ADVISOR_MAP_ALLOC;
}

// One thread per kernel: a kernel has a handful of variables (the paper's
// kernels map a few arrays), so each thread walks its own segment; adjacent
// threads walk adjacent segments, which keeps the loads of a wave within a
// few cache lines.
__global__ __launch_bounds__(DF_THREADS) void classify_kernel(
    const uint8_t *__restrict__ access, const int64_t *__restrict__ nbytes,
    const int64_t *__restrict__ var_off, int64_t n_k, int64_t n_vars, uint8_t *__restrict__ cls,
    int64_t *__restrict__ enter, int64_t *__restrict__ exit_, int64_t *__restrict__ naive)
{
    const int64_t stride = (int64_t)gridDim.x * DF_THREADS;
    for (int64_t k = (int64_t)blockIdx.x * DF_THREADS + threadIdx.x; k < n_k; k += stride) {
        const int64_t lo = max((int64_t)0, min(var_off[k], n_vars));
        const int64_t hi = max(lo, min(var_off[k + 1], n_vars));
        int64_t e = 0, x = 0, nv = 0;
        for (int64_t i = lo; i < hi; ++i) {
            const int c = map_class(access[i]);
            if (cls) cls[i] = (uint8_t)c;
            const int64_t b = nbytes[i];
            if (c == ADVISOR_MAP_TO || c == ADVISOR_MAP_TOFROM) e += b;
            if (c == ADVISOR_MAP_FROM || c == ADVISOR_MAP_TOFROM) x += b;
            if (c <= ADVISOR_MAP_TOFROM) nv += 2 * b;
        }
        if (enter) enter[k] = e;
        if (exit_) exit_[k] = x;
        if (naive) naive[k] = nv;
    }
}

}  // namespace

}  // namespace adv

using namespace adv;

extern "C" int advisor_classify_maps(const uint8_t *access, const int64_t *nbytes,
                                     const int64_t *var_offsets, int64_t n_kernels,
                                     int64_t n_vars, uint8_t *class_out, int64_t *enter_bytes,
                                     int64_t *exit_bytes, int64_t *naive_bytes, void *stream)
{
    clear_error();
    if (n_kernels < 0 || n_vars < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_kernels >= (int64_t)1 << 31) return fail(ADVISOR_ESHAPE, "n_kernels must be < 2^31");
    if (n_kernels == 0) return ADVISOR_OK;
    if (!var_offsets || (n_vars > 0 && (!access || !nbytes)))
        return fail(ADVISOR_EINVAL, "advisor_classify_maps: null pointer");
    hipStream_t s = as_stream(stream);
    const int64_t blocks = std::min<int64_t>((n_kernels + DF_THREADS - 1) / DF_THREADS, 1 << 20);
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)blocks), dim3(DF_THREADS), 0, s, access,
                       nbytes, var_offsets, n_kernels, n_vars, class_out, enter_bytes, exit_bytes,
                       naive_bytes);
    ADV_LAUNCHED("classify_kernel");
    return ADVISOR_OK;
}
