// Multi-stage ranking for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the stages of advisor_rank_cascade on a workspace that is a
// file-scope device array of fixed size instead of a model-owned arena.
//
// The array lives in this file's code object, so each GPU that loads it holds
// its own copy until the process ends. Host code never passes the array's
// name to a kernel or a copy (on the host that name is only a stand-in for
// the symbol): the device address of the calling GPU's copy is looked up
// once per device with hipGetSymbolAddress and kept.
#include <mutex>

#include "internal.h"

namespace adv {
namespace {

constexpr int NA_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[ADVISOR_NOALLOC_SCRATCH_BYTES];

std::mutex g_na_mu;
unsigned char *g_na_ptr[NA_MAX_DEVICES] = {};

// The device address of the current GPU's copy of `scratch` (looked up on
// the first call on each device, with that device current).
int scratch_for_device(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= NA_MAX_DEVICES) return fail(ADVISOR_EUNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(ADVISOR_EHIP, "hipGetSymbolAddress(scratch) returned null");
        g_na_ptr[dev] = reinterpret_cast<unsigned char *>(p);
    }
    *out = g_na_ptr[dev];
    return ADVISOR_OK;
}

}  // namespace
}  // namespace adv

using namespace adv;

extern "C" int advisor_rank_cascade_noalloc(advisor_model *const *models, const int *keep,
                                            int n_stages, const int64_t *kdesc,
                                            const int64_t *vdesc, const int64_t *offsets,
                                            int64_t n_kernels, int64_t n_variants,
                                            int64_t *best_out, float *pred_out, void *stream)
{
    clear_error();
    int rc = cascade_check(models, keep, n_stages, kdesc, vdesc, offsets, n_kernels, n_variants,
                           best_out);
    if (rc || n_kernels == 0) return rc;
    int dev = -1;
    ADV_HIP(hipGetDevice(&dev));
    if (models[0]->device != dev)
        return fail(ADVISOR_EINVAL, "advisor_rank_cascade_noalloc: the models live on another device");
    unsigned char *ws = nullptr;
    if (n_stages > 1) {
        const CascadeLayout L = cascade_layout(n_variants, n_kernels, keep, n_stages,
                                               pred_out == nullptr);
        if (L.total > (size_t)ADVISOR_NOALLOC_SCRATCH_BYTES)
            return fail(ADVISOR_ESHAPE,
                        "advisor_rank_cascade_noalloc: the stages need " + std::to_string(L.total) +
                            " bytes of workspace, above the fixed " +
                            std::to_string((size_t)ADVISOR_NOALLOC_SCRATCH_BYTES) +
                            " (fewer kernels or candidates per call, or pass pred_out)");
        rc = scratch_for_device(dev, &ws);
        if (rc) return rc;
    }
    // every workspace buffer is written before it is read (candidate lists,
    // their descriptors and offsets by the gather, the winners' keys by the
    // key-initialization kernel of each stage), so nothing is cleared; the
    // opt-in offsets check is skipped because it allocates
    return cascade_run(models, keep, n_stages, kdesc, vdesc, offsets, n_kernels, n_variants,
                       best_out, pred_out, ws, as_stream(stream), false);
}
