// Captured launch plans: one advisor_rank or advisor_train_step call with
// fixed buffers recorded into a HIP graph and replayed with one launch. The
// kernels are the same as the direct calls; replays give the same bits.
#include "internal.h"

struct advisor_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace adv {

int repack_transposed_now(advisor_model *m, hipStream_t s);  // train.hip
int reserve_train_ws(advisor_model *m, int64_t n);           // train.hip

// Record what `body` enqueues on a private capture stream into a new plan.
template <class F>
static int capture(F body, advisor_plan **out)
{
    *out = nullptr;
    advisor_plan *p = new (std::nothrow) advisor_plan();
    if (!p) return fail(ADVISOR_ENOMEM, "host allocation");
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(ADVISOR_EHIP, "hipGetDevice failed");
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    int rc = ADVISOR_OK;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        rc = hip_fail(e, "hipStreamBeginCapture");
    } else {
        rc = body(cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (!rc && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        p->graph = g;
        if (!rc) {
            e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
        }
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
        advisor_plan_destroy(p);
        return rc;
    }
    *out = p;
    return ADVISOR_OK;
}

}  // namespace adv

using namespace adv;

extern "C" void advisor_plan_destroy(advisor_plan *p)
{
    if (!p) return;
    // the runtime does not defer freeing an executable graph whose launches
    // are still queued or running: wait for the plan's device to go idle first
    if (p->exec) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != p->device) (void)hipSetDevice(p->device);
        (void)hipDeviceSynchronize();
        if (prev >= 0 && prev != p->device) (void)hipSetDevice(prev);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

extern "C" int advisor_rank_plan_create(const advisor_model *model, const int64_t *kdesc,
                                        const int64_t *vdesc, const int64_t *offsets,
                                        int64_t n_kernels, int64_t n_variants, int64_t *best_out,
                                        float *pred_out, advisor_plan **out)
{
    clear_error();
    if (!out) return fail(ADVISOR_EINVAL, "advisor_rank_plan_create: out is null");
    *out = nullptr;
    if (!model) return fail(ADVISOR_EINVAL, "null model");
    return capture(
        [&](hipStream_t cs) {
            return advisor_rank(model, kdesc, vdesc, offsets, n_kernels, n_variants, best_out,
                                pred_out, cs);
        },
        out);
}

extern "C" int advisor_train_plan_create(advisor_model *model, const int64_t *feat, const double *y,
                                         int64_t n, float lr, float beta1, float beta2, float eps,
                                         double *loss_out, double *gnorm_out, advisor_plan **out)
{
    clear_error();
    if (!out) return fail(ADVISOR_EINVAL, "advisor_train_plan_create: out is null");
    *out = nullptr;
    if (!model) return fail(ADVISOR_EINVAL, "null model");
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    // everything that allocates or must run once happens before the capture
    int rc = reserve_train_ws(model, n);
    if (rc) return rc;
    rc = repack_transposed_now(model, nullptr);
    if (rc) return rc;
    ADV_HIP(hipDeviceSynchronize());
    return capture(
        [&](hipStream_t cs) {
            return advisor_train_step(model, feat, y, n, lr, beta1, beta2, eps, loss_out,
                                      gnorm_out, cs);
        },
        out);
}

extern "C" int advisor_train_plan_create_rmsprop(advisor_model *model, const int64_t *feat,
                                                 const double *y, int64_t n, float lr,
                                                 float alpha, float eps, float weight_decay,
                                                 int loss, double *loss_out, double *gnorm_out,
                                                 advisor_plan **out)
{
    clear_error();
    if (!out) return fail(ADVISOR_EINVAL, "advisor_train_plan_create_rmsprop: out is null");
    *out = nullptr;
    if (!model) return fail(ADVISOR_EINVAL, "null model");
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    int rc = reserve_train_ws(model, n);
    if (rc) return rc;
    rc = repack_transposed_now(model, nullptr);
    if (rc) return rc;
    ADV_HIP(hipDeviceSynchronize());
    return capture(
        [&](hipStream_t cs) {
            return advisor_train_step_rmsprop(model, feat, y, n, lr, alpha, eps, weight_decay, loss,
                                              loss_out, gnorm_out, cs);
        },
        out);
}

extern "C" int advisor_train_plan_create_rmsprop_multi(
    advisor_model *const *models, const int64_t *const *feats, const double *const *ys,
    const int64_t *ns, int n_models, float lr, float alpha, float eps, float weight_decay, int loss,
    double *loss_out, double *gnorm_out, advisor_plan **out)
{
    clear_error();
    if (!out) return fail(ADVISOR_EINVAL, "advisor_train_plan_create_rmsprop_multi: out is null");
    *out = nullptr;
    if (n_models < 1 || n_models > 64 || !models || !feats || !ys || !ns)
        return fail(ADVISOR_EINVAL, "need 1 to 64 models with their batches");
    for (int t = 0; t < n_models; ++t) {
        if (!models[t]) return fail(ADVISOR_EINVAL, "null model");
        for (int u = 0; u < t; ++u)
            if (models[u] == models[t]) return fail(ADVISOR_EINVAL, "a model appears twice");
        if (ns[t] < 1 || ns[t] >= ((int64_t)1 << 32))
            return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
        int rc = reserve_train_ws(models[t], ns[t]);
        if (rc) return rc;
        rc = repack_transposed_now(models[t], nullptr);
        if (rc) return rc;
    }
    ADV_HIP(hipDeviceSynchronize());
    // The models' steps are recorded one after another on the capture
    // stream: one branch, like every other plan. (Graphs with one branch per
    // model, forked through events onto their own streams, ran the models
    // concurrently but crashed the host inside hipGraphLaunch under long runs
    // of unsynchronized replays, so that form is not used.)
    return capture(
        [&](hipStream_t cs) -> int {
            for (int t = 0; t < n_models; ++t) {
                int r = advisor_train_step_rmsprop(models[t], feats[t], ys[t], ns[t], lr, alpha, eps,
                                                   weight_decay, loss,
                                                   loss_out ? loss_out + t : nullptr,
                                                   gnorm_out ? gnorm_out + t : nullptr, cs);
                if (r) return r;
            }
            return ADVISOR_OK;
        },
        out);
}

extern "C" int advisor_plan_launch(advisor_plan *p, void *stream)
{
    clear_error();
    if (!p || !p->exec) return fail(ADVISOR_EINVAL, "advisor_plan_launch: null plan");
    int dev = -1;
    ADV_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(ADVISOR_EINVAL, "plan was captured on another device");
    ADV_HIP(hipGraphLaunch(p->exec, as_stream(stream)));
    return ADVISOR_OK;
}
