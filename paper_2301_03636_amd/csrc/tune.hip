// Autotuner of the fused tile kernel's shape: times every tile shape built
// for a model's precision and width on the caller's ranking workload, keeps
// the fastest for that model, and remembers it in a small JSON file keyed by
// (GPU architecture, precision, layer widths) so later models of the same
// shape start from the tuned choice.
#include <stdio.h>
#include <stdlib.h>
#include <sys/stat.h>

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.h"

namespace adv {

constexpr int N_SHAPES = 4;  // tile shapes per (precision, width), see mlp.hip

static std::mutex g_tune_mu;

// $ADVISOR_TUNE_CACHE, else $HOME/.cache/libadvisor/tune.json; an empty
// ADVISOR_TUNE_CACHE turns the cache off.
static std::string cache_path()
{
    const char *e = getenv("ADVISOR_TUNE_CACHE");
    if (e) return std::string(e);
    const char *h = getenv("HOME");
    if (!h || !*h) return std::string();
    return std::string(h) + "/.cache/libadvisor/tune.json";
}

static std::string tune_key(const advisor_model *m)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, m->device) == hipSuccess) arch = prop.gcnArchName;
    static const char *pn[] = {"fp32", "bf16", "fp8"};
    std::ostringstream k;
    k << arch << "|" << pn[m->precision] << "|";
    for (int i = 0; i < m->n_widths; ++i) k << (i ? "," : "") << m->widths[i];
    return k.str();
}

// One entry per line: "key": value,
static std::map<std::string, int> read_cache(const std::string &path)
{
    std::map<std::string, int> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"');
        if (a == std::string::npos) continue;
        const size_t b = line.find('"', a + 1);
        const size_t c = line.find(':', b == std::string::npos ? a : b);
        if (b == std::string::npos || c == std::string::npos) continue;
        out[line.substr(a + 1, b - a - 1)] = atoi(line.c_str() + c + 1);
    }
    return out;
}

static void write_cache(const std::string &path, const std::map<std::string, int> &entries)
{
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        // create the directory chain if needed (best effort)
        const std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') {
                const std::string d = dir.substr(0, i);
                if (!d.empty()) (void)mkdir(d.c_str(), 0755);
            }
    }
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t i = 0;
        for (const auto &kv : entries)
            f << "  \"" << kv.first << "\": " << kv.second << (++i < entries.size() ? "," : "")
              << "\n";
        f << "}\n";
    }
    (void)rename(tmp.c_str(), path.c_str());
}

int tuned_variant(const advisor_model *m)
{
    const std::string path = cache_path();
    if (path.empty()) return 0;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto entries = read_cache(path);
    const auto it = entries.find(tune_key(m));
    if (it == entries.end()) return 0;
    return tile_shape_exists(m->precision, m->tile_w, it->second) ? it->second : 0;
}

}  // namespace adv

using namespace adv;

extern "C" int advisor_model_set_tile_variant(advisor_model *m, int v)
{
    clear_error();
    if (!m) return fail(ADVISOR_EINVAL, "null model");
    if (!tile_shape_exists(m->precision, m->tile_w, v))
        return fail(ADVISOR_EUNSUPPORTED, "no such tile shape for this precision and width");
    m->tile_variant = v;
    return ADVISOR_OK;
}

extern "C" int advisor_model_get_tile_variant(const advisor_model *m)
{
    return m ? m->tile_variant : -1;
}

extern "C" int advisor_autotune(advisor_model *m, const int64_t *kdesc, const int64_t *vdesc,
                                const int64_t *offsets, int64_t n_kernels, int64_t n_variants,
                                int reps, double *times_ms, int max_variants, int *chosen,
                                void *stream)
{
    clear_error();
    if (!m) return fail(ADVISOR_EINVAL, "null model");
    if (reps < 1 || max_variants < 0 || (max_variants > 0 && !times_ms))
        return fail(ADVISOR_EINVAL, "advisor_autotune: bad reps or times buffer");
    if (n_kernels < 1) return fail(ADVISOR_ESHAPE, "advisor_autotune needs at least one kernel");
    hipStream_t s = as_stream(stream);
    int64_t *best = nullptr;
    ADV_HIP(hipMalloc((void **)&best, sizeof(int64_t) * n_kernels));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ADVISOR_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(ADVISOR_EHIP, "hipEventCreate failed");
    const int before = m->tile_variant;
    int pick = -1;
    double pick_ms = 0.0;
    for (int v = 0; v < N_SHAPES && !rc; ++v) {
        double ms = -1.0;
        if (tile_shape_exists(m->precision, m->tile_w, v)) {
            m->tile_variant = v;
            for (int w = 0; w < 2 && !rc; ++w)
                rc = advisor_rank(m, kdesc, vdesc, offsets, n_kernels, n_variants, best, nullptr, s);
            if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fail(ADVISOR_EHIP, "hipEventRecord");
            for (int r = 0; r < reps && !rc; ++r)
                rc = advisor_rank(m, kdesc, vdesc, offsets, n_kernels, n_variants, best, nullptr, s);
            float t = 0.0f;
            if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                rc = fail(ADVISOR_EHIP, "event timing failed");
            if (!rc) {
                ms = t / reps;
                if (pick < 0 || ms < pick_ms) {
                    pick = v;
                    pick_ms = ms;
                }
            }
        }
        if (v < max_variants) times_ms[v] = ms;
    }
    for (int v = N_SHAPES; v < max_variants; ++v) times_ms[v] = -1.0;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(best);
    if (rc || pick < 0) {
        m->tile_variant = before;
        return rc ? rc : fail(ADVISOR_EUNSUPPORTED, "no tile shape ran");
    }
    m->tile_variant = pick;
    if (chosen) *chosen = pick;
    const std::string path = cache_path();
    if (!path.empty()) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto entries = read_cache(path);
        entries[tune_key(m)] = pick;
        write_cache(path, entries);
    }
    return ADVISOR_OK;
}
