// Launch-shape autotuner.  A kernel with several launch shapes (work-group size, occupancy hint,
// work-group order) asks tuned_choice() which one to use for a key (kernel, precision, mode,
// lattice, right-hand sides).  On the first request the shapes are timed on the caller's data
// (one warm-up and three timed launches each, hipEvents on the caller's stream) and the fastest
// is kept for the process; with DIRAC_TUNE_CACHE=<file> the choices are also read from and
// written to a JSON object {"key": shape, ...}.  DIRAC_TUNE=0 disables tuning (shape 0);
// DIRAC_HOP_SHAPE=<n> forces a shape.  No timing happens while the stream is being captured
// into a graph: the cached choice or shape 0 is used.  The shapes of one kernel compute
// identical results, so the choice never changes a result.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.h"

namespace dl {
namespace {

std::mutex g_mu;
std::map<std::string, int> g_cache;
bool g_loaded = false;

const char *cache_path() { return getenv("DIRAC_TUNE_CACHE"); }

void load_cache() {
    if (g_loaded) return;
    g_loaded = true;
    const char *p = cache_path();
    if (!p) return;
    std::ifstream f(p);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    while ((i = t.find('"', i)) != std::string::npos) {
        const size_t j = t.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = t.substr(i + 1, j - i - 1);
        const size_t c = t.find(':', j);
        if (c == std::string::npos) break;
        g_cache[key] = atoi(t.c_str() + c + 1);
        i = t.find_first_of(",}", c);
        if (i == std::string::npos) break;
    }
}

void save_cache() {
    const char *p = cache_path();
    if (!p) return;
    std::ofstream f(p);
    f << "{";
    bool first = true;
    for (auto &kv : g_cache) {
        f << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": " << kv.second;
        first = false;
    }
    f << "\n}\n";
}

}  // namespace

const char *prec_name(dirac_prec pr) {
    return pr == DIRAC_F64 ? "f64" : pr == DIRAC_F32 ? "f32" : pr == DIRAC_F16 ? "f16" : "bf16";
}

int tuned_choice(const char *key, int nshapes, const std::function<void(int)> &launch, hipStream_t s) {
    if (const char *f = getenv("DIRAC_HOP_SHAPE")) {
        const int v = atoi(f);
        return v >= 0 && v < nshapes ? v : 0;
    }
    if (const char *t = getenv("DIRAC_TUNE"))
        if (atoi(t) == 0) return 0;
    std::string k = std::string(key) + "|gfx950";
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache();
        auto it = g_cache.find(k);
        if (it != g_cache.end() && it->second >= 0 && it->second < nshapes) return it->second;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return 0;
    }
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < nshapes; ++v) {
        launch(v);
        HIP_CHECK(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) launch(v);
        HIP_CHECK(hipEventRecord(e1, s));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[k] = best;
    save_cache();
    return best;
}

int tuned_lookup(const char *key) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache();
    auto it = g_cache.find(std::string(key) + "|gfx950");
    return it == g_cache.end() ? -1 : it->second;
}

}  // namespace dl
