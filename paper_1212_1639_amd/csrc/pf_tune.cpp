// Autotuner of the launch configuration: items per thread (tile size), the
// resampling search strategy and the CDF scan, chosen by timing candidate
// configurations on the caller's stream with the caller's observations.
// Built only on the public calls of include/pf.h; the choice changes tile
// boundaries (hence the summation order of the CDF) but not the random draws,
// which are indexed by particle slot.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "pf.h"

namespace pf {
int set_error(int code, const char* msg);
}

namespace {

constexpr int kIpts[] = {1, 2, 4, 8};

// Tile sizes the library refuses for a configuration (pf_workspace_bytes and
// pf_create return PF_EINVAL for them): double-precision stochastic-
// volatility particle learning at 4 items per thread is switched off.
bool refused_ipt(const pf_config& c, int ipt) {
    return c.model == PF_SV_PL && c.precision == PF_FP64 && ipt == 4;
}
constexpr int64_t kBlock = 256;
constexpr int64_t kCutMax = 2048;

struct Choice {
    int32_t ipt, strategy, lookback;
    double ms;
};

using Key = std::tuple<int, int, int, int, int, int>;  // device, model, precision, scheme, keep, log2 N
std::mutex g_mu;
std::map<Key, Choice> g_cache;

int ceil_log2(int64_t n) {
    int k = 0;
    while ((int64_t(1) << k) < n) ++k;
    return k;
}

// Strategies the library accepts for (scheme, n, ipt).
std::vector<int32_t> strategies(int32_t scheme, int64_t n, int ipt) {
    const int64_t win = 2 * kBlock * ipt;
    const int64_t cut = win < kCutMax ? win : kCutMax;
    std::vector<int32_t> s;
    // the cut-point search: in LDS up to `cut`, with its table in device
    // memory above (multinomial uniforms only: sorted ones merge)
    if (n <= cut || scheme == PF_MULTINOMIAL) s.push_back(PF_SEARCH_CUTPOINT);
    if (scheme != PF_MULTINOMIAL || n <= win) s.push_back(PF_SEARCH_MERGE);
    s.push_back(PF_SEARCH_BINARY);
    return s;
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events() {
        hipEventCreate(&a);
        hipEventCreate(&b);
    }
    ~Events() {
        if (a) hipEventDestroy(a);
        if (b) hipEventDestroy(b);
    }
    bool ok() const { return a && b; }
};

// Milliseconds per step of one filter under `c`: two warm-up observations,
// then the rest timed with events on `s`.  PF_ENOMEM from creation is
// returned as is (the caller skips the candidate).
int time_filter(const pf_config& c, const double* y, int64_t n_obs, hipStream_t s, double* ms) {
    pf_filter* f = nullptr;
    int rc = pf_create(&c, nullptr, 0, s, &f);
    if (rc != PF_OK) return rc;
    Events ev;
    if (!ev.ok()) {
        pf_destroy(f);
        return pf::set_error(PF_EDEVICE, "autotune: event creation failed");
    }
    rc = pf_step(f, y, 2);
    if (rc == PF_OK && hipEventRecord(ev.a, s) != hipSuccess) rc = PF_EDEVICE;
    if (rc == PF_OK) rc = pf_step(f, y + 2, n_obs - 2);
    if (rc == PF_OK && hipEventRecord(ev.b, s) != hipSuccess) rc = PF_EDEVICE;
    float t = 0.0f;
    if (rc == PF_OK && (hipEventSynchronize(ev.b) != hipSuccess ||
                        hipEventElapsedTime(&t, ev.a, ev.b) != hipSuccess))
        rc = PF_EDEVICE;
    const int rd = pf_destroy(f);
    if (rc == PF_EDEVICE) return pf::set_error(PF_EDEVICE, "autotune: timing failed");
    if (rc != PF_OK) return rc;
    if (rd != PF_OK) return rd;
    *ms = static_cast<double>(t) / static_cast<double>(n_obs - 2);
    return PF_OK;
}

// Milliseconds per step of the filters `cs` stepped as one batch.
int time_batch(const std::vector<pf_config>& cs, const double* y, int64_t n_obs, hipStream_t s,
               double* ms) {
    const int n = static_cast<int>(cs.size());
    std::vector<pf_filter*> fs(n, nullptr);
    int rc = PF_OK;
    for (int k = 0; k < n && rc == PF_OK; ++k) rc = pf_create(&cs[k], nullptr, 0, s, &fs[k]);
    pf_batch* b = nullptr;
    if (rc == PF_OK) rc = pf_batch_create(fs.data(), n, n, n_obs < 64 ? static_cast<int32_t>(n_obs) : 64, &b);
    Events ev;
    if (rc == PF_OK && !ev.ok()) rc = pf::set_error(PF_EDEVICE, "autotune: event creation failed");
    if (rc == PF_OK) rc = pf_batch_step(b, y, 2);
    if (rc == PF_OK && hipEventRecord(ev.a, s) != hipSuccess) rc = PF_EDEVICE;
    if (rc == PF_OK) rc = pf_batch_step(b, y + 2 * static_cast<int64_t>(n), n_obs - 2);
    if (rc == PF_OK && hipEventRecord(ev.b, s) != hipSuccess) rc = PF_EDEVICE;
    float t = 0.0f;
    if (rc == PF_OK && (hipEventSynchronize(ev.b) != hipSuccess ||
                        hipEventElapsedTime(&t, ev.a, ev.b) != hipSuccess))
        rc = PF_EDEVICE;
    if (b) pf_batch_destroy(b);
    for (pf_filter* f : fs)
        if (f) pf_destroy(f);
    if (rc == PF_EDEVICE) return pf::set_error(PF_EDEVICE, "autotune: timing failed");
    if (rc != PF_OK) return rc;
    *ms = static_cast<double>(t) / static_cast<double>(n_obs - 2);
    return PF_OK;
}

bool finite_obs(const double* y, int64_t m) {
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(y[i])) return false;
    return true;
}

}  // namespace

extern "C" {

int pf_autotune(pf_config* cfg, const double* y, int64_t n_obs, void* hip_stream,
                double* ms_per_step) {
    if (!cfg || !y) return pf::set_error(PF_EINVAL, "autotune: NULL argument");
    if (n_obs < 3) return pf::set_error(PF_EINVAL, "autotune: needs n_obs >= 3 observations");
    if (!finite_obs(y, n_obs)) return pf::set_error(PF_EINVAL, "autotune: observation is not finite");
    if (pf_workspace_bytes(cfg) == 0) return PF_EINVAL;  // message set by the validation
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return pf::set_error(PF_EDEVICE, "autotune: no device");
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int keep = (cfg->flags & PF_FLAG_KEEP_ANCESTORS) ? 1 : 0;
    const Key key{dev, cfg->model, cfg->precision, cfg->scheme, keep, ceil_log2(cfg->n_particles)};
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            cfg->items_per_thread = it->second.ipt;
            cfg->strategy = it->second.strategy;
            cfg->flags = (cfg->flags & ~PF_FLAG_LOOKBACK_SCAN) |
                         (it->second.lookback ? PF_FLAG_LOOKBACK_SCAN : 0);
            if (ms_per_step) *ms_per_step = it->second.ms;
            return PF_OK;
        }
    }
    pf_config c = *cfg;
    c.flags &= ~PF_FLAG_LOOKBACK_SCAN;
    c.strategy = PF_SEARCH_AUTO;
    Choice best{0, PF_SEARCH_AUTO, 0, INFINITY};
    auto consider = [&](const pf_config& cand) -> int {
        double ms = 0.0;
        const int rc = time_filter(cand, y, n_obs, s, &ms);
        if (rc == PF_ENOMEM) return PF_OK;  // candidate does not fit: skip it
        if (rc != PF_OK) return rc;
        if (ms < best.ms)
            best = Choice{cand.items_per_thread, cand.strategy,
                          (cand.flags & PF_FLAG_LOOKBACK_SCAN) ? 1 : 0, ms};
        return PF_OK;
    };
    // 1. tile size, with the library's default strategy and the tile scan
    for (int ipt : kIpts) {
        if (refused_ipt(c, ipt)) continue;
        c.items_per_thread = ipt;
        const int rc = consider(c);
        if (rc != PF_OK) return rc;
    }
    if (!(best.ms < INFINITY)) return pf::set_error(PF_ENOMEM, "autotune: no candidate fits in memory");
    // 2. search strategy at that tile size
    c.items_per_thread = best.ipt;
    for (int32_t st : strategies(c.scheme, c.n_particles, best.ipt)) {
        c.strategy = st;
        const int rc = consider(c);
        if (rc != PF_OK) return rc;
    }
    // 3. scan: the decoupled look-back instead of the tile scan (sorted
    //    multinomial resampling and the cut-point table in device memory
    //    need the tile scan)
    c.strategy = best.strategy;
    const int64_t win = 2 * kBlock * best.ipt;
    const bool cut_global = best.strategy == PF_SEARCH_CUTPOINT &&
                            c.n_particles > (win < kCutMax ? win : kCutMax);
    if (c.scheme != PF_SORTED_MULTINOMIAL && !cut_global) {
        c.flags |= PF_FLAG_LOOKBACK_SCAN;
        const int rc = consider(c);
        if (rc != PF_OK) return rc;
    }
    cfg->items_per_thread = best.ipt;
    cfg->strategy = best.strategy;
    cfg->flags = (cfg->flags & ~PF_FLAG_LOOKBACK_SCAN) | (best.lookback ? PF_FLAG_LOOKBACK_SCAN : 0);
    if (ms_per_step) *ms_per_step = best.ms;
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key] = best;
    return PF_OK;
}

int pf_autotune_batch(pf_config* cfgs, int32_t n, const double* y, int64_t n_obs,
                      void* hip_stream, double* ms_per_step) {
    if (!cfgs || !y || n < 1) return pf::set_error(PF_EINVAL, "autotune: NULL argument or n < 1");
    if (n_obs < 3) return pf::set_error(PF_EINVAL, "autotune: needs n_obs >= 3 observations");
    if (!finite_obs(y, n_obs * static_cast<int64_t>(n)))
        return pf::set_error(PF_EINVAL, "autotune: observation is not finite");
    for (int32_t k = 0; k < n; ++k) {
        if (pf_workspace_bytes(&cfgs[k]) == 0) return PF_EINVAL;
        if (cfgs[k].flags & PF_FLAG_LOOKBACK_SCAN)
            return pf::set_error(PF_EINVAL, "autotune: batched filters use the tile scan");
    }
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<pf_config> cs(cfgs, cfgs + n);
    Choice best{0, PF_SEARCH_AUTO, 0, INFINITY};
    auto consider = [&](int ipt, bool binary) -> int {
        for (pf_config& c : cs) {
            c.items_per_thread = ipt;
            c.strategy = binary ? PF_SEARCH_BINARY : PF_SEARCH_AUTO;
        }
        double ms = 0.0;
        const int rc = time_batch(cs, y, n_obs, s, &ms);
        if (rc == PF_ENOMEM) return PF_OK;
        if (rc != PF_OK) return rc;
        if (ms < best.ms) best = Choice{ipt, binary ? PF_SEARCH_BINARY : PF_SEARCH_AUTO, 0, ms};
        return PF_OK;
    };
    for (int ipt : kIpts) {
        bool refused = false;
        for (const pf_config& c : cs) refused = refused || refused_ipt(c, ipt);
        if (refused) continue;
        const int rc = consider(ipt, false);
        if (rc != PF_OK) return rc;
    }
    if (!(best.ms < INFINITY)) return pf::set_error(PF_ENOMEM, "autotune: no candidate fits in memory");
    {
        const int rc = consider(best.ipt, true);
        if (rc != PF_OK) return rc;
    }
    for (int32_t k = 0; k < n; ++k) {
        cfgs[k].items_per_thread = best.ipt;
        cfgs[k].strategy = best.strategy;
    }
    if (ms_per_step) *ms_per_step = best.ms;
    return PF_OK;
}

}  // extern "C"
