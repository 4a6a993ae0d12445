// Host runtime of libpf_mi355x.so: configuration checks, workspace layout,
// the per-filter launch sequence and the C-ABI of include/pf.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "pf.h"
#include "pf_internal.h"

namespace pf {
hipError_t launch_step(int model, bool fp64, int ipt, const StepArgs& a, int grid, hipStream_t s,
                       bool init);
hipError_t launch_scan_tiles(double* agg, int32_t num_tiles, int64_t n, int32_t ts, TileAB* ab,
                             int32_t* hint, Totals* tot, DevState* st, double* chunk,
                             const TileAB* pos, hipStream_t s);
hipError_t launch_spacings(int ipt, uint64_t seed, uint32_t t, int64_t n, int32_t num_tiles,
                           double* aggE, TileAB* abE, Totals* totE, double* chunk, hipStream_t s);
int32_t scan_chunks(int32_t num_tiles);
hipError_t static_scratch(int32_t** out);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_cut_table(bool fp64, const void* c, const TileAB* ab, int64_t n, int32_t ts,
                            int32_t tiles, int32_t* table, hipStream_t s);
hipError_t launch_batch(int model, bool fp64, int ipt, const StepArgs* descs, const int2* tile_map,
                        int32_t capacity, BatchState* bs, int grid, hipStream_t s);
hipError_t launch_batch_map(const int32_t* base, int32_t n_filters, int2* tile_map, hipStream_t s);
hipError_t launch_moments(int model, const double* partials, int32_t num_tiles, int64_t n,
                          int32_t weighted, uint32_t t, const ModelParams& p, DevState* st,
                          hipStream_t s);
hipError_t launch_search(int strategy, const double* q, int64_t n, const double* u, int64_t m,
                         int32_t* anc, int32_t* table, int32_t* bad, hipStream_t s);
}  // namespace pf

namespace {

thread_local std::string g_error;

int fail(int code, const std::string& msg) {
    g_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(PF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace pf {
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace pf

namespace {

constexpr int kBlock = 256;
constexpr size_t kAlign = 256;
// Sorted multinomial resampling (exponential spacings).  Its first GPU run
// faulted in the double-precision SV-PL kernel of 4 items per thread, which
// stays refused (it gives wrong weights under every scheme).  The single-
// precision kernels of 4 items per thread carry no sorted-multinomial code:
// the library picks 2 items there and refuses an explicit 4.
constexpr bool kSortedMultinomial = true;
constexpr int64_t kCutMax = 2048;  // largest CDF with an in-LDS cut-point table

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int model_fields(int32_t model) {
    switch (model) {
    case PF_LL_PF: return 1;
    case PF_LL_PL: return 5;
    case PF_SV_PF: return 1;
    case PF_SV_PL: return 6;
    }
    return 0;
}

int model_moments(int32_t model) {
    switch (model) {
    case PF_LL_PF: return 3;
    case PF_LL_PL: return 6;
    case PF_SV_PF: return 3;
    case PF_SV_PL: return 7;
    }
    return 0;
}

// Double-precision stochastic-volatility particle learning with 4 items per
// thread is switched off: that kernel gave wrong weights from its first
// resampling on (and the one run that faulted the GPU used it), while the
// same model at 1, 2 and 8 items per thread, and every other model at 4,
// match the oracle; the cause is not yet found.
bool switched_off_ipt(const pf_config& c, int ipt) {
    return c.model == PF_SV_PL && c.precision == PF_FP64 && ipt == 4;
}

int choose_ipt(const pf_config& c) {
    if (c.items_per_thread) return c.items_per_thread;
    if (switched_off_ipt(c, 4)) return 1;
    if (c.scheme == PF_SORTED_MULTINOMIAL && c.precision == PF_FP32) return 2;
    // measured on MI355X: 4 items per thread (with 5 resident work-groups
    // per CU) beats 2 and 8 from 2^20 to 2^26 particles
    return 4;
}

struct Layout {
    int ipt = 0, ts = 0, num_tiles = 0, fields = 0, rsz = 0, strategy = 0;
    int64_t pitch = 0;
    size_t rec[2], c[2], samp[2], tiles[2], tot[2], status, state, partials, anc, agg, ab, hint,
        chunk, aggE, abE, totE, cut, total;
    bool spacings = false;  // sorted multinomial: the exponential spacings' tile scan
    bool lookback = false;
    bool cut_global = false;  // cut-point table in device memory (CDF larger than LDS)
};

bool finite_all(std::initializer_list<double> v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// Validates `c` and fills the workspace layout; returns 0 or PF_EINVAL.
int plan(const pf_config* c, Layout* L) {
    if (!c) return fail(PF_EINVAL, "pf_config is NULL");
    if (c->model < PF_LL_PF || c->model > PF_SV_PL) return fail(PF_EINVAL, "unknown model");
    if (c->scheme < PF_MULTINOMIAL || c->scheme > PF_SORTED_MULTINOMIAL)
        return fail(PF_EINVAL, "unknown resampling scheme");
    if (c->scheme == PF_SORTED_MULTINOMIAL && !kSortedMultinomial)
        return fail(PF_EINVAL, "sorted multinomial resampling is switched off "
                               "(its first GPU runs ended in a memory fault whose cause has "
                               "not been found)");
    if (c->scheme == PF_SORTED_MULTINOMIAL && (c->flags & PF_FLAG_LOOKBACK_SCAN))
        return fail(PF_EINVAL, "sorted multinomial resampling uses the tile scan "
                               "(PF_FLAG_LOOKBACK_SCAN is not available with it)");
    if (c->precision != PF_FP32 && c->precision != PF_FP64)
        return fail(PF_EINVAL, "precision must be PF_FP32 or PF_FP64");
    if (c->strategy < PF_SEARCH_AUTO || c->strategy > PF_SEARCH_MERGE)
        return fail(PF_EINVAL, "unknown search strategy");
    if (c->n_particles < 1 || c->n_particles > INT32_MAX)
        return fail(PF_EINVAL, "n_particles must be in [1, 2^31 - 1]");
    if (c->flags & ~(PF_FLAG_KEEP_ANCESTORS | PF_FLAG_LOOKBACK_SCAN | PF_FLAG_TEST_SCAN_STALL))
        return fail(PF_EINVAL, "unknown bits in flags");
    const int ipt = choose_ipt(*c);
    if (ipt != 1 && ipt != 2 && ipt != 4 && ipt != 8)
        return fail(PF_EINVAL, "items_per_thread must be 0, 1, 2, 4 or 8");
    if (switched_off_ipt(*c, ipt))
        return fail(PF_EINVAL, "double-precision PF_SV_PL with 4 items per thread is switched off "
                               "(wrong weights whose cause has not been found); use 1, 2 or 8");
    if (c->scheme == PF_SORTED_MULTINOMIAL && c->precision == PF_FP32 && ipt == 4)
        return fail(PF_EINVAL, "sorted multinomial in PF_FP32 runs at 1, 2 or 8 items per thread "
                               "(the 4-item single-precision kernels carry no code for it)");
    if (!finite_all({c->x0_mean, c->x0_var}) || !(c->x0_var > 0))
        return fail(PF_EINVAL, "x0_var must be finite and > 0");
    switch (c->model) {
    case PF_LL_PF:
        if (!(c->sigma_v2 > 0) || !(c->sigma_w2 > 0) || !finite_all({c->sigma_v2, c->sigma_w2}))
            return fail(PF_EINVAL, "sigma_v2 and sigma_w2 must be finite and > 0");
        break;
    case PF_LL_PL:
        if (!(c->a_v >= 1) || !(c->a_w >= 1) || !(c->b_v > 0) || !(c->b_w > 0) ||
            !finite_all({c->a_v, c->a_w, c->b_v, c->b_w}))
            return fail(PF_EINVAL, "IG priors need shape >= 1 and scale > 0");
        break;
    case PF_SV_PF:
        if (!(c->sigma2 > 0) || !finite_all({c->mu, c->phi, c->sigma2}))
            return fail(PF_EINVAL, "sigma2 must be finite and > 0");
        break;
    case PF_SV_PL: {
        const double p0 = c->prior_prec[0], p1 = c->prior_prec[1], p2 = c->prior_prec[2];
        if (!(p0 > 0) || !(p0 * p2 - p1 * p1 > 0) || !finite_all({p0, p1, p2}))
            return fail(PF_EINVAL, "prior_prec must be symmetric positive definite");
        if (!(c->a_s >= 1) || !(c->d_s > 0) || !finite_all({c->a_s, c->d_s, c->prior_mean[0],
                                                            c->prior_mean[1]}))
            return fail(PF_EINVAL, "IG prior of sigma^2 needs shape >= 1 and scale > 0");
        break;
    }
    }
    L->ipt = ipt;
    L->ts = kBlock * ipt;
    const int64_t n = c->n_particles;
    L->num_tiles = static_cast<int>((n + L->ts - 1) / L->ts);
    L->fields = model_fields(c->model);
    L->rsz = c->precision == PF_FP64 ? 8 : 4;
    L->pitch = static_cast<int64_t>(align_up(static_cast<size_t>(n), 64));
    const int64_t win = 2 * static_cast<int64_t>(L->ts);
    const int64_t cut_max = win < kCutMax ? win : kCutMax;
    int strat = c->strategy;
    if (strat == PF_SEARCH_AUTO) {
        if (c->scheme == PF_MULTINOMIAL)
            strat = n <= cut_max ? PF_SEARCH_CUTPOINT : (n <= win ? PF_SEARCH_MERGE : PF_SEARCH_CUTPOINT);
        else
            strat = PF_SEARCH_MERGE;
    }
    // above one LDS window the cut-point table lives in device memory and is
    // built by its own launch after each weighting (tile-scan form only)
    L->cut_global = strat == PF_SEARCH_CUTPOINT && n > cut_max;
    if (L->cut_global && (c->flags & PF_FLAG_LOOKBACK_SCAN))
        return fail(PF_EINVAL, "the cut-point search above min(2048, 2 * 256 * items_per_thread) "
                               "particles builds its table from the tile scan's output; "
                               "PF_FLAG_LOOKBACK_SCAN is not available with it");
    if (strat == PF_SEARCH_MERGE && c->scheme == PF_MULTINOMIAL && n > win)
        return fail(PF_EINVAL, "the merge search needs sorted uniforms (stratified or systematic) "
                               "when N exceeds one LDS window");
    L->strategy = strat;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, kAlign);
        return at;
    };
    const size_t rec_bytes = static_cast<size_t>(L->fields) * L->pitch * L->rsz;
    for (int b = 0; b < 2; ++b) L->rec[b] = take(rec_bytes);
    for (int b = 0; b < 2; ++b) L->c[b] = take(static_cast<size_t>(L->pitch) * L->rsz);
    for (int b = 0; b < 2; ++b)
        L->samp[b] = take(static_cast<size_t>(L->num_tiles) * pf::kSegments * L->rsz);
    for (int b = 0; b < 2; ++b) L->tiles[b] = take(sizeof(pf::TileInfo) * L->num_tiles);
    for (int b = 0; b < 2; ++b) L->tot[b] = take(sizeof(pf::Totals));
    L->status = take(sizeof(uint64_t) * pf::kStatusWords * L->num_tiles);
    L->state = take(sizeof(pf::DevState));
    L->partials = take(sizeof(double) * pf::kPartialStride * L->num_tiles);
    L->anc = (c->flags & PF_FLAG_KEEP_ANCESTORS) ? take(sizeof(int32_t) * L->pitch) : 0;
    L->agg = take(sizeof(double) * 2 * L->num_tiles);
    L->ab = take(sizeof(pf::TileAB) * L->num_tiles);
    L->hint = take(sizeof(int32_t) * (L->num_tiles + 1));
    const int64_t chunks = pf::scan_chunks(L->num_tiles);
    L->chunk = take(sizeof(double) * (3 * chunks + 1));
    L->spacings = c->scheme == PF_SORTED_MULTINOMIAL;
    L->aggE = L->spacings ? take(sizeof(double) * 2 * L->num_tiles) : 0;
    L->abE = L->spacings ? take(sizeof(pf::TileAB) * L->num_tiles) : 0;
    L->totE = L->spacings ? take(sizeof(pf::Totals)) : 0;
    L->cut = L->cut_global ? take(sizeof(int32_t) * static_cast<size_t>(n)) : 0;
    L->lookback = (c->flags & PF_FLAG_LOOKBACK_SCAN) != 0;
    L->total = off;
    return PF_OK;
}

pf::ModelParams params_of(const pf_config& c) {
    pf::ModelParams p{};
    p.x0_mean = c.x0_mean;
    p.x0_var = c.x0_var;
    p.sigma_v2 = c.sigma_v2;
    p.sigma_w2 = c.sigma_w2;
    p.a_v = c.a_v;
    p.b_v = c.b_v;
    p.a_w = c.a_w;
    p.b_w = c.b_w;
    p.mu = c.mu;
    p.phi = c.phi;
    p.sigma2 = c.sigma2;
    p.b0a = c.prior_mean[0];
    p.b0b = c.prior_mean[1];
    p.p0 = c.prior_prec[0];
    p.p1 = c.prior_prec[1];
    p.p2 = c.prior_prec[2];
    p.a_s = c.a_s;
    p.d_s = c.d_s;
    return p;
}

}  // namespace

struct pf_filter {
    pf_config cfg;
    Layout L;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    bool owns_ws = false;
    int cur = 0;             // record buffer holding the current particles
    int cdf = 0;             // buffer holding the latest CDF
    bool have_cdf = false;   // the latest particles carry weights (a CDF)
    bool pending = false;    // particle learning: weighted for y_pend, not yet propagated
    double y_pend = 0.0;
    uint32_t t = 0;          // propagations done
    uint32_t epoch = 0;      // look-back tag of the latest weighting launch
    int32_t weighted_partials = 0;
    pf::ModelParams mp;
    // asynchronous copies of a record buffer to the host: a launch that
    // overwrites buffer b first waits for copy_ev[b]
    hipEvent_t copy_ev[2] = {nullptr, nullptr};
    bool copy_pending[2] = {false, false};
    hipEvent_t step_ev = nullptr;

    int wait_copy(hipStream_t s, int b) {
        if (!copy_pending[b]) return PF_OK;
        copy_pending[b] = false;
        const hipError_t e = hipStreamWaitEvent(s, copy_ev[b], 0);
        return e == hipSuccess ? PF_OK : hip_fail(e, "wait for a particle copy");
    }
    int wait_copies(hipStream_t s) {
        int rc = wait_copy(s, 0);
        return rc != PF_OK ? rc : wait_copy(s, 1);
    }

    // kernel timing: event pairs bracketing the cycle-kernel launches
    std::vector<hipEvent_t> tev;
    int64_t timed = 0;       // bracketed launches so far
    int64_t launches = 0;    // cycle launches since timing was armed
    int64_t every = 1;       // bracket one launch in `every`

    template <typename T>
    T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
    template <typename T>
    const T* at(size_t off) const { return reinterpret_cast<const T*>(ws + off); }

    pf::StepArgs args() {
        pf::StepArgs a{};
        a.n = cfg.n_particles;
        a.pitch = L.pitch;
        a.num_tiles = L.num_tiles;
        a.scheme = cfg.scheme;
        a.strategy = L.strategy;
        a.seed = cfg.seed;
        a.status = at<uint64_t>(L.status);
        a.st = at<pf::DevState>(L.state);
        a.partials = at<double>(L.partials);
        a.anc_out = (cfg.flags & PF_FLAG_KEEP_ANCESTORS) ? at<int32_t>(L.anc) : nullptr;
        a.scan = L.lookback ? pf::kScanLookback : pf::kScanTiles;
        a.ts = L.ts;
        a.rsz = L.rsz;
        a.test_stall = (cfg.flags & PF_FLAG_TEST_SCAN_STALL) ? 1 : 0;
        a.ab_out = at<pf::TileAB>(L.ab);
        a.hint_out = at<int32_t>(L.hint);
        a.ab_in = at<pf::TileAB>(L.ab);
        a.hint_in = at<int32_t>(L.hint);
        a.agg_out = at<double>(L.agg);
        a.chunk = at<double>(L.chunk);
        a.abE = L.spacings ? at<pf::TileAB>(L.abE) : nullptr;
        a.cut_in = L.cut_global ? at<int32_t>(L.cut) : nullptr;
        a.p = mp;
        return a;
    }

    // Arguments of one cycle and the host-side state change it implies.
    // resample: draw ancestors from the latest CDF; propagate: move with
    // y_prop; weight: score against y_weight.
    pf::StepArgs prepare(bool resample, bool propagate, bool weight, double y_prop,
                         double y_weight) {
        pf::StepArgs a = args();
        a.flags = (resample ? pf::kResample : 0) | (propagate ? pf::kPropagate : 0) |
                  (weight ? pf::kWeight : 0);
        const bool weighted_mom = weight && cfg.model != PF_LL_PL;
        if (weighted_mom) a.flags |= pf::kWeightedMoments;
        // small filters scan their tiles in the cycle kernel's last work-group
        if (weight && fused_scan()) a.flags |= pf::kFusedScan;
        a.t = t + 1;
        a.y_prop = y_prop;
        a.y_weight = y_weight;
        a.rec_in = ws + L.rec[cur];
        a.rec_out = ws + L.rec[1 - cur];
        a.c_in = ws + L.c[cdf];
        a.samp_in = ws + L.samp[cdf];
        a.samp_out = ws + L.samp[1 - cdf];
        a.tiles_in = at<pf::TileInfo>(L.tiles[cdf]);
        a.tot_in = at<pf::Totals>(L.tot[cdf]);
        a.c_out = ws + L.c[1 - cdf];
        a.tiles_out = at<pf::TileInfo>(L.tiles[1 - cdf]);
        a.tot_out = at<pf::Totals>(L.tot[1 - cdf]);
        if (weight) {
            if (++epoch == 0) epoch = 1;
        }
        a.epoch = epoch;
        if (propagate) {
            cur = 1 - cur;
            ++t;
        }
        if (weight) {
            cdf = 1 - cdf;
            have_cdf = true;
        } else if (propagate) {
            have_cdf = false;
        }
        weighted_partials = weighted_mom ? 1 : 0;
        return a;
    }

    // The cycle for one observation: particle learning weights y_{t+1}
    // before it propagates with y_t, so it runs one observation behind.
    pf::StepArgs prepare_obs(double y) {
        if (cfg.model == PF_LL_PL) {
            pf::StepArgs a = pending ? prepare(true, true, true, y_pend, y)
                                     : prepare(false, false, true, 0.0, y);
            pending = true;
            y_pend = y;
            return a;
        }
        return prepare(have_cdf, true, true, y, y);
    }

    bool fused_scan() const {
        return !L.lookback && !L.spacings && L.num_tiles <= pf::kFusedScanMax;
    }

    int run(const pf::StepArgs& a) {
        if (a.flags & pf::kPropagate) {
            const int b = a.rec_out == static_cast<void*>(ws + L.rec[0]) ? 0 : 1;
            const int rc = wait_copy(stream, b);
            if (rc != PF_OK) return rc;
        }
        const bool timing = 2 * timed + 1 < static_cast<int64_t>(tev.size()) &&
                            launches++ % every == 0;
        if (timing && hipEventRecord(tev[2 * timed], stream) != hipSuccess)
            return hip_fail(hipGetLastError(), "timing event");
        hipError_t e = pf::launch_step(cfg.model, cfg.precision == PF_FP64, L.ipt, a, L.num_tiles,
                                       stream, false);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        if (timing) {
            if (hipEventRecord(tev[2 * timed + 1], stream) != hipSuccess)
                return hip_fail(hipGetLastError(), "timing event");
            ++timed;
        }
        if ((a.flags & pf::kWeight) && !L.lookback && !(a.flags & pf::kFusedScan)) {
            const pf::TileAB* pos = nullptr;
            if (L.spacings) {
                // the uniforms of the next resampling (the cycle that uses this
                // CDF): its time index is this launch's, or the next if this
                // launch propagated
                const uint32_t next_t = (a.flags & pf::kPropagate) ? a.t + 1 : a.t;
                e = pf::launch_spacings(L.ipt, cfg.seed, next_t, cfg.n_particles, L.num_tiles,
                                        at<double>(L.aggE), at<pf::TileAB>(L.abE),
                                        at<pf::Totals>(L.totE), at<double>(L.chunk), stream);
                if (e != hipSuccess) return hip_fail(e, "spacing launch");
                pos = at<pf::TileAB>(L.abE);
            }
            e = pf::launch_scan_tiles(a.agg_out, L.num_tiles, cfg.n_particles, L.ts,
                                      at<pf::TileAB>(L.ab), at<int32_t>(L.hint), a.tot_out, a.st,
                                      at<double>(L.chunk), pos, stream);
            if (e != hipSuccess) return hip_fail(e, "tile scan launch");
        }
        if ((a.flags & pf::kWeight) && L.cut_global) {
            // the cut-point table of the CDF this launch weighed
            e = pf::launch_cut_table(cfg.precision == PF_FP64, a.c_out, at<pf::TileAB>(L.ab),
                                     cfg.n_particles, L.ts, L.num_tiles, at<int32_t>(L.cut), stream);
            if (e != hipSuccess) return hip_fail(e, "cut-point table launch");
        }
        return PF_OK;
    }

    int launch(bool resample, bool propagate, bool weight, double y_prop, double y_weight) {
        return run(prepare(resample, propagate, weight, y_prop, y_weight));
    }
};

// A batch: filters of one model, precision and tile size whose cycles run
// together, one persistent step launch and one scan launch per observation,
// replayed from a captured graph.  Each step's arguments are staged in a
// device ring of `ring` blocks of n StepArgs.
struct pf_batch {
    std::vector<pf_filter*> fs;
    hipStream_t stream = nullptr;
    int model = 0, ipt = 0;
    bool fp64 = false;
    int32_t ring = 0, capacity = 0;
    int64_t total_tiles = 0;
    uint64_t issued = 0;          // steps queued so far (the device counter follows)
    pf::StepArgs* d_descs = nullptr;
    int32_t* d_base = nullptr;
    int2* d_map = nullptr;        // global tile -> (member, member's tile)
    int64_t map_cap = 0;          // tiles d_map holds
    pf::BatchState* d_state = nullptr;
    pf::StepArgs* h_stage = nullptr;  // pinned staging of the ring
    std::vector<hipEvent_t> slot_copied;  // slot's staging copy has completed
    // pinned staging of membership updates: kMemberSlots blocks of
    // (capacity + 1) tile offsets followed by a MemberTail
    static constexpr int kMemberSlots = 4;
    struct MemberTail {
        int32_t n_filters, capacity;
        int64_t total_tiles;
    };
    size_t member_block_ints() const { return static_cast<size_t>(capacity) + 1 + 6; }
    int32_t* h_member = nullptr;
    hipEvent_t member_copied[kMemberSlots] = {};
    int member_next = 0;
    hipGraphExec_t exec = nullptr;
};
extern "C" {

int pf_fields(int32_t model) { return model_fields(model); }

size_t pf_workspace_bytes(const pf_config* cfg) {
    Layout L;
    if (plan(cfg, &L) != PF_OK) return 0;
    return L.total;
}

int pf_create(const pf_config* cfg, void* workspace, size_t ws_bytes, void* hip_stream,
              pf_filter** out) {
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    int rc = plan(cfg, &L);
    if (rc != PF_OK) return rc;
    pf_filter* f = new (std::nothrow) pf_filter();
    if (!f) return fail(PF_ENOMEM, "host allocation failed");
    f->cfg = *cfg;
    f->L = L;
    f->stream = static_cast<hipStream_t>(hip_stream);
    f->mp = params_of(*cfg);
    if (workspace) {
        if (ws_bytes < L.total) {
            delete f;
            return fail(PF_ENOMEM, "workspace smaller than pf_workspace_bytes()");
        }
        if (reinterpret_cast<uintptr_t>(workspace) % kAlign) {
            delete f;
            return fail(PF_EINVAL, "workspace must be 256-byte aligned");
        }
        f->ws = static_cast<char*>(workspace);
    } else {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, L.total);
        if (e != hipSuccess) {
            delete f;
            return fail(PF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        f->ws = static_cast<char*>(p);
        f->owns_ws = true;
    }
    // Step 0 of both algorithms: sample the initial particles
    pf::StepArgs a = f->args();
    a.rec_out = f->ws + L.rec[0];
    hipError_t e = pf::launch_step(cfg->model, cfg->precision == PF_FP64, L.ipt, a, L.num_tiles,
                                   f->stream, true);
    if (e != hipSuccess) {
        if (f->owns_ws) hipFree(f->ws);
        delete f;
        return hip_fail(e, "init kernel launch");
    }
    *out = f;
    g_error.clear();
    return PF_OK;
}

int pf_step(pf_filter* f, const double* y, int64_t n_obs) {
    if (!f) return fail(PF_EINVAL, "filter is NULL");
    if (!y || n_obs < 1) return fail(PF_EINVAL, "need n_obs >= 1 observations");
    for (int64_t i = 0; i < n_obs; ++i)
        if (!std::isfinite(y[i])) return fail(PF_EINVAL, "observation is not finite");
    for (int64_t i = 0; i < n_obs; ++i) {
        const int rc = f->run(f->prepare_obs(y[i]));
        if (rc != PF_OK) return rc;
    }
    return PF_OK;
}

int pf_loglik(const pf_filter* f, double* out) {
    if (!f || !out) return fail(PF_EINVAL, "NULL argument");
    pf::DevState st;
    hipError_t e = hipMemcpyAsync(&st, f->at<pf::DevState>(f->L.state), sizeof(st),
                                  hipMemcpyDeviceToHost, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_loglik copy");
    *out = st.loglik;
    if (st.flags & pf::kScanStall) return fail(PF_EDEVICE, "a tile scan in the cycle kernel stopped waiting for a tile's sums");
    if (st.flags & pf::kDegenerate) return fail(PF_EDEGENERATE, "a step's weights were all zero or not finite");
    return PF_OK;
}

int pf_moments(pf_filter* f, double* out, int32_t n_out) {
    if (!f || !out) return fail(PF_EINVAL, "NULL argument");
    const int need = model_moments(f->cfg.model);
    if (n_out < need) return fail(PF_EINVAL, "n_out smaller than the model's moment count");
    if (f->cfg.model == PF_LL_PL && f->pending) {
        int rc = f->launch(true, true, false, f->y_pend, 0.0);
        if (rc != PF_OK) return rc;
        f->pending = false;
    }
    hipError_t e = pf::launch_moments(f->cfg.model, f->at<double>(f->L.partials), f->L.num_tiles,
                                      f->cfg.n_particles, f->weighted_partials, f->t, f->mp,
                                      f->at<pf::DevState>(f->L.state), f->stream);
    if (e != hipSuccess) return hip_fail(e, "moment kernel launch");
    pf::DevState st;
    e = hipMemcpyAsync(&st, f->at<pf::DevState>(f->L.state), sizeof(st), hipMemcpyDeviceToHost,
                       f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_moments copy");
    for (int k = 0; k < n_out; ++k) out[k] = k < need ? st.moments[k] : 0.0;
    if (st.flags & pf::kScanStall) return fail(PF_EDEVICE, "a tile scan in the cycle kernel stopped waiting for a tile's sums");
    if (st.flags & pf::kDegenerate) return fail(PF_EDEGENERATE, "a step's weights were all zero or not finite");
    return PF_OK;
}

static void release_timing(pf_filter* f) {
    for (hipEvent_t ev : f->tev) hipEventDestroy(ev);
    f->tev.clear();
    f->timed = 0;
    f->launches = 0;
    f->every = 1;
}

int pf_timing_start(pf_filter* f, int64_t max_launches, int64_t every) {
    if (!f) return fail(PF_EINVAL, "null filter");
    if (max_launches < 1 || max_launches > (1 << 20))
        return fail(PF_EINVAL, "max_launches must be in [1, 2^20]");
    if (every < 1) return fail(PF_EINVAL, "every must be >= 1");
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_timing_start synchronise");
    release_timing(f);
    f->every = every;
    f->tev.resize(static_cast<size_t>(2 * max_launches));
    for (size_t i = 0; i < f->tev.size(); ++i) {
        e = hipEventCreate(&f->tev[i]);
        if (e != hipSuccess) {
            f->tev.resize(i);
            release_timing(f);
            return hip_fail(e, "pf_timing_start event");
        }
    }
    return PF_OK;
}

int pf_timing_read(pf_filter* f, double* total_ms, int64_t* launches) {
    if (!f || !total_ms || !launches) return fail(PF_EINVAL, "null argument");
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_timing_read synchronise");
    double sum = 0.0;
    for (int64_t k = 0; k < f->timed; ++k) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, f->tev[2 * k], f->tev[2 * k + 1]);
        if (e != hipSuccess) {
            release_timing(f);
            return hip_fail(e, "pf_timing_read elapsed time");
        }
        sum += ms;
    }
    *total_ms = sum;
    *launches = f->timed;
    release_timing(f);
    return PF_OK;
}

// ------------------------------------------------------------ checkpoints
namespace {
constexpr uint64_t kCkptMagic = 0x31305450434b4650ull;  // "PFKCPT01"
constexpr uint32_t kCkptVersion = 1;

// What a snapshot records besides device memory: the configuration the
// workspace layout follows and the host side of the filter's state.
struct CkptHeader {
    uint64_t magic;
    uint32_t version, header_bytes;
    int32_t model, scheme, precision, strategy, ipt, fields, rsz, num_tiles;
    int64_t n_particles, pitch;
    uint64_t seed, flags, ws_total, payload;
    pf::ModelParams mp;
    int32_t cur, cdf, have_cdf, pending;
    double y_pend;
    uint32_t t, epoch;
    int32_t weighted_partials, pad;
};

// The workspace regions a snapshot holds, in address order: everything but
// the record buffer and the CDF-prefix buffer the next cycle writes without
// reading (rec[1 - cur], c[1 - cdf]); at most three pieces.
int live_regions(const pf_filter* f, size_t off[3], size_t len[3]);
}  // namespace

namespace {
int live_regions(const pf_filter* f, size_t off[3], size_t len[3]) {
    const size_t rec_bytes = f->L.rec[1] - f->L.rec[0];
    const size_t c_bytes = f->L.c[1] - f->L.c[0];
    size_t dead_off[2] = {f->L.rec[1 - f->cur], f->L.c[1 - f->cdf]};
    size_t dead_len[2] = {rec_bytes, c_bytes};
    if (dead_off[1] < dead_off[0]) {
        std::swap(dead_off[0], dead_off[1]);
        std::swap(dead_len[0], dead_len[1]);
    }
    int k = 0;
    size_t at = 0;
    for (int d = 0; d < 2; ++d) {
        if (dead_off[d] > at) {
            off[k] = at;
            len[k++] = dead_off[d] - at;
        }
        at = dead_off[d] + dead_len[d];
    }
    if (f->L.total > at) {
        off[k] = at;
        len[k++] = f->L.total - at;
    }
    return k;
}

size_t ckpt_payload(const pf_filter* f) {
    return f->L.total - (f->L.rec[1] - f->L.rec[0]) - (f->L.c[1] - f->L.c[0]);
}
}  // namespace

size_t pf_checkpoint_bytes(const pf_filter* f) {
    if (!f) return 0;
    return sizeof(CkptHeader) + ckpt_payload(f);
}

int pf_checkpoint_save(pf_filter* f, void* host_out, size_t bytes) {
    if (!f || !host_out) return fail(PF_EINVAL, "NULL argument");
    if (bytes < pf_checkpoint_bytes(f)) return fail(PF_EINVAL, "host buffer smaller than pf_checkpoint_bytes()");
    int rc = f->wait_copies(f->stream);
    if (rc != PF_OK) return rc;
    CkptHeader h{};
    h.magic = kCkptMagic;
    h.version = kCkptVersion;
    h.header_bytes = sizeof(CkptHeader);
    h.model = f->cfg.model;
    h.scheme = f->cfg.scheme;
    h.precision = f->cfg.precision;
    h.strategy = f->L.strategy;
    h.ipt = f->L.ipt;
    h.fields = f->L.fields;
    h.rsz = f->L.rsz;
    h.num_tiles = f->L.num_tiles;
    h.n_particles = f->cfg.n_particles;
    h.pitch = f->L.pitch;
    h.seed = f->cfg.seed;
    h.flags = f->cfg.flags;
    h.ws_total = f->L.total;
    h.payload = ckpt_payload(f);
    h.mp = f->mp;
    h.cur = f->cur;
    h.cdf = f->cdf;
    h.have_cdf = f->have_cdf ? 1 : 0;
    h.pending = f->pending ? 1 : 0;
    h.y_pend = f->y_pend;
    h.t = f->t;
    h.epoch = f->epoch;
    h.weighted_partials = f->weighted_partials;
    char* dst = static_cast<char*>(host_out);
    std::memcpy(dst, &h, sizeof(h));
    size_t off[3], len[3];
    const int k = live_regions(f, off, len);
    size_t pos = sizeof(h);
    hipError_t e = hipSuccess;
    for (int r = 0; r < k && e == hipSuccess; ++r) {
        e = hipMemcpyAsync(dst + pos, f->ws + off[r], len[r], hipMemcpyDeviceToHost, f->stream);
        pos += len[r];
    }
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_checkpoint_save");
    return PF_OK;
}

int pf_checkpoint_restore(pf_filter* f, const void* host_in, size_t bytes) {
    if (!f || !host_in) return fail(PF_EINVAL, "NULL argument");
    if (bytes < sizeof(CkptHeader)) return fail(PF_EINVAL, "not a filter snapshot (too short)");
    CkptHeader h;
    std::memcpy(&h, host_in, sizeof(h));
    if (h.magic != kCkptMagic || h.header_bytes != sizeof(CkptHeader))
        return fail(PF_EINVAL, "not a filter snapshot");
    if (h.version != kCkptVersion) return fail(PF_EINVAL, "snapshot of another format version");
    const bool same =
        h.model == f->cfg.model && h.scheme == f->cfg.scheme && h.precision == f->cfg.precision &&
        h.strategy == f->L.strategy && h.ipt == f->L.ipt && h.fields == f->L.fields &&
        h.rsz == f->L.rsz && h.num_tiles == f->L.num_tiles &&
        h.n_particles == f->cfg.n_particles && h.pitch == f->L.pitch && h.seed == f->cfg.seed &&
        h.flags == f->cfg.flags && h.ws_total == f->L.total &&
        std::memcmp(&h.mp, &f->mp, sizeof(h.mp)) == 0;
    if (!same)
        return fail(PF_EINVAL, "the snapshot was taken from a filter of another configuration");
    if (h.payload != ckpt_payload(f) || bytes < sizeof(CkptHeader) + h.payload)
        return fail(PF_EINVAL, "snapshot truncated");
    if ((h.cur != 0 && h.cur != 1) || (h.cdf != 0 && h.cdf != 1))
        return fail(PF_EINVAL, "corrupt snapshot");
    // nothing queued on the filter may still write its workspace
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_checkpoint_restore synchronise");
    int rc = f->wait_copies(f->stream);
    if (rc != PF_OK) return rc;
    f->cur = h.cur;
    f->cdf = h.cdf;
    f->have_cdf = h.have_cdf != 0;
    f->pending = h.pending != 0;
    f->y_pend = h.y_pend;
    f->t = h.t;
    f->epoch = h.epoch;
    f->weighted_partials = h.weighted_partials;
    size_t off[3], len[3];
    const int k = live_regions(f, off, len);
    const char* src = static_cast<const char*>(host_in) + sizeof(h);
    for (int r = 0; r < k && e == hipSuccess; ++r) {
        e = hipMemcpyAsync(f->ws + off[r], src, len[r], hipMemcpyHostToDevice, f->stream);
        src += len[r];
    }
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_checkpoint_restore");
    return PF_OK;
}

int pf_destroy(pf_filter* f) {
    if (!f) return PF_OK;
    hipError_t e = hipStreamSynchronize(f->stream);
    // the workspace may still be read by a particle copy on another stream
    for (int b = 0; b < 2; ++b) {
        if (f->copy_ev[b]) {
            const hipError_t e2 = hipEventSynchronize(f->copy_ev[b]);
            if (e == hipSuccess) e = e2;
            hipEventDestroy(f->copy_ev[b]);
        }
    }
    if (f->step_ev) hipEventDestroy(f->step_ev);
    release_timing(f);
    if (f->owns_ws) hipFree(f->ws);
    delete f;
    if (e != hipSuccess) return hip_fail(e, "pf_destroy synchronise");
    return PF_OK;
}

const char* pf_last_error(void) { return g_error.c_str(); }

int pf_debug_search(const double* cdf_dev, const double* u_dev, int64_t n, int64_t m,
                    int32_t strategy, int32_t* anc_dev, void* hip_stream) {
    if (!cdf_dev || n < 1 || n > INT32_MAX) return fail(PF_EINVAL, "need a CDF of 1 <= n < 2^31 entries");
    if (m < 0 || (m > 0 && (!u_dev || !anc_dev))) return fail(PF_EINVAL, "bad uniforms / output");
    if (strategy == PF_SEARCH_AUTO) strategy = PF_SEARCH_MERGE;
    if (strategy < PF_SEARCH_BINARY || strategy > PF_SEARCH_MERGE)
        return fail(PF_EINVAL, "unknown search strategy");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int32_t* table = nullptr;
    int32_t* bad = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&bad), sizeof(int32_t));
    if (e != hipSuccess) return fail(PF_ENOMEM, "hipMalloc of the check flag failed");
    if (strategy == PF_SEARCH_CUTPOINT) {
        e = hipMalloc(reinterpret_cast<void**>(&table), sizeof(int32_t) * static_cast<size_t>(n));
        if (e != hipSuccess) {
            hipFree(bad);
            return fail(PF_ENOMEM, "hipMalloc of the cut-point table failed");
        }
    }
    int rc = PF_OK;
    e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = pf::launch_search(strategy, cdf_dev, n, u_dev, m, anc_dev, table, bad, s);
    int32_t hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "pf_debug_search");
    else if (hbad) rc = fail(PF_EINVAL, "CDF is decreasing somewhere or not finite");
    hipFree(bad);
    if (table) hipFree(table);
    return rc;
}

int pf_debug_search_noalloc(const double* cdf_dev, const double* u_dev, int64_t n, int64_t m,
                            int32_t strategy, int32_t* anc_dev, void* hip_stream) {
    if (!cdf_dev || n < 1 || n > INT32_MAX) return fail(PF_EINVAL, "need a CDF of 1 <= n < 2^31 entries");
    if (m < 0 || (m > 0 && (!u_dev || !anc_dev))) return fail(PF_EINVAL, "bad uniforms / output");
    if (strategy == PF_SEARCH_AUTO) strategy = PF_SEARCH_MERGE;
    if (strategy < PF_SEARCH_BINARY || strategy > PF_SEARCH_MERGE)
        return fail(PF_EINVAL, "unknown search strategy");
    if (strategy == PF_SEARCH_CUTPOINT && n > pf::kStaticCutMax)
        return fail(PF_EINVAL, "pf_debug_search_noalloc: the cut-point table holds at most 2^20 "
                               "entries (use pf_debug_search for larger CDFs)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int32_t* scr = nullptr;
    hipError_t e = pf::static_scratch(&scr);
    if (e != hipSuccess) return hip_fail(e, "pf_debug_search_noalloc: static scratch");
    int32_t* bad = scr;
    int32_t* table = strategy == PF_SEARCH_CUTPOINT ? scr + pf::kStaticTableOffset : nullptr;
    // the array keeps the previous call's contents: the flag starts at zero
    e = pf::launch_fill_i32(bad, 1, 0, s);
    if (e == hipSuccess) e = pf::launch_search(strategy, cdf_dev, n, u_dev, m, anc_dev, table, bad, s);
    int32_t hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pf_debug_search_noalloc");
    if (hbad) return fail(PF_EINVAL, "CDF is decreasing somewhere or not finite");
    return PF_OK;
}

int pf_debug_particles(pf_filter* f, void* host_out, size_t bytes, int64_t* t_out) {
    if (!f || !host_out) return fail(PF_EINVAL, "NULL argument");
    const int64_t n = f->cfg.n_particles;
    const size_t rec = static_cast<size_t>(f->L.fields) * n * f->L.rsz;
    if (bytes < rec + sizeof(int32_t) * n) return fail(PF_EINVAL, "host buffer too small");
    char* dst = static_cast<char*>(host_out);
    hipError_t e = hipSuccess;
    for (int fld = 0; fld < f->L.fields && e == hipSuccess; ++fld)
        e = hipMemcpyAsync(dst + static_cast<size_t>(fld) * n * f->L.rsz,
                           f->ws + f->L.rec[f->cur] + static_cast<size_t>(fld) * f->L.pitch * f->L.rsz,
                           static_cast<size_t>(n) * f->L.rsz, hipMemcpyDeviceToHost, f->stream);
    if (e == hipSuccess) {
        if (f->cfg.flags & PF_FLAG_KEEP_ANCESTORS)
            e = hipMemcpyAsync(dst + rec, f->ws + f->L.anc, sizeof(int32_t) * n,
                               hipMemcpyDeviceToHost, f->stream);
        else
            std::memset(dst + rec, 0xff, sizeof(int32_t) * n);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_debug_particles");
    if (t_out) *t_out = f->t;
    return PF_OK;
}

// Switched off: the first GPU run of this path (a pitched device-to-host
// copy into pinned memory on a second stream, ordered by events) ended in a
// GPU memory fault whose cause has not been found; until it is, the call
// refuses to run.
constexpr bool kAsyncParticleCopies = false;

int pf_copy_particles_async(pf_filter* f, void* host_dst, size_t bytes, void* copy_stream) {
    if (!kAsyncParticleCopies)
        return fail(PF_EDEVICE, "asynchronous particle copies are switched off");
    if (!f || !host_dst) return fail(PF_EINVAL, "null argument");
    const size_t row = static_cast<size_t>(f->cfg.n_particles) * f->L.rsz;
    const size_t need = row * static_cast<size_t>(f->L.fields);
    if (bytes < need) return fail(PF_EINVAL, "host buffer smaller than the particle record");
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; ++b)
        if (!f->copy_ev[b]) e = hipEventCreateWithFlags(&f->copy_ev[b], hipEventDisableTiming);
    if (e == hipSuccess && !f->step_ev) e = hipEventCreateWithFlags(&f->step_ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "pf_copy_particles_async event");
    const hipStream_t cs = static_cast<hipStream_t>(copy_stream);
    const int b = f->cur;
    e = hipEventRecord(f->step_ev, f->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, f->step_ev, 0);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(host_dst, row, f->ws + f->L.rec[b],
                             static_cast<size_t>(f->L.pitch) * f->L.rsz, row,
                             static_cast<size_t>(f->L.fields), hipMemcpyDeviceToHost, cs);
    if (e == hipSuccess) e = hipEventRecord(f->copy_ev[b], cs);
    if (e != hipSuccess) return hip_fail(e, "pf_copy_particles_async");
    f->copy_pending[b] = true;
    return PF_OK;
}

namespace {
// A filter may join a batch of this model, precision and tile size.
int check_member(const pf_filter* f, int model, int precision, int ipt) {
    if (!f) return fail(PF_EINVAL, "filter is NULL");
    if (f->cfg.model != model || f->cfg.precision != precision || f->L.ipt != ipt)
        return fail(PF_EINVAL, "a batch needs one model, precision and items_per_thread");
    if (f->L.lookback) return fail(PF_EINVAL, "batched filters use the tile scan");
    if (f->L.spacings)
        return fail(PF_EINVAL, "sorted multinomial filters are stepped alone (not in batches)");
    return PF_OK;
}
}  // namespace

namespace {
// Entries of a tile map allocated for `tiles` global tiles (with slack, so
// that members joining later rarely force a new allocation).
int64_t map_capacity(int64_t tiles) {
    return std::max<int64_t>(tiles, 2 * (tiles / 2 + 512));
}
}  // namespace

size_t pf_batch_bytes(int32_t capacity, int32_t ring, int64_t tiles) {
    if (capacity < 1 || tiles < 0) return 0;
    if (ring < 1) ring = 64;
    const size_t descs = sizeof(pf::StepArgs) * static_cast<size_t>(ring) * capacity;
    const size_t base = sizeof(int32_t) * (static_cast<size_t>(capacity) + 1);
    const size_t map = tiles > 0 ? sizeof(int2) * static_cast<size_t>(map_capacity(tiles)) : 0;
    return descs + base + map + sizeof(pf::BatchState);
}

int pf_batch_update(pf_batch* b, pf_filter* const* filters, int32_t n) {
    if (!b) return fail(PF_EINVAL, "batch is NULL");
    if (n < 0 || n > b->capacity || (n > 0 && !filters))
        return fail(PF_EINVAL, "need 0 <= n <= the batch's capacity filters");
    const int precision = b->fp64 ? PF_FP64 : PF_FP32;
    for (int32_t i = 0; i < n; ++i) {
        const int rc = check_member(filters[i], b->model, precision, b->ipt);
        if (rc != PF_OK) return rc;
        for (int32_t k = 0; k < i; ++k)
            if (filters[k] == filters[i]) return fail(PF_EINVAL, "a filter appears twice in the batch");
    }
    // work already queued on the members' own streams finishes first
    for (int32_t i = 0; i < n; ++i) {
        if (filters[i]->stream == b->stream) continue;
        const hipError_t se = hipStreamSynchronize(filters[i]->stream);
        if (se != hipSuccess) return hip_fail(se, "pf_batch_update synchronise");
    }
    std::vector<int32_t> base(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (static_cast<int64_t>(base[i]) + filters[i]->L.num_tiles > INT32_MAX)
            return fail(PF_EINVAL, "too many tiles in one batch");
        base[i + 1] = base[i] + filters[i]->L.num_tiles;
    }
    hipError_t e = hipSuccess;
    if (base[n] > b->map_cap) {
        // a larger tile map: steps already queued still read the old one,
        // and the captured graph holds its address (captured again below)
        e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, "pf_batch_update synchronise");
        if (b->exec) {
            hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->d_map) hipFree(b->d_map);
        b->d_map = nullptr;
        b->map_cap = 0;
        const int64_t cap = map_capacity(base[n]);
        e = hipMalloc(reinterpret_cast<void**>(&b->d_map), sizeof(int2) * static_cast<size_t>(cap));
        if (e != hipSuccess) return fail(PF_ENOMEM, "pf_batch_update: hipMalloc of the tile map failed");
        b->map_cap = cap;
    }
    // a pinned block whose previous copy has completed (kMemberSlots updates ago)
    const int k = b->member_next;
    b->member_next = (k + 1) % pf_batch::kMemberSlots;
    e = hipEventSynchronize(b->member_copied[k]);
    if (e != hipSuccess) return hip_fail(e, "pf_batch_update wait");
    int32_t* blk = b->h_member + static_cast<size_t>(k) * b->member_block_ints();
    std::memcpy(blk, base.data(), sizeof(int32_t) * (n + 1));
    const pf_batch::MemberTail tail{n, b->capacity, base[n]};
    int32_t* tail_at = blk + b->capacity + 2;
    std::memcpy(tail_at, &tail, sizeof(tail));
    e = hipMemcpyAsync(b->d_base, blk, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&b->d_state->n_filters, tail_at, sizeof(tail), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->member_copied[k], b->stream);
    if (e == hipSuccess) e = pf::launch_batch_map(b->d_base, n, b->d_map, b->stream);
    if (e != hipSuccess) return hip_fail(e, "pf_batch_update copy");
    b->fs.assign(filters, filters + n);
    b->total_tiles = base[n];
    return PF_OK;
}

int pf_batch_create(pf_filter* const* filters, int32_t n, int32_t capacity, int32_t ring,
                    pf_batch** out) {
    if (!out) return fail(PF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!filters || n < 1) return fail(PF_EINVAL, "need at least one filter");
    if (capacity < n) capacity = n;
    if (ring < 1) ring = 64;
    const pf_filter* f0 = filters[0];
    int rc = check_member(f0, f0 ? f0->cfg.model : 0, f0 ? f0->cfg.precision : 0,
                          f0 ? f0->L.ipt : 0);
    if (rc != PF_OK) return rc;
    pf_batch* b = new (std::nothrow) pf_batch();
    if (!b) return fail(PF_ENOMEM, "host allocation failed");
    b->stream = f0->stream;
    b->model = f0->cfg.model;
    b->fp64 = f0->cfg.precision == PF_FP64;
    b->ipt = f0->L.ipt;
    b->ring = ring;
    b->capacity = capacity;
    const size_t ring_bytes = sizeof(pf::StepArgs) * static_cast<size_t>(ring) * capacity;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->d_descs), ring_bytes);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&b->d_base), sizeof(int32_t) * (capacity + 1));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b->d_state), sizeof(pf::BatchState));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_stage), ring_bytes, 0);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_member),
                          sizeof(int32_t) * pf_batch::kMemberSlots * b->member_block_ints(), 0);
    b->slot_copied.assign(ring, nullptr);
    for (int32_t i = 0; i < ring && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&b->slot_copied[i], hipEventDisableTiming);
    for (int i = 0; i < pf_batch::kMemberSlots && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&b->member_copied[i], hipEventDisableTiming);
    if (e == hipSuccess) {
        pf::BatchState bs{};
        bs.ring = static_cast<uint32_t>(ring);
        bs.capacity = capacity;
        // pageable source; the synchronisation below completes the copy
        e = hipMemcpyAsync(b->d_state, &bs, sizeof(bs), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        pf_batch_destroy(b);
        return hip_fail(e, "pf_batch_create");
    }
    rc = pf_batch_update(b, filters, n);
    if (rc != PF_OK) {
        pf_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PF_OK;
}

int pf_batch_step(pf_batch* b, const double* y, int64_t n_steps) {
    if (!b) return fail(PF_EINVAL, "batch is NULL");
    if (!y || n_steps < 1) return fail(PF_EINVAL, "need n_steps >= 1 observations per filter");
    const int64_t n = static_cast<int64_t>(b->fs.size());
    if (n == 0) return PF_OK;  // an empty batch has nothing to step
    const int64_t cap = b->capacity;
    for (int64_t i = 0; i < n * n_steps; ++i)
        if (!std::isfinite(y[i])) return fail(PF_EINVAL, "observation is not finite");
    // members' particles still being copied to the host are overwritten by
    // the batched steps: wait for those copies first
    for (pf_filter* f : b->fs) {
        const int rc = f->wait_copies(b->stream);
        if (rc != PF_OK) return rc;
    }
    hipError_t e = hipSuccess;
    if (!b->exec) {
        // capture one batched cycle (its arguments come from the device ring)
        // on a private stream: the filters' stream may be the null stream,
        // which cannot capture; the graph is then launched on that stream
        hipGraph_t g = nullptr;
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            // one work-group per entry of the tile map (those beyond the
            // members' tiles return at once); a larger map is captured anew
            hipError_t le = pf::launch_batch(b->model, b->fp64, b->ipt, b->d_descs, b->d_map,
                                             b->capacity, b->d_state,
                                             static_cast<int>(b->map_cap), cs);
            e = hipStreamEndCapture(cs, &g);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (cs) hipStreamDestroy(cs);
        if (e != hipSuccess) return hip_fail(e, "batch graph capture");
    }
    int64_t done = 0;
    while (done < n_steps) {
        // stage up to `ring` steps at once (the previous staging copy must
        // have been consumed before the pinned buffer is rewritten)
        const int64_t chunk = std::min<int64_t>(b->ring, n_steps - done);
        const uint64_t first = b->issued;
        for (int64_t s = 0; s < chunk; ++s) {
            const uint64_t slot = (first + s) % static_cast<uint64_t>(b->ring);
            // the copy that last read this pinned slot (ring steps ago) is done
            e = hipEventSynchronize(b->slot_copied[slot]);
            if (e != hipSuccess) return hip_fail(e, "batch staging wait");
            for (int64_t i = 0; i < n; ++i)
                b->h_stage[slot * cap + i] = b->fs[i]->prepare_obs(y[(done + s) * n + i]);
        }
        // the slots [first, first+chunk) mod ring: only their first n
        // descriptors are live, so a batch running below its capacity copies
        // n per slot (one copy per slot), a full one whole runs of slots
        // (at most two pieces)
        const uint64_t s0 = first % static_cast<uint64_t>(b->ring);
        const uint64_t c0 = std::min<uint64_t>(chunk, b->ring - s0);
        if (n == cap) {
            e = hipMemcpyAsync(b->d_descs + s0 * cap, b->h_stage + s0 * cap,
                               sizeof(pf::StepArgs) * c0 * cap, hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess && c0 < static_cast<uint64_t>(chunk))
                e = hipMemcpyAsync(b->d_descs, b->h_stage,
                                   sizeof(pf::StepArgs) * (chunk - c0) * cap,
                                   hipMemcpyHostToDevice, b->stream);
        } else {
            for (int64_t s = 0; s < chunk && e == hipSuccess; ++s) {
                const uint64_t slot = (first + s) % static_cast<uint64_t>(b->ring);
                e = hipMemcpyAsync(b->d_descs + slot * cap, b->h_stage + slot * cap,
                                   sizeof(pf::StepArgs) * n, hipMemcpyHostToDevice, b->stream);
            }
        }
        for (int64_t s = 0; s < chunk && e == hipSuccess; ++s)
            e = hipEventRecord(b->slot_copied[(first + s) % static_cast<uint64_t>(b->ring)],
                               b->stream);
        for (int64_t s = 0; s < chunk && e == hipSuccess; ++s) e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch step");
        b->issued += chunk;
        done += chunk;
    }
    return PF_OK;
}

int pf_batch_destroy(pf_batch* b) {
    if (!b) return PF_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (b->exec) hipGraphExecDestroy(b->exec);
    for (hipEvent_t ev : b->slot_copied)
        if (ev) hipEventDestroy(ev);
    for (hipEvent_t ev : b->member_copied)
        if (ev) hipEventDestroy(ev);
    if (b->h_stage) hipHostFree(b->h_stage);
    if (b->h_member) hipHostFree(b->h_member);
    if (b->d_descs) hipFree(b->d_descs);
    if (b->d_base) hipFree(b->d_base);
    if (b->d_map) hipFree(b->d_map);
    if (b->d_state) hipFree(b->d_state);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "pf_batch_destroy synchronise");
    return PF_OK;
}

int pf_step_batch(pf_filter* const* filters, int32_t n, const double* y_each) {
    pf_batch* b = nullptr;
    int rc = pf_batch_create(filters, n, n, 1, &b);
    if (rc != PF_OK) return rc;
    rc = pf_batch_step(b, y_each, 1);
    const int rc2 = pf_batch_destroy(b);
    return rc != PF_OK ? rc : rc2;
}

}  // extern "C"
