// HIP kernels of the particle-filter cycle for gfx950 (wave64).
//
// One launch of k_step advances a filter by one cycle (Section 3.2: the whole
// cycle runs in parallel on the device):
//   1. each output slot j forms its resampling uniform u_j (Section 3.1) and
//      finds its ancestor a_j = min{k : q(k) >= u_j} in the previous step's
//      CDF (Section 3.2), either cooperatively for a tile of sorted uniforms
//      (merge against the CDF staged in LDS), by the paper's cut-point table
//      built in LDS, or by bisection;
//   2. gathers the ancestor's record from the structure-of-arrays buffer,
//      propagates it (and, for particle learning, updates its statistics and
//      draws its parameters) and writes the new record;
//   3. scores the new particle (log-weight), takes the tile's max-shifted
//      sum of exp(l - m) and its in-tile inclusive prefix (the CDF, equation
//      (resample.cdf), up to the tile's offset and the global normaliser).
// The tile prefixes over all tiles then come from one of two scans:
//   - tile scan (default): every tile stores its (max, sum); k_scan_tiles, a
//     single work-group, scans them in a fixed order, normalises them into
//     per-tile affine constants (q = a + c[k] b), forms the log-likelihood
//     increment and, for sorted uniforms, the source tile of every output
//     tile's first uniform (search hints);
//   - decoupled look-back: each tile obtains its exclusive prefix inside
//     k_step from the (max, sum) aggregates of its predecessors, and the
//     tile with the last ticket forms the totals.
// The normalised CDF is never materialised.
#include <hip/hip_runtime.h>

#include <mutex>
#include <math.h>
#include <stdint.h>

#include "pf_internal.h"
#include "pf_models.hpp"

namespace pf {

constexpr int kWave = 64;
// Largest CDF whose cut-point table is built in LDS by the cycle kernel.
constexpr int kCutMax = 2048;
// A tile's sorted uniforms are merged against at most this many LDS windows
// of the CDF; a wider bracket (a long run of near-zero weights inside it,
// Section 3.2's worst case) is searched by bisection per uniform instead.
constexpr int kMaxWindows = 16;
// Predecessor tiles each lane inspects per look-back round.
constexpr int kLookPer = 4;

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Pointers typed in the global address space.  A buffer pointer read from
// device memory (a batch's per-filter arguments) is generic to the compiler,
// which then emits flat accesses with 64-bit vector addresses; every buffer
// of a filter is device global memory, so the cycle accesses them through
// these types (global loads and stores with a scalar base).
// (The host pass of the compiler only checks device code; it sees plain
// types.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using G = __attribute__((address_space(1))) T;
#else
template <typename T>
using G = T;
#endif
template <typename T>
__device__ __forceinline__ G<T>* gp(T* p) {
    return (G<T>*)p;
}

// A value the whole work-group holds (read back from LDS), marked as
// wave-uniform so that addresses derived from it stay in scalar registers.
__device__ __forceinline__ uint32_t uniform32(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint64_t u = static_cast<uint64_t>(v);
    const uint64_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint64_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((hi << 32) | lo);
}

// Cross-lane moves of a double through the VALU's data-parallel primitives
// (DPP: two 32-bit moves, no LDS round trip).  Lanes whose source lies
// outside the pattern, or whose row is masked off, receive `old`.
constexpr int kDppRowShr = 0x110;     // + k: from lane - k of the same 16-lane row
constexpr int kDppRowBcast15 = 0x142; // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143; // lane 31 to rows 2 and 3
constexpr int kDppWaveShr1 = 0x138;   // from lane - 1 across the wave

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const uint64_t o = static_cast<uint64_t>(__double_as_longlong(old));
    const uint64_t x = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        static_cast<int>(static_cast<uint32_t>(o)), static_cast<int>(static_cast<uint32_t>(x)),
        CTRL, ROW_MASK, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        static_cast<int>(static_cast<uint32_t>(o >> 32)),
        static_cast<int>(static_cast<uint32_t>(x >> 32)), CTRL, ROW_MASK, 0xF, false));
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// The value of lane 63, in every lane (a wave-uniform scalar).
__device__ __forceinline__ double lane63(double v) {
    const uint64_t x = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(x)), kWave - 1));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(x >> 32)), kWave - 1));
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// Inclusive prefix sum over the wave: Hillis-Steele within each 16-lane row,
// then the row totals carried across rows.
__device__ __forceinline__ double wave_incl_sum(double v) {
    v += dpp_f64<kDppRowShr + 1, 0xF>(0.0, v);
    v += dpp_f64<kDppRowShr + 2, 0xF>(0.0, v);
    v += dpp_f64<kDppRowShr + 4, 0xF>(0.0, v);
    v += dpp_f64<kDppRowShr + 8, 0xF>(0.0, v);
    v += dpp_f64<kDppRowBcast15, 0xA>(0.0, v);
    v += dpp_f64<kDppRowBcast31, 0xC>(0.0, v);
    return v;
}

__device__ __forceinline__ double wave_incl_max(double v) {
    constexpr double lo = -INFINITY;
    v = fmax(v, dpp_f64<kDppRowShr + 1, 0xF>(lo, v));
    v = fmax(v, dpp_f64<kDppRowShr + 2, 0xF>(lo, v));
    v = fmax(v, dpp_f64<kDppRowShr + 4, 0xF>(lo, v));
    v = fmax(v, dpp_f64<kDppRowShr + 8, 0xF>(lo, v));
    v = fmax(v, dpp_f64<kDppRowBcast15, 0xA>(lo, v));
    v = fmax(v, dpp_f64<kDppRowBcast31, 0xC>(lo, v));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return lane63(wave_incl_sum(v)); }

// Wave maximum in the weights' precision (single precision: one 32-bit
// move per step), returned in double precision in every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                      ROW_MASK, 0xF, false));
}
__device__ __forceinline__ double wave_max_r(float v) {
    constexpr float lo = -INFINITY;
    v = fmaxf(v, dpp_f32<kDppRowShr + 1, 0xF>(lo, v));
    v = fmaxf(v, dpp_f32<kDppRowShr + 2, 0xF>(lo, v));
    v = fmaxf(v, dpp_f32<kDppRowShr + 4, 0xF>(lo, v));
    v = fmaxf(v, dpp_f32<kDppRowShr + 8, 0xF>(lo, v));
    v = fmaxf(v, dpp_f32<kDppRowBcast15, 0xA>(lo, v));
    v = fmaxf(v, dpp_f32<kDppRowBcast31, 0xC>(lo, v));
    return static_cast<double>(
        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1)));
}
__device__ __forceinline__ double wave_max_r(double v) { return lane63(wave_incl_max(v)); }

// Sum over each half wave (lanes 0-31 and 32-63), left in lanes 31 and 63.
__device__ __forceinline__ double half_wave_sum(double v) {
    v += dpp_f64<kDppRowShr + 1, 0xF>(0.0, v);
    v += dpp_f64<kDppRowShr + 2, 0xF>(0.0, v);
    v += dpp_f64<kDppRowShr + 4, 0xF>(0.0, v);
    v += dpp_f64<kDppRowShr + 8, 0xF>(0.0, v);
    v += dpp_f64<kDppRowBcast15, 0xA>(0.0, v);
    return v;
}
__device__ __forceinline__ double wave_max(double v) { return lane63(wave_incl_max(v)); }

// The previous lane's value (lane 0 receives `first`).
__device__ __forceinline__ double wave_shr1(double v, double first) {
    return dpp_f64<kDppWaveShr1, 0xF>(first, v);
}

// (max, sum of exp(l - max)) monoid of the max-shifted log-sum-exp.
struct Agg {
    double m, s;
};
__device__ __forceinline__ Agg agg_identity() { return {-INFINITY, 0.0}; }
__device__ __forceinline__ Agg agg_combine(Agg a, Agg b) {
    if (a.m == -INFINITY) return b;
    if (b.m == -INFINITY) return a;
    const double m = fmax(a.m, b.m);
    return {m, a.s * exp(a.m - m) + b.s * exp(b.m - m)};
}
__device__ __forceinline__ Agg wave_agg(Agg v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Agg o{__shfl_xor(v.m, off, kWave), __shfl_xor(v.s, off, kWave)};
        v = agg_combine(v, o);
    }
    return v;
}

// A tile scan inside the cycle kernel (the fused scan of the last
// work-group, the look-back) waits at most this many polls (each followed by
// a short sleep) for one tile's words before it reports a stall.
constexpr uint32_t kFusedScanSpins = 1u << 22;
// The same waits under PF_FLAG_TEST_SCAN_STALL.
constexpr uint32_t kTestSpins = 64;

// ------------------------------------------------------------ look-back words
// Each 64-bit word = (epoch << 32) | 32 payload bits; relaxed agent-scope
// atomics keep every word single-copy atomic and coherent across the XCDs'
// L2s without a release/acquire fence (which would write back the L2).
__device__ __forceinline__ void put_word(uint64_t* p, uint32_t epoch, uint32_t bits) {
    __hip_atomic_store(p, (static_cast<uint64_t>(epoch) << 32) | bits, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t get_word(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put_agg(uint64_t* p, uint32_t epoch, Agg a) {
    const uint64_t mb = __double_as_longlong(a.m), sb = __double_as_longlong(a.s);
    put_word(p + 0, epoch, static_cast<uint32_t>(mb));
    put_word(p + 1, epoch, static_cast<uint32_t>(mb >> 32));
    put_word(p + 2, epoch, static_cast<uint32_t>(sb));
    put_word(p + 3, epoch, static_cast<uint32_t>(sb >> 32));
}
// Returns true (and the value) when all four words carry `epoch`.
__device__ __forceinline__ bool get_agg(const uint64_t* p, uint32_t epoch, Agg& a) {
    const uint64_t w0 = get_word(p + 0), w1 = get_word(p + 1);
    const uint64_t w2 = get_word(p + 2), w3 = get_word(p + 3);
    const uint64_t tag = static_cast<uint64_t>(epoch);
    if ((w0 >> 32) != tag || (w1 >> 32) != tag || (w2 >> 32) != tag || (w3 >> 32) != tag)
        return false;
    a.m = __longlong_as_double(static_cast<long long>((w0 & 0xffffffffull) | (w1 << 32)));
    a.s = __longlong_as_double(static_cast<long long>((w2 & 0xffffffffull) | (w3 << 32)));
    return true;
}

// ------------------------------------------------------------ CDF of the previous step
// q(k) = A_b + c[k] B_b for k in tile b.  A_b, B_b come either from the
// tile-scan table (ab != nullptr) or from the look-back's (max, sum) form.
template <typename R>
struct PrevCdf {
    G<const R>* c;
    G<const TileInfo>* tiles;
    G<const TileAB>* ab;
    double M, S;
    int64_t n;
    int32_t ts;  // elements per tile

    __device__ __forceinline__ void tile_ab(int64_t b, double& ta, double& tb) const {
        if (ab) {
            const TileAB v = ab[b];
            ta = v.a;
            tb = v.b;
        } else {
            const TileInfo ti = tiles[b];
            ta = ti.s_ex == 0.0 ? 0.0 : ti.s_ex * exp(ti.m_ex - M) / S;
            tb = exp(ti.m_b - M) / S;
        }
    }
    // q(k); the last entry is 1 by definition (equation resample.cdf).
    __device__ __forceinline__ double at(int64_t k) const {
        if (k >= n - 1) return 1.0;
        double ta, tb;
        tile_ab(k / ts, ta, tb);
        return fma(static_cast<double>(c[k]), tb, ta);
    }
};

struct PlainCdf {
    const double* q;
    int64_t n;
    __device__ __forceinline__ double at(int64_t k) const { return q[k]; }
};

// First k in [lo, hi] with q(k) >= u, or hi if none, found by one wave with
// 64 strided probes per round.
template <typename CDF>
__device__ int64_t wave_search(const CDF& cdf, double u, int64_t lo, int64_t hi) {
    const int lane = lane_id();
    while (hi > lo) {
        const int64_t len = hi - lo + 1;
        const int64_t stride = (len + kWave - 1) / kWave;
        int64_t k = lo + static_cast<int64_t>(lane) * stride;
        if (k > hi) k = hi;
        const bool ge = cdf.at(k) >= u;
        const uint64_t mask = __ballot(ge);
        if (stride == 1) {
            return mask ? lo + static_cast<int64_t>(__ffsll(static_cast<long long>(mask)) - 1) : hi;
        }
        if (mask == 0) {
            const int64_t last = lo + static_cast<int64_t>(kWave - 1) * stride;
            if (last >= hi) return hi;
            lo = last + 1;
        } else {
            const int first = __ffsll(static_cast<long long>(mask)) - 1;
            const int64_t kf = lo + static_cast<int64_t>(first) * stride;
            hi = kf > hi ? hi : kf;
            if (first > 0) lo = lo + static_cast<int64_t>(first - 1) * stride + 1;
        }
    }
    return lo;
}

// Bisection by one thread: first k in [lo, hi] with q(k) >= u, else hi.
template <typename CDF>
__device__ int64_t thread_search(const CDF& cdf, double u, int64_t lo, int64_t hi) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (cdf.at(mid) >= u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// First index in s_q[0, cnt) with value >= u, or cnt.
__device__ __forceinline__ int lds_lower_bound(const double* s_q, int cnt, double u) {
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_q[mid] >= u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Tile constants the bracket search already read (the hint tiles of the
// tile's first and last uniforms) and the first one's last value q, kept
// in LDS so that the first window over those tiles skips its own loads.
struct WindowPre {
    int64_t h[2];  // source tiles, -1: none
    double ta[2], tb[2];
    double last0;  // q at tile h[0]'s last element
};

// Stage q(w0 .. w0+cnt-1) in LDS, non-decreasing.  Inside a tile the stored
// prefix is non-decreasing and q = A_b + c[k] B_b (one fma, B_b >= 0) keeps
// that order; across tiles rounding of the affine constants can leave a
// tile's first value an ulp below its predecessor's last, so every value is
// raised to the largest last value of the window's earlier tiles (and to
// `floor`, the previous window's top).  Loads are coalesced.  Ends with a
// barrier.
template <int BLOCK, typename R>
__device__ void stage_window(const PrevCdf<R>& P, int64_t w0, int cnt, double floor, double* s_q,
                             double* s_ta, double* s_tb, double* s_last,
                             const WindowPre* pre = nullptr) {
    const int tid = threadIdx.x;
    const int64_t b0 = w0 / P.ts, b1 = (w0 + cnt - 1) / P.ts;
    const int nb = static_cast<int>(b1 - b0 + 1);
    // a window over one preloaded tile, or over the two consecutive
    // preloaded tiles, needs no loads of its own (and no barrier for them)
    int pa = -1;
    if (pre && nb <= 2) {
        if (b0 == pre->h[0]) pa = 0;
        else if (nb == 1 && b0 == pre->h[1]) pa = 1;
        if (nb == 2 && !(pa == 0 && b1 == pre->h[1])) pa = -1;
    }
    if (pa < 0) {
        for (int k = tid; k < nb; k += BLOCK) {
            double ta, tb;
            P.tile_ab(b0 + k, ta, tb);
            s_ta[k] = ta;
            s_tb[k] = tb;
            // the tile's last element inside the window
            const int64_t e = min(w0 + cnt - 1, (b0 + k + 1) * P.ts - 1);
            s_last[k] = e >= P.n - 1 ? 1.0 : fma(static_cast<double>(P.c[e]), tb, ta);
        }
        __syncthreads();
    }
    // (a window of two preloaded tiles: the first tile's last element lies
    // below the window's end, so below N - 1, and its q is pre->last0)
    const double* ta_of = pa < 0 ? s_ta : pre->ta + pa;
    const double* tb_of = pa < 0 ? s_tb : pre->tb + pa;
    const double* last_of = pa < 0 ? s_last : &pre->last0;
    // four of the thread's entries per round, their loads issued together
    // (indices clamped to N - 1 keep every load in bounds; entries past cnt
    // are not stored), so that a window costs few memory latencies
    constexpr int kBatch = 4;
    for (int k0 = tid; k0 < cnt; k0 += kBatch * BLOCK) {
        R cv[kBatch];
#pragma unroll
        for (int r = 0; r < kBatch; ++r) cv[r] = P.c[min(w0 + k0 + r * BLOCK, P.n - 1)];
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
            const int k = k0 + r * BLOCK;
            if (k < cnt) {
                const int64_t g = w0 + k;
                const int bb = static_cast<int>(g / P.ts - b0);
                double v = 1.0;
                if (g < P.n - 1) v = fma(static_cast<double>(cv[r]), tb_of[bb], ta_of[bb]);
                double f = floor;
                for (int q = 0; q < bb; ++q) f = fmax(f, last_of[q]);
                s_q[k] = fmax(v, f);
            }
        }
    }
    __syncthreads();
}

// Cut-point table of Section 3.2 built in LDS over s_q[0, n) (the whole
// CDF): with L_j = ceil(n q(j)), element j owns entries L_{j-1}+1 .. L_j
// (1-based) and writes its index there; the last element also owns every
// entry above L_n.  Ends with a barrier.
template <int BLOCK>
__device__ void build_cutpoints(const double* s_q, int n, int* s_cut) {
    const double dn = static_cast<double>(n);
    for (int j = threadIdx.x; j < n; j += BLOCK) {
        double cj = ceil(dn * s_q[j]);
        const int Lj = cj < 0.0 ? 0 : (cj > dn ? n : static_cast<int>(cj));
        int Lp = 0;
        if (j > 0) {
            const double cp = ceil(dn * s_q[j - 1]);
            Lp = cp < 0.0 ? 0 : (cp > dn ? n : static_cast<int>(cp));
        }
        const int top = (j == n - 1) ? n : Lj;
        for (int k = top; k > Lp; --k) s_cut[k - 1] = j;
    }
    __syncthreads();
}

// Cut-point draw (Section 3.2, Algorithm "Parallelized Cut-Point Method"):
// start at I_{ceil(n u)} and climb while u is above the CDF; after 16 climbs
// finish by bisection above the current point (same answer, bounded work).
__device__ __forceinline__ int cutpoint_draw(const double* s_q, const int* s_cut, int n, double u) {
    double ce = ceil(static_cast<double>(n) * u);
    int e = ce < 1.0 ? 1 : (ce > static_cast<double>(n) ? n : static_cast<int>(ce));
    int k = s_cut[e - 1];
    for (int c = 0; c < 16 && k < n - 1 && u > s_q[k]; ++c) ++k;
    if (k < n - 1 && u > s_q[k]) {
        const int r = lds_lower_bound(s_q + k + 1, n - 1 - k, u);
        k = k + 1 + r;
        if (k > n - 1) k = n - 1;
    }
    return k;
}

// Cut-point draw against a table in device memory (the parallelized
// cut-point method of Section 3.2 for CDFs larger than one LDS window):
// start at I_{ceil(n u)}, which the table's construction keeps at or below
// the answer, and climb; after 16 climbs, bisection above the current
// point.  A start whose predecessor already reaches u (possible only through
// rounding where two tiles meet) falls back to bisection below it.
template <typename R>
__device__ __forceinline__ int64_t cut_draw_global(const PrevCdf<R>& P, G<const int32_t>* table,
                                                   double u) {
    const int64_t n = P.n;
    const double ce = ceil(static_cast<double>(n) * u);
    const int64_t e = ce < 1.0 ? 1 : (ce > static_cast<double>(n) ? n : static_cast<int64_t>(ce));
    int64_t k = min(max(static_cast<int64_t>(table[e - 1]), int64_t(0)), n - 1);
    if (k > 0 && P.at(k - 1) >= u) return thread_search(P, u, int64_t(0), k - 1);
    for (int c = 0; c < 16 && k < n - 1 && u > P.at(k); ++c) ++k;
    if (k < n - 1 && u > P.at(k)) k = thread_search(P, u, k + 1, n - 1);
    return k;
}

// Resampling uniform of slot j (Section 3.1), in double precision.  With
// EXACT the stratum position is divided by N (correctly rounded, as the
// double-precision reference does); otherwise it is multiplied by 1/N
// (within an ulp; exact when N is a power of two).
template <bool EXACT>
__device__ __forceinline__ double resample_uniform(int32_t scheme, int64_t j, int64_t n,
                                                   double inv_n, uint32_t w0, double u_sys) {
    if (scheme == kMultinomial) return unit64(w0);
    const double pos = static_cast<double>(j) + (scheme == kStratified ? unit64(w0) : u_sys);
    return EXACT ? pos / static_cast<double>(n) : pos * inv_n;
}

// ------------------------------------------------------------ sorted multinomial
// The branch is compiled into the cycle kernels of every tile size in double
// precision and of 1, 2 and 8 items per thread in single precision; the
// single-precision kernels of 4 items per thread (the large-filter and batch
// kernels) carry none of its code, and the host does not give them the
// scheme.
template <typename R, int IPT>
constexpr bool sorted_kernel() { return sizeof(R) == 8 || IPT != 4; }

// Exponential spacing -log U of a resampling word (double precision).
__device__ __forceinline__ double spacing(uint32_t w0) { return -log(unit64(w0)); }

// Inclusive prefix over a tile in slot order, slots dealt in blocks (thread
// tid holds slots tid * IPT + i in v[i]); v[i] is replaced by its prefix,
// *total receives the tile's sum.  The same order gives the same bits in
// every kernel that calls it.  Ends with a barrier.
template <int BLOCK, int IPT>
__device__ __forceinline__ void tile_incl_prefix(double (&v)[IPT], double* s_red, double* total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        run += v[i];
        v[i] = run;
    }
    const double incl = wave_incl_sum(run);
    __syncthreads();
    if (lane == kWave - 1) s_red[wave] = incl;
    __syncthreads();
    double base = 0.0, tot = 0.0;
    for (int q = 0; q < NW; ++q) {
        if (q == wave) base = tot;
        tot += s_red[q];
    }
    base += wave_shr1(incl, 0.0);
#pragma unroll
    for (int i = 0; i < IPT; ++i) v[i] += base;
    *total = tot;
    __syncthreads();
}

// Each tile's sum of the exponential spacings of time t (slots j0 .. j0+TS-1
// below n; the last tile also adds the spacing of index n), as a (0, sum)
// pair for the tile scan, which then yields the normalised offsets.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_spacing_tiles(uint64_t seed, uint32_t t, int64_t n,
                                                         double* aggE) {
    constexpr int TS = BLOCK * IPT;
    __shared__ double s_red[BLOCK / kWave];
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * TS;
    double v[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t j = j0 + static_cast<int64_t>(threadIdx.x) * IPT + i;
        v[i] = j < n ? spacing(philox(seed, static_cast<uint32_t>(j), t, kStep, 0).w0) : 0.0;
    }
    double tot;
    tile_incl_prefix<BLOCK, IPT>(v, s_red, &tot);
    if (threadIdx.x == 0) {
        if (j0 + TS >= n)
            tot += spacing(philox(seed, static_cast<uint32_t>(n), t, kStep, 0).w0);
        aggE[2 * static_cast<int64_t>(blockIdx.x)] = 0.0;
        aggE[2 * static_cast<int64_t>(blockIdx.x) + 1] = tot;
    }
}

template <int NT, int PER, typename Load>
__device__ __forceinline__ void tile_scan_core(Load load, int32_t num_tiles, int64_t n,
                                               int32_t ts, TileAB* ab, int32_t* hint,
                                               Totals* tot, DevState* st, const TileAB* pos,
                                               double* s_red, double* s_first);

// ------------------------------------------------------------ shared memory
template <int BLOCK, int IPT>
struct StepSmem {
    static constexpr int TS = BLOCK * IPT;
    static constexpr int WIN = 2 * TS;
    static constexpr int NW = BLOCK / kWave;
    double q[WIN];           // staged CDF window; reused for the scan
    int cut[kCutMax];        // cut-point table (CDFs of up to kCutMax entries)
    double ta[8], tb[8];     // per-tile affine constants of the window
    WindowPre pre;           // the bracket's tile constants
    double last[8];          // each window tile's last value
    double red[NW * 16];     // reductions
    int64_t lo, hi;
    double u_first, u_last;  // sorted multinomial: the tile's end uniforms
    uint32_t tile;
    int32_t scan_here;       // fused tile scan: this work-group finished last
    double ex_m, ex_s;
};

// ------------------------------------------------------------ the cycle
// Slots of a tile are dealt to threads in blocks: thread tid holds the IPT
// consecutive slots j0 + tid * IPT + i, i < IPT.  Sorted uniforms of one
// thread then have nearby ancestors (found by a short forward walk from the
// previous one), the records and CDF prefixes a thread writes are contiguous
// (vector stores), and the tile's prefix needs no transposition.

// Streaming store of v[0 .. IPT) to p[0 .. IPT) (p aligned to IPT elements),
// in pieces of up to 16 bytes.
template <typename R, int IPT>
__device__ __forceinline__ void store_run(G<R>* p, const R (&v)[IPT]) {
    constexpr int PIECE = (16 / static_cast<int>(sizeof(R))) < IPT ? 16 / static_cast<int>(sizeof(R))
                                                                    : IPT;
    typedef R VecT __attribute__((ext_vector_type(PIECE)));
#pragma unroll
    for (int i0 = 0; i0 < IPT; i0 += PIECE) {
        VecT x;
#pragma unroll
        for (int k = 0; k < PIECE; ++k) x[k] = v[i0 + k];
        __builtin_nontemporal_store(x, reinterpret_cast<G<VecT>*>(p + i0));
    }
}

// First index in [lo, cnt) of s_q with a value >= u, clamped to cnt - 1,
// for a caller that knows no index below lo qualifies (the previous, smaller
// uniform of the same thread ended at lo): a short walk, then bisection.
// Equal to min(lds_lower_bound(s_q, cnt, u), cnt - 1).
__device__ __forceinline__ int lds_walk(const double* s_q, int lo, int cnt, double u) {
    int k = lo;
    for (int s = 0; s < 8 && k < cnt - 1 && s_q[k] < u; ++s) ++k;
    if (k < cnt - 1 && s_q[k] < u) k = k + 1 + lds_lower_bound(s_q + k + 1, cnt - 2 - k, u);
    return k < cnt - 1 ? k : cnt - 1;
}

// One tile of one filter's cycle (the work of one work-group).
template <int MODEL, typename R, int BLOCK, int IPT>
__device__ __forceinline__ void cycle(const StepArgs& A, uint32_t tile,
                                      StepSmem<BLOCK, IPT>& sm) {
    using MD = ModelDef<MODEL>;
    constexpr int F = MD::F, NG = MD::NG;
    constexpr int TS = BLOCK * IPT, NW = BLOCK / kWave;
    constexpr int WIN = StepSmem<BLOCK, IPT>::WIN;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const bool weight = (A.flags & kWeight) != 0;
    const bool resample = (A.flags & kResample) != 0;
    const bool propagate = (A.flags & kPropagate) != 0;
    const bool weighted_mom = (A.flags & kWeightedMoments) != 0;
    const bool lookback = weight && A.scan == kScanLookback;
    const int64_t n = A.n;
    const int64_t j0 = static_cast<int64_t>(tile) * TS;
    // first slot of this thread's block
    const int64_t jt = j0 + static_cast<int64_t>(tid) * IPT;

    // ---------------------------------------------------------- 1. ancestors
    // The resampling's first reads (the previous CDF's totals and, for the
    // merge search over the tile table, the hints of this tile and the
    // next) are issued before the random words are formed, so their latency
    // overlaps that work.
    const bool merge_indexed =
        resample && A.scan == kScanTiles && A.strategy == kMerge && n > WIN;
    int32_t hint_pre = 0;
    if (merge_indexed && wave < 2) hint_pre = gp(A.hint_in)[tile + wave];
    double tot_M = 0.0, tot_S = 0.0;
    if (resample) {
        const Totals tt = *gp(A.tot_in);
        tot_M = tt.M;
        tot_S = tt.S;
    }
    Words w[IPT];
    int32_t anc[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t j = jt + i;
        anc[i] = static_cast<int32_t>(j < n ? j : n - 1);
        if (propagate && j < n) w[i] = philox(A.seed, static_cast<uint32_t>(j), A.t, kStep, 0);
        else w[i] = {0u, 0u, 0u, 0u};
    }
    if (resample) {
        PrevCdf<R> P{gp(static_cast<const R*>(A.c_in)), gp(A.tiles_in),
                     A.scan == kScanTiles ? gp(A.ab_in) : nullptr, tot_M, tot_S, n, TS};
        const bool ok = (P.S > 0.0) && isfinite(P.S) && isfinite(P.M);
        if (!ok) {
            if (tid == 0) atomicOr(&A.st->flags, kDegenerate);
        } else {
            constexpr bool kExact = sizeof(R) == 8;
            const double inv_n = 1.0 / static_cast<double>(n);
            double u_sys = 0.0;
            if (A.scheme == kSystematicScheme)
                u_sys = unit64(philox(A.seed, 0, A.t, kSystematic, 0).w0);
            double u[IPT];
            const int64_t jlast = min(j0 + TS, n) - 1;
            const bool sorted_mult = sorted_kernel<R, IPT>() && A.scheme == kSortedMultinomial;
            // the uniforms rise with the slot (a thread's own ones too)
            const bool sorted_u = A.scheme != kMultinomial;
            if (sorted_mult) {
                // order statistics from exponential spacings: the tile's
                // offset and scale come from the spacings' tile scan
#pragma unroll
                for (int i = 0; i < IPT; ++i) u[i] = jt + i < n ? spacing(w[i].w0) : 0.0;
                double tot;
                tile_incl_prefix<BLOCK, IPT>(u, sm.red, &tot);
                const TileAB e = gp(A.abE)[tile];
#pragma unroll
                for (int i = 0; i < IPT; ++i) u[i] = fma(u[i], e.b, e.a);
                const int64_t last_off = jlast - j0;
                if (tid == 0) sm.u_first = u[0];
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (static_cast<int64_t>(tid) * IPT + i == last_off) sm.u_last = u[i];
                __syncthreads();
            } else {
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    u[i] = resample_uniform<kExact>(A.scheme, jt + i, n, inv_n, w[i].w0, u_sys);
            }
            const int strategy = A.strategy;
            if (n <= WIN && strategy != kBinary) {
                // the whole CDF fits one LDS window
                stage_window<BLOCK>(P, 0, static_cast<int>(n), -INFINITY, sm.q, sm.ta, sm.tb, sm.last);
                if (strategy == kCutpoint) build_cutpoints<BLOCK>(sm.q, static_cast<int>(n), sm.cut);
                int kprev = -1;
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    int k;
                    if (strategy == kCutpoint) {
                        k = cutpoint_draw(sm.q, sm.cut, static_cast<int>(n), u[i]);
                    } else if (sorted_u && kprev >= 0) {
                        k = lds_walk(sm.q, kprev, static_cast<int>(n), u[i]);
                    } else {
                        k = lds_lower_bound(sm.q, static_cast<int>(n), u[i]);
                        if (k > n - 1) k = static_cast<int>(n - 1);
                    }
                    kprev = k;
                    if (jt + i < n) anc[i] = k;
                }
                __syncthreads();
            } else if (strategy == kMerge) {
                // sorted uniforms: the tile's ancestors lie in [a(u_first), a(u_last)].
                // With the tile-scan table, the hints bound them to the source
                // tiles of CDF positions j0/N and (j0+TS)/N (one tile of slack
                // either side for rounding); otherwise search the whole CDF.
                const bool indexed = A.scan == kScanTiles;
                // (the tile's first uniform is thread 0's first; the last one
                // takes a Philox block only where the scheme draws per slot)
                const double u0 = __shfl(u[0], 0);
                if (wave == 0 || wave == 1) {
                    const int64_t js = wave == 0 ? j0 : jlast;
                    double us;
                    if (sorted_mult) {
                        us = wave == 0 ? sm.u_first : sm.u_last;
                    } else if (wave == 0) {
                        us = u0;
                    } else {
                        const uint32_t wj = A.scheme == kSystematicScheme
                                                ? 0u
                                                : philox(A.seed, static_cast<uint32_t>(js), A.t,
                                                         kStep, 0).w0;
                        us = resample_uniform<kExact>(A.scheme, js, n, inv_n, wj, u_sys);
                    }
                    int64_t a;
                    if (indexed) {
                        // the hint names the source tile of CDF position js/N;
                        // its segment samples bracket u to one segment
                        constexpr int SEG = TS / kSegments;
                        const int64_t tmax = A.num_tiles - 1;
                        const int64_t h = min(max(int64_t(hint_pre), int64_t(0)), tmax);
                        double ta, tb;
                        P.tile_ab(h, ta, tb);
                        G<const R>* samp = gp(static_cast<const R*>(A.samp_in));
                        const double qs = fma(static_cast<double>(samp[h * kSegments + lane]), tb, ta);
                        // (kept for the first window: the tile's constants,
                        // and the last segment's end, which is the tile's end)
                        if (lane == 0) {
                            sm.pre.h[wave] = h;
                            sm.pre.ta[wave] = ta;
                            sm.pre.tb[wave] = tb;
                        }
                        if (wave == 0 && lane == kSegments - 1) sm.pre.last0 = qs;
                        const uint64_t mask = __ballot(qs >= us);
                        const int f = mask ? __ffsll(static_cast<long long>(mask)) - 1 : kSegments;
                        if (wave == 0) {
                            // every segment before f ends below u_first
                            a = h * TS + static_cast<int64_t>(f) * SEG;
                        } else {
                            // segment f ends at or above u_last
                            a = mask ? h * TS + static_cast<int64_t>(f + 1) * SEG - 1
                                     : (h + 2) * TS - 1;
                        }
                        a = min(max(a, int64_t(0)), n - 1);
                    } else {
                        a = wave_search(P, us, int64_t(0), n - 1);
                        if (lane == 0) sm.pre.h[wave] = -1;
                    }
                    if (lane == 0) {
                        if (wave == 0) sm.lo = a; else sm.hi = a;
                    }
                }
                __syncthreads();
                // (a_hi < a_lo only if the CDF were decreasing; keep one window)
                const int64_t a_lo = sm.lo, a_hi = max(sm.hi, sm.lo);
                if (a_hi - a_lo + 1 > static_cast<int64_t>(kMaxWindows) * WIN) {
                    // a bracket of more than kMaxWindows windows (a long run of
                    // near-zero weights between the tile's first and last
                    // ancestors): bisection per uniform over the whole CDF,
                    // O(log N) per slot instead of O(run / window)
#pragma unroll
                    for (int i = 0; i < IPT; ++i)
                        if (jt + i < n) anc[i] = static_cast<int32_t>(thread_search(P, u[i], 0, n - 1));
                } else {
                uint32_t pending = 0;
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (jt + i < n) pending |= 1u << i;
                double floor = -INFINITY;
                for (int64_t w0 = a_lo; w0 <= a_hi; w0 += WIN) {
                    const int cnt = static_cast<int>(min(static_cast<int64_t>(WIN), a_hi - w0 + 1));
                    stage_window<BLOCK>(P, w0, cnt, floor, sm.q, sm.ta, sm.tb, sm.last,
                                        w0 == a_lo ? &sm.pre : nullptr);
                    const bool last = (w0 + cnt - 1 == a_hi);
                    const double top = sm.q[cnt - 1];
                    const bool first = (w0 == a_lo);
                    // window index of the previous item's ancestor when it
                    // was found in this window (the next one lies at or above)
                    int kprev = -1;
#pragma unroll
                    for (int i = 0; i < IPT; ++i) {
                        if ((pending >> i) & 1u) {
                            if (last || u[i] <= top) {
                                int64_t k;
                                if (first && a_lo > 0 && u[i] <= sm.q[0] && P.at(a_lo - 1) >= u[i]) {
                                    // the bracket was too high (rounding): exact search below
                                    k = thread_search(P, u[i], int64_t(0), a_lo - 1);
                                    kprev = -1;
                                } else if (u[i] > top && a_hi < n - 1) {
                                    // above the bracket: exact search beyond it
                                    k = thread_search(P, u[i], a_hi + 1, n - 1);
                                    kprev = -1;
                                } else {
                                    int kk;
                                    if (kprev >= 0) {
                                        kk = lds_walk(sm.q, kprev, cnt, u[i]);
                                    } else {
                                        kk = lds_lower_bound(sm.q, cnt, u[i]);
                                        if (kk > cnt - 1) kk = cnt - 1;
                                    }
                                    kprev = kk;
                                    k = w0 + kk;
                                }
                                anc[i] = static_cast<int32_t>(k);
                                pending &= ~(1u << i);
                            }
                        }
                    }
                    floor = top;
                    __syncthreads();
                }
                }
            } else if (strategy == kCutpoint && A.cut_in) {
                // the paper's cut-point method with the table in device memory
                G<const int32_t>* table = gp(A.cut_in);
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (jt + i < n) anc[i] = static_cast<int32_t>(cut_draw_global(P, table, u[i]));
            } else {
                // bisection per slot over the tiled CDF
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (jt + i < n) anc[i] = static_cast<int32_t>(thread_search(P, u[i], 0, n - 1));
            }
        }
    }

    // ---------------------------------------------------------- 2. propagate
    const ModelParams& p = A.p;
    G<const R>* rin = gp(static_cast<const R*>(A.rec_in));
    G<R>* rout = gp(static_cast<R*>(A.rec_out));
    G<int32_t>* anc_out = A.anc_out ? gp(A.anc_out) : nullptr;
    const bool full = jt + IPT <= n;   // all of the thread's slots are particles
    // single precision under systematic resampling: a slot's draws fit one
    // Philox block (the model decides whether it needs more)
    const bool one_block = sizeof(R) == 4 && A.scheme == kSystematicScheme;
    using M = Math<R>;
    // ew[i] = exp(l_i - pm): the item's weight relative to the thread's
    // reference pm (its first weight, raised when a later one exceeds it by
    // more than kRefSlack, which keeps every ew below e^kRefSlack); tmx is
    // the thread's largest log-weight.  The tile CDF reuses ew, so each
    // particle takes one exponential.  Moment partials: weighted ones
    // relative to pm, equal-weight ones as plain sums; folded into double
    // precision across the tile below.
    constexpr float kRefSlack = 32.0f;
    R ew[IPT];
    R pm = R(-INFINITY), tmx = R(-INFINITY), pe = R(0), pe2 = R(0);
    R pg[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) pg[k] = R(0);
    R zout[F][IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        // slot and ancestor indices fit 32 bits (N < 2^31): uniform per-field
        // base pointers plus a 32-bit offset keep the address math scalar
        const uint32_t j = static_cast<uint32_t>(jt) + static_cast<uint32_t>(i);
        ew[i] = R(0);
#pragma unroll
        for (int f = 0; f < F; ++f) zout[f][i] = R(0);
        if (static_cast<int64_t>(j) < n) {
            const uint32_t a = static_cast<uint32_t>(anc[i]);
            R z[F], zn[F];
#pragma unroll
            // ordinary (cached) loads: a thread's slots are consecutive, so
            // the IPT gathers of one field share cache lines (streaming loads
            // would fetch each line once per load)
            for (int f = 0; f < F; ++f) z[f] = (rin + f * A.pitch)[a];
            R g[NG];
            if (propagate) {
                MD::template propagate<R>(p, A.seed, j, A.t, A.y_prop, w[i], z, zn, g, one_block);
#pragma unroll
                for (int f = 0; f < F; ++f) zout[f][i] = zn[f];
            } else {
#pragma unroll
                for (int f = 0; f < F; ++f) zn[f] = z[f];
                MD::template terms<R>(p, A.t, zn, g);
            }
            if (anc_out) anc_out[j] = anc[i];
            const R l = weight ? MD::template logw<R>(p, zn, A.y_weight) : R(-INFINITY);
            if (weight) {
                tmx = fmax(tmx, l);
                if (i == 0) pm = l;
                if (l > pm + R(kRefSlack) || (pm == R(-INFINITY) && l > pm)) {
                    // (rare) a new reference: rescale what is relative to the old one
                    const R sc = M::exp(pm - l);
#pragma unroll
                    for (int k = 0; k < i; ++k) ew[k] *= sc;
                    pe *= sc;
                    pe2 *= sc * sc;
#pragma unroll
                    for (int k = 0; k < NG; ++k) pg[k] *= sc;
                    pm = l;
                }
                ew[i] = (l == R(-INFINITY)) ? R(0) : M::exp(l - pm);
            }
            if (weighted_mom) {
                const R e = ew[i];
                pe += e;
                pe2 += e * e;
#pragma unroll
                for (int k = 0; k < NG; ++k) pg[k] += e * g[k];
            } else {
#pragma unroll
                for (int k = 0; k < NG; ++k) pg[k] += g[k];
                pe += R(1);
            }
        }
    }
    if (propagate) {
        // the new record: each field's IPT values of this thread are contiguous
#pragma unroll
        for (int f = 0; f < F; ++f) {
            G<R>* dst = rout + f * A.pitch + jt;
            if (full) {
                store_run<R, IPT>(dst, zout[f]);
            } else {
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (jt + i < n) __builtin_nontemporal_store(zout[f][i], dst + i);
            }
        }
    }

    // ---------------------------------------------------------- moment partials
    {
        // The threads' partials (weighted ones relative to the thread's
        // reference) are brought to the tile's largest reference and summed
        // in a fixed order: with room in the LDS window, every sum is folded
        // by 32 lanes over eight threads' entries each and then across the
        // lanes; otherwise by wave reductions and a fold over the waves.
        constexpr int NS = 2 + NG;  // e, e^2, e g[0 .. NG)
        constexpr bool kLdsFold = BLOCK == 256 && NS <= BLOCK / 32 && NS * BLOCK <= WIN;
        const double tm = static_cast<double>(pm);
        G<double>* dst = gp(A.partials) + static_cast<int64_t>(tile) * kPartialStride;
        if constexpr (kLdsFold) {
            // (every search path ends with a barrier, so the window in LDS
            // is free again here)
            double Mx = 0.0, sc = 1.0;
            if (weighted_mom) {
                const double m = wave_max(tm);
                if (lane == 0) sm.red[wave] = m;
                __syncthreads();
                Mx = -INFINITY;
                for (int q = 0; q < NW; ++q) Mx = fmax(Mx, sm.red[q]);
                sc = (tm == -INFINITY) ? 0.0 : exp(tm - Mx);
            }
            double* buf = sm.q;
            buf[tid] = static_cast<double>(pe) * sc;
            buf[BLOCK + tid] = static_cast<double>(pe2) * sc * sc;
#pragma unroll
            for (int k = 0; k < NG; ++k) buf[(2 + k) * BLOCK + tid] = static_cast<double>(pg[k]) * sc;
            __syncthreads();
            constexpr int PER = BLOCK / 32;
            const int v = tid / 32, part = tid % 32;
            double acc = 0.0;
            if (v < NS) {
#pragma unroll
                for (int r = 0; r < PER; ++r) acc += buf[v * BLOCK + part * PER + r];
            }
            acc = half_wave_sum(acc);
            if (v < NS && part == 31) dst[1 + v] = acc;
            if (tid == 0) dst[0] = weighted_mom ? Mx : 0.0;
            __syncthreads();
        } else {
            double m = weighted_mom ? wave_max(tm) : 0.0;
            const double sc = weighted_mom ? (tm == -INFINITY ? 0.0 : exp(tm - m)) : 1.0;
            const double v_e = wave_sum(static_cast<double>(pe) * sc);
            const double v_e2 = wave_sum(static_cast<double>(pe2) * sc * sc);
            double v_g[NG];
#pragma unroll
            for (int k = 0; k < NG; ++k) v_g[k] = wave_sum(static_cast<double>(pg[k]) * sc);
            if (lane == 0) {
                double* r = sm.red + wave * 16;
                r[0] = m;
                r[1] = v_e;
                r[2] = v_e2;
#pragma unroll
                for (int k = 0; k < NG; ++k) r[3 + k] = v_g[k];
            }
            __syncthreads();
            if (tid == 0) {
                double Mx = -INFINITY;
                if (weighted_mom)
                    for (int q = 0; q < NW; ++q) Mx = fmax(Mx, sm.red[q * 16]);
                double out[3 + NG];
                for (int k = 0; k < 3 + NG; ++k) out[k] = 0.0;
                for (int q = 0; q < NW; ++q) {
                    const double* r = sm.red + q * 16;
                    const double f = weighted_mom ? (r[0] == -INFINITY ? 0.0 : exp(r[0] - Mx)) : 1.0;
                    out[1] += r[1] * f;
                    out[2] += r[2] * f * f;
                    for (int k = 0; k < NG; ++k) out[3 + k] += r[3 + k] * f;
                }
                out[0] = weighted_mom ? Mx : 0.0;
                for (int k = 0; k < 3 + NG; ++k) dst[k] = out[k];
            }
            __syncthreads();
        }
    }

    if (!weight) return;

    // ---------------------------------------------------------- 3. tile CDF
    const double mloc = wave_max_r(tmx);
    if (lane == 0) sm.red[wave] = mloc;
    __syncthreads();
    double mb = -INFINITY;
    for (int q = 0; q < NW; ++q) mb = fmax(mb, sm.red[q]);
    // e_k = exp(l_k - m_b) = ew_k exp(pm - m_b): one exponential per thread,
    // in double precision where the weights' precision would underflow
    double fac = 0.0;
    if (mb != -INFINITY && pm != R(-INFINITY)) {
        const double d = static_cast<double>(pm) - mb;
        fac = (sizeof(R) == 4 && d > -80.0) ? static_cast<double>(M::exp(static_cast<R>(d)))
                                             : exp(d);
    }
    // the thread's own IPT slots, then the threads' sums scanned
    double v[IPT];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        run += static_cast<double>(ew[i]) * fac;
        v[i] = run;
    }
    const double tincl = wave_incl_sum(run);
    if (lane == kWave - 1) sm.red[NW + wave] = tincl;
    __syncthreads();
    double base = 0.0;
    for (int q = 0; q < wave; ++q) base += sm.red[NW + q];
    double total = 0.0;
    for (int q = 0; q < NW; ++q) total += sm.red[NW + q];
    double texcl = wave_shr1(tincl, 0.0);
    base += texcl;
    // the threads' bases and runs are rounded separately, so a thread's first
    // prefix can fall an ulp below its predecessor's last: raise each value to
    // the largest last value of the threads before it (stored prefixes are
    // then non-decreasing in the tile)
    const double tlast = base + v[IPT - 1];
    const double wmax = wave_incl_max(tlast);
    if (lane == kWave - 1) sm.red[2 * NW + wave] = wmax;
    __syncthreads();
    double carry = -INFINITY;
    for (int q = 0; q < wave; ++q) carry = fmax(carry, sm.red[2 * NW + q]);
    double wex = wave_shr1(wmax, -INFINITY);
    carry = fmax(carry, wex);
    // single precision rounds toward zero so that a tile's last prefix never
    // exceeds the tile total the scan uses
    R cst[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const double cval = fmax(base + v[i], carry);
        cst[i] = sizeof(R) == 4 ? static_cast<R>(__double2float_rz(cval)) : static_cast<R>(cval);
    }
    G<R>* cout = gp(static_cast<R*>(A.c_out));
    if (full) {
        store_run<R, IPT>(cout + jt, cst);
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i)
            if (jt + i < n) __builtin_nontemporal_store(cst[i], cout + jt + i);
    }
    if (!lookback) {
        // segment samples of this tile's prefix: segment s ends at offset
        // (s + 1) SEG - 1, the last slot of a thread; segments that run past
        // N take the last particle's value, written by the thread holding it
        constexpr int SEG = TS / kSegments;
        static_assert(SEG % IPT == 0, "a segment ends on a thread's last slot");
        G<R>* samp = gp(static_cast<R*>(A.samp_out)) + static_cast<int64_t>(tile) * kSegments;
        const int64_t plast = min(static_cast<int64_t>(TS), n - j0) - 1;
        const int off_end = tid * IPT + IPT - 1;
        if ((off_end + 1) % SEG == 0 && off_end <= plast) samp[off_end / SEG] = cst[IPT - 1];
        if (plast < TS - 1 && tid == static_cast<int>(plast / IPT)) {
            R vl = cst[0];
#pragma unroll
            for (int i = 1; i < IPT; ++i)
                if (i == static_cast<int>(plast % IPT)) vl = cst[i];
            for (int s = static_cast<int>((plast + 1) / SEG); s < kSegments; ++s) samp[s] = vl;
        }
    }
    const Agg mine{mb, mb == -INFINITY ? 0.0 : total};

    if (!lookback) {
        if (!(A.flags & kFusedScan)) {
            // tile scan: publish the tile's (max, sum); k_scan_tiles does the rest
            if (tid == 0) {
                G<double>* agg = gp(A.agg_out);
                agg[2 * static_cast<int64_t>(tile)] = mine.m;
                agg[2 * static_cast<int64_t>(tile) + 1] = mine.s;
            }
            return;
        }
        // fused tile scan: publish the tile's (max, sum) as epoch-tagged words,
        // then count this work-group done; the one that finishes last scans.
        // Every tile publishes before it counts itself, so each word the last
        // work-group waits on is at most still in flight.
        if (tid == 0) {
            put_agg(A.status + static_cast<int64_t>(tile) * kStatusWords, A.epoch, mine);
            const uint32_t dn = __hip_atomic_fetch_add(&A.st->done, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            sm.scan_here = (dn + 1u == static_cast<uint32_t>(A.num_tiles)) ? 1 : 0;
        }
        __syncthreads();
        const bool scan_here = sm.scan_here != 0;
        // every wave has read the flag before any leaves (the batched kernel
        // reuses the work-group's shared fields for its next tile)
        __syncthreads();
        if (!scan_here) return;
        if (tid == 0) __hip_atomic_store(&A.st->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // (a test run waits for words no tile writes, and gives up sooner)
        const uint32_t epoch = A.test_stall ? (A.epoch ^ 0x80000000u) : A.epoch;
        const uint32_t spin_limit = A.test_stall ? kTestSpins : kFusedScanSpins;
        const uint64_t* status = A.status;
        DevState* st = A.st;
        // all of the thread's words are requested at once; a tile whose words
        // do not all carry this epoch yet is polled again (bounded)
        auto load = [&](int b0, int b1, double (&m)[4], double (&w)[4]) {
            uint64_t wd[4][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t* p = status + static_cast<int64_t>(min(b0 + k, b1 - 1)) * kStatusWords;
#pragma unroll
                for (int q = 0; q < 4; ++q) wd[k][q] = b0 + k < b1 ? get_word(p + q) : 0;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                m[k] = -INFINITY;
                w[k] = 0.0;
                if (b0 + k >= b1) continue;
                const uint64_t tag = static_cast<uint64_t>(epoch);
                Agg v;
                if ((wd[k][0] >> 32) == tag && (wd[k][1] >> 32) == tag &&
                    (wd[k][2] >> 32) == tag && (wd[k][3] >> 32) == tag) {
                    v.m = __longlong_as_double(
                        static_cast<long long>((wd[k][0] & 0xffffffffull) | (wd[k][1] << 32)));
                    v.s = __longlong_as_double(
                        static_cast<long long>((wd[k][2] & 0xffffffffull) | (wd[k][3] << 32)));
                } else {
                    const uint64_t* p = status + static_cast<int64_t>(b0 + k) * kStatusWords;
                    for (uint32_t spin = 0; !get_agg(p, epoch, v); ++spin) {
                        if (spin >= spin_limit) {
                            atomicOr(&st->flags, kScanStall);
                            v = agg_identity();
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                m[k] = v.m;
                w[k] = v.s;
            }
        };
        static_assert(BLOCK * 4 >= kFusedScanMax, "fused scan: 4 tiles per thread");
        tile_scan_core<BLOCK, 4>(load, A.num_tiles, n, TS, A.ab_out, A.hint_out, A.tot_out, A.st,
                                 nullptr, sm.red, sm.q);
        return;
    }

    // ---------------------------------------------------------- 4. look-back
    if (wave == 0) {
        const uint32_t epoch = A.epoch;
        // (a test run waits for words no tile writes, and gives up sooner)
        const uint32_t wait_epoch = A.test_stall ? (epoch ^ 0x80000000u) : epoch;
        const uint32_t spin_limit = A.test_stall ? kTestSpins : kFusedScanSpins;
        uint64_t* st = A.status;
        if (lane == 0) put_agg(st + static_cast<int64_t>(tile) * kStatusWords, epoch, mine);
        // each lane covers kLookPer consecutive predecessors (nearest first),
        // so one round reads 64 * kLookPer tiles and stops at the nearest
        // one that has published its inclusive prefix
        Agg acc = agg_identity();
        if (tile > 0) {
            int64_t top = static_cast<int64_t>(tile) - 1;
            while (true) {
                Agg part = agg_identity();
                bool has_incl = false;
#pragma unroll
                for (int p = 0; p < kLookPer; ++p) {
                    if (has_incl) break;
                    const int64_t idx = top - static_cast<int64_t>(lane) * kLookPer - p;
                    Agg val = agg_identity();
                    bool incl = true;  // before tile 0: the inclusive identity
                    if (idx >= 0) {
                        const uint64_t* s = st + idx * kStatusWords;
                        for (uint32_t spin = 0;; ++spin) {
                            if (get_agg(s + 4, wait_epoch, val)) { incl = true; break; }
                            if (get_agg(s, wait_epoch, val)) { incl = false; break; }
                            if (spin >= spin_limit) {
                                // the predecessor never published: report it
                                // and end the look-back here
                                atomicOr(&A.st->flags, kScanStall);
                                val = agg_identity();
                                incl = true;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    part = agg_combine(val, part);
                    has_incl = incl;
                }
                const uint64_t incl_mask = __ballot(has_incl);
                const int stop = incl_mask ? __ffsll(static_cast<long long>(incl_mask)) - 1 : kWave;
                const Agg wsum = wave_agg(lane <= stop ? part : agg_identity());
                acc = agg_combine(wsum, acc);
                if (incl_mask) break;
                top -= static_cast<int64_t>(kWave) * kLookPer;
            }
        }
        const Agg incl = agg_combine(acc, mine);
        if (lane == 0) {
            put_agg(st + static_cast<int64_t>(tile) * kStatusWords + 4, epoch, incl);
            A.tiles_out[tile] = TileInfo{acc.m, acc.s, mine.m, mine.s};
            if (tile == static_cast<uint32_t>(A.num_tiles - 1)) {
                A.tot_out->M = incl.m;
                A.tot_out->S = incl.s;
                const bool ok = (incl.s > 0.0) && isfinite(incl.s) && isfinite(incl.m);
                if (!ok) atomicOr(&A.st->flags, kDegenerate);
                A.st->loglik += incl.m + log(incl.s / static_cast<double>(n));
                // every ticket of this launch has been handed out
                __hip_atomic_store(&A.st->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// One filter, one cycle: a work-group per tile.  With the look-back, tiles
// are taken from a dynamic ticket, so that every tile a look-back waits on
// was handed out earlier and is resident or done.
// Work-groups per CU the register allocation is held to: the cycle is
// latency-bound (dependent global loads for the search bracket, the window
// and the gathers), so more resident waves pay for a few spilled registers.
// With 8 items per thread the LDS window already limits residency to three.
template <int IPT>
constexpr int step_min_blocks() { return IPT >= 8 ? 3 : 5; }
template <int MODEL, typename R, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK, step_min_blocks<IPT>()) void k_step(StepArgs A) {
    __shared__ StepSmem<BLOCK, IPT> sm;
    uint32_t tile = blockIdx.x;
    if ((A.flags & kWeight) && A.scan == kScanLookback) {
        if (threadIdx.x == 0)
            sm.tile = __hip_atomic_fetch_add(&A.st->ticket, 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        tile = uniform32(sm.tile);
    }
    cycle<MODEL, R, BLOCK, IPT>(A, tile, sm);
}

// Many filters, one cycle each, in one launch: work-group g takes global
// tile g, tile_map[g] = (member f, tile of f); filter f's arguments for
// step s are descs[(s mod ring) * capacity + f], where s is the batch's
// device-side step counter (advanced by k_scan_batch), so the same pair of
// launches can be replayed step after step.  The grid covers the tile map's
// capacity; work-groups at or beyond the batch's current tile count return
// at once, so membership can change between replays.  (A persistent grid
// that took tiles from a ticket held one work-group fewer per CU and paid a
// dependent ticket-map-descriptor prologue per tile: 12% slower.)
template <int MODEL, typename R, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK, step_min_blocks<IPT>()) void k_step_batch(
    const StepArgs* __restrict__ descs, const int2* __restrict__ tile_map, BatchState* bs) {
    __shared__ StepSmem<BLOCK, IPT> sm;
    const int64_t g = blockIdx.x;
    const int64_t total = uniform64(bs->total_tiles);
    if (g >= total) return;
    // the batch's state is the same for the whole grid: keep it (and every
    // address derived from it) in scalar registers
    const uint64_t step = static_cast<uint64_t>(uniform64(static_cast<int64_t>(
        __hip_atomic_load(&bs->step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))));
    const uint32_t ring = uniform32(bs->ring);
    const uint32_t capacity = uniform32(static_cast<uint32_t>(bs->capacity));
    const StepArgs* d = descs + (step % ring) * capacity;
    const int2 owner = tile_map[g];
    const int32_t f = static_cast<int32_t>(uniform32(static_cast<uint32_t>(owner.x)));
    const uint32_t tile = uniform32(static_cast<uint32_t>(owner.y));
    cycle<MODEL, R, BLOCK, IPT>(d[f], tile, sm);
}

// tile_map[base[f] + k] = (f, k) for every tile k of member f (one
// work-group per member).
__global__ __launch_bounds__(256) void k_batch_map(const int32_t* __restrict__ base,
                                                   int32_t n_filters, int2* __restrict__ tile_map) {
    const int32_t f = blockIdx.x;
    if (f >= n_filters) return;
    const int32_t b0 = base[f], b1 = base[f + 1];
    for (int32_t k = threadIdx.x; b0 + k < b1; k += blockDim.x) tile_map[b0 + k] = make_int2(f, k);
}

// ------------------------------------------------------------ cut-point table
// The parallelized cut-point search of Section 3.2 over the tiled CDF
// q(k) = A_b + c[k] B_b: entry e (1-based) of the table receives
// I_e = min{j : L'_j >= e}, where L'_j is an upper envelope of
// L_j = ceil(n q(j)) that is non-decreasing in j.  Inside a tile q is
// non-decreasing, so L' = max(L, F_b) there, with the tile's floor
// F_b = ceil(n A_b) + 1 (F_0 = 0) bounding every L of the tiles before it
// (their q are at most A_b up to a few ulps); a tile's last element takes
// F_{b+1} and the CDF's last element n.  Since L' >= L, I_e never exceeds
// the answer min{k : q(k) >= u} of any u with ceil(n u) = e, so a climb
// from it is exact; since L' is non-decreasing, element j owns exactly the
// entries (L'_{j-1}, L'_j] and writes its index there, and every entry is
// written once.  A thread writes at most kCutRun entries of its own range;
// the rest of a longer range (a heavy particle) is filled by its whole
// work-group.
constexpr int kCutRun = 32;

template <typename R>
struct CutEnvelope {
    const R* c;
    const TileAB* ab;
    int64_t n;
    int32_t ts, tiles;
    // ceil(x) as an entry count in [0, n] (0 for NaN)
    __device__ __forceinline__ int64_t count(double x) const {
        return x >= 1.0 ? (x >= static_cast<double>(n) ? n : static_cast<int64_t>(x)) : 0;
    }
    __device__ __forceinline__ int64_t floor_of(int64_t b) const {
        return b <= 0 ? 0 : count(ceil(static_cast<double>(n) * ab[b].a) + 1.0);
    }
    // L'_k, with L'_{-1} = 0
    __device__ __forceinline__ int64_t at(int64_t k) const {
        if (k < 0) return 0;
        if (k >= n - 1) return n;
        const int64_t b = k / ts;
        if (k == (b + 1) * ts - 1) return floor_of(b + 1);
        const TileAB t = ab[b];
        const double L = ceil(static_cast<double>(n) * fma(static_cast<double>(c[k]), t.b, t.a));
        return max(count(L), floor_of(b));
    }
};

// Entries of the elements j0 .. j0 + NT - 1 (one per thread) written by a
// work-group of NT threads; s_lo, s_hi, s_j hold NT entries, *s_count one.
template <int NT, typename R>
__device__ __forceinline__ void cut_table_block(const CutEnvelope<R>& E, int64_t j0,
                                                int32_t* __restrict__ table, int64_t* s_lo,
                                                int64_t* s_hi, int32_t* s_j, int* s_count) {
    const int tid = threadIdx.x;
    if (tid == 0) *s_count = 0;
    __syncthreads();
    const int64_t j = j0 + tid;
    if (j < E.n) {
        const int64_t lo = E.at(j - 1), hi = E.at(j);
        const int64_t own = min(hi, lo + kCutRun);
        for (int64_t e = lo; e < own; ++e) table[e] = static_cast<int32_t>(j);
        if (hi > own) {
            const int slot = atomicAdd(s_count, 1);
            s_lo[slot] = own;
            s_hi[slot] = hi;
            s_j[slot] = static_cast<int32_t>(j);
        }
    }
    __syncthreads();
    const int count = *s_count;
    for (int q = 0; q < count; ++q) {
        const int32_t v = s_j[q];
        for (int64_t e = s_lo[q] + tid; e < s_hi[q]; e += NT) table[e] = v;
    }
    __syncthreads();
}

template <typename R>
__global__ __launch_bounds__(256) void k_cut_table(CutEnvelope<R> E, int32_t* __restrict__ table) {
    __shared__ int64_t s_lo[256], s_hi[256];
    __shared__ int32_t s_j[256];
    __shared__ int s_count;
    cut_table_block<256>(E, static_cast<int64_t>(blockIdx.x) * 256, table, s_lo, s_hi, s_j,
                         &s_count);
}

// ------------------------------------------------------------ tile scan
// The tile scan turns the tiles' (m_b, s_b) into
//   A_b = sum_{b' < b} s_b' e^{m_b' - M} / S  (non-decreasing),
//   B_b = e^{m_b - M} / S,
// with M = max_b m_b taken first, so that each tile costs one exponential
// and the prefix is a plain double-precision sum, S = sum_b s_b e^{m_b - M}
// (fixed order: the result does not depend on timing); adds M + log(S / n)
// to the log-likelihood; and writes hint[h] = the tile whose range
// [A_b, A_{b+1}) holds the CDF position h * ts / n, for h = 0..tiles, where
// the next cycle's tile h starts its search for sorted uniforms.  Up to
// 4096 tiles one work-group does it all; above, three launches over chunks
// of kScanBlock tiles (or one work-group that does the same arithmetic, in
// a batch).  The (m_b, s_b) pairs are only read.
constexpr int kScanBlock = 1024;

// The single-work-group tile scan: up to kTileScanBlock * kTileScanPer
// tiles, each thread keeping its (at most kTileScanPer) tiles in registers:
// one pass reads the (max, sum) pairs, one writes the table and the hints,
// three barriers.
constexpr int kTileScanBlock = 512;
constexpr int kTileScanPer = 4096 / kTileScanBlock;

// Search positions of the output tiles: h ts / n (stratified, systematic),
// or, for sorted multinomial, pos[h].a, the normalised spacing prefix before
// output tile h.  first_h(b) = the first output tile h >= 1 whose position
// is at least A_b (tile 0 starts at 0; T + 1 past the last tile).
struct HintPos {
    const TileAB* pos;  // sorted multinomial, else null
    int32_t T;
    double scale;       // n / ts
    __device__ __forceinline__ int64_t first_h(int64_t b, double ab_a) const {
        if (b == 0) return 0;
        if (b >= T) return static_cast<int64_t>(T) + 1;
        if (!pos) {
            const double v = ceil(ab_a * scale);
            return v > static_cast<double>(T) ? static_cast<int64_t>(T) : static_cast<int64_t>(v);
        }
        int lo = 1, hi = T;  // first h in [1, T) with pos[h].a >= ab_a, else T
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (pos[mid].a >= ab_a) hi = mid; else lo = mid + 1;
        }
        return lo;
    }
};

// The scan over NT threads, each holding at most PER tiles; load(b0, b1,
// m, w) fills m[k], w[k] with tile b0 + k's (max, sum) for b0 + k < b1 and
// with (-inf, 0) beyond.  s_red holds NT / 64 doubles, s_first NT.
template <int NT, int PER, typename Load>
__device__ __forceinline__ void tile_scan_core(Load load, int32_t num_tiles, int64_t n,
                                               int32_t ts, TileAB* ab, int32_t* hint,
                                               Totals* tot, DevState* st, const TileAB* pos,
                                               double* s_red, double* s_first) {
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int T = num_tiles;
    const int per = (T + NT - 1) / NT;
    const int b0 = min(T, tid * per), b1 = min(T, b0 + per);
    double m[PER], w[PER], e[PER];
    // 1. M = max_b m_b
    double mx = -INFINITY;
    load(b0, b1, m, w);
#pragma unroll
    for (int k = 0; k < PER; ++k) mx = fmax(mx, m[k]);
    mx = wave_max(mx);
    if (lane == 0) s_red[wave] = mx;
    __syncthreads();
    double M = -INFINITY;
    for (int q = 0; q < NW; ++q) M = fmax(M, s_red[q]);
    __syncthreads();
    // 2. e_b = e^{m_b - M}, w_b = s_b e_b; exclusive scan of the threads' sums
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        e[k] = (m[k] == -INFINITY || M == -INFINITY) ? 0.0 : exp(m[k] - M);
        w[k] *= e[k];
        part += w[k];
    }
    const double incl = wave_incl_sum(part);
    if (lane == kWave - 1) s_red[wave] = incl;
    __syncthreads();
    double wbase = 0.0, S = 0.0;
    for (int q = 0; q < NW; ++q) {
        if (q == wave) wbase = S;
        S += s_red[q];
    }
    double excl = wave_shr1(incl, 0.0);
    excl += wbase;
    const bool ok = (S > 0.0) && isfinite(S) && isfinite(M);
    // 3. A_b, running max in the thread, then over the threads before it
    double a[PER];
    double run = excl, amax = -INFINITY;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        amax = fmax(amax, ok ? run / S : 0.0);
        a[k] = amax;
        run += w[k];
    }
    if (b0 >= b1) amax = -INFINITY;
    s_first[tid] = b0 < b1 ? a[0] : -INFINITY;
    __syncthreads();  // s_red is read above, by every thread, before this
    const double top = wave_incl_max(amax);
    if (lane == kWave - 1) s_red[wave] = top;
    __syncthreads();
    double carry = -INFINITY;
    for (int q = 0; q < wave; ++q) carry = fmax(carry, s_red[q]);
    double ex = wave_shr1(top, -INFINITY);
    carry = fmax(carry, ex);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        a[k] = fmax(a[k], carry);
        if (b0 + k < b1) ab[b0 + k] = TileAB{a[k], ok ? e[k] / S : 0.0};
    }
    // 4. hints: tile b owns the output tiles h with ceil(A_b n / ts) <= h <
    //    ceil(A_{b+1} n / ts); tile 0 starts at h = 0, the last tile runs to
    //    h = T.  The next thread's first A (after its own carry, which is
    //    this thread's carry raised by this thread's last value) closes the
    //    thread's last range.
    if (tid == 0) {
        tot->M = M;
        tot->S = S;
        if (st) {
            if (!ok) atomicOr(&st->flags, kDegenerate);
            st->loglik += M + log(S / static_cast<double>(n));
        }
    }
    if (b0 >= b1 || !hint) return;
    const HintPos hp{pos, T, static_cast<double>(n) / static_cast<double>(ts)};
    const double next_a = b1 < T ? fmax(s_first[tid + 1], fmax(carry, amax)) : 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int b = b0 + k;
        if (b < b1) {
            const double an = (b + 1 < b1) ? a[k + 1 < PER ? k + 1 : k] : next_a;
            const int64_t h0 = hp.first_h(b, a[k]), h1 = hp.first_h(b + 1, an);
            for (int64_t h = h0; h < h1; ++h) hint[h] = b;
        }
    }
}

__device__ __forceinline__ void scan_tiles_regs(const double* agg, int32_t num_tiles, int64_t n,
                                                int32_t ts, TileAB* ab, int32_t* hint,
                                                Totals* tot, DevState* st,
                                                const TileAB* pos = nullptr) {
    __shared__ double s_red[kTileScanBlock / kWave], s_first[kTileScanBlock];
    auto load = [&](int b0, int b1, double (&m)[kTileScanPer], double (&w)[kTileScanPer]) {
#pragma unroll
        for (int k = 0; k < kTileScanPer; ++k) {
            m[k] = -INFINITY;
            w[k] = 0.0;
            if (b0 + k < b1) {
                const double2 v = reinterpret_cast<const double2*>(agg)[b0 + k];
                m[k] = v.x;
                w[k] = v.y;
            }
        }
    };
    tile_scan_core<kTileScanBlock, kTileScanPer>(load, num_tiles, n, ts, ab, hint, tot, st, pos,
                                                 s_red, s_first);
}

// Launched for at most kTileScanBlock * kTileScanPer tiles (more take the
// chunked launches below).
__global__ __launch_bounds__(kTileScanBlock) void k_scan_tiles(const double* agg,
                                                           int32_t num_tiles, int64_t n,
                                                           int32_t ts, TileAB* ab, int32_t* hint,
                                                           Totals* tot, DevState* st,
                                                           const TileAB* pos) {
    scan_tiles_regs(agg, num_tiles, n, ts, ab, hint, tot, st, pos);
}

// ------------------------------------------------------------ chunked tile scan
// For many tiles the same table comes from three launches over chunks of
// kScanBlock consecutive tiles, one work-group per chunk, each tile read
// by one thread (coalesced):
//   k_scan_chunks: chunk c's (m_c, s_c) = (max_b m_b, sum_b s_b e^{m_b - m_c});
//   k_scan_top:    M = max_c m_c, the chunks' weights s_c e^{m_c - M}, their
//                  exclusive prefix P_c (made non-decreasing; S = P_G), the
//                  totals and the log-likelihood increment M + log(S / n);
//   k_scan_apply:  tile weights s_b e^{m_b - M}, their exclusive prefix in
//                  the chunk from P_c, A_b = min(P_c + prefix, P_{c+1}) / S
//                  made non-decreasing, B_b = e^{m_b - M} / S, and the search
//                  hints of the chunk's tiles.
// Clamping every A_b of chunk c to P_{c+1} / S, which is exactly the first
// A of chunk c + 1, keeps A non-decreasing across chunks although the chunk
// prefixes and the in-chunk prefixes are rounded separately.  Fixed order
// throughout: the result does not depend on timing.
template <int NW>
__device__ __forceinline__ double block_max(double v, double* s_red) {
    v = wave_max(v);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = v;
    __syncthreads();
    double r = -INFINITY;
    for (int q = 0; q < NW; ++q) r = fmax(r, s_red[q]);
    __syncthreads();
    return r;
}

// Exclusive prefix sum in thread order; *total receives the block's sum.
template <int NW>
__device__ __forceinline__ double block_excl_sum(double v, double* s_red, double* total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const double incl = wave_incl_sum(v);
    if (lane == kWave - 1) s_red[wave] = incl;
    __syncthreads();
    double base = 0.0, tot = 0.0;
    for (int q = 0; q < NW; ++q) {
        if (q == wave) base = tot;
        tot += s_red[q];
    }
    __syncthreads();
    double ex = wave_shr1(incl, 0.0);
    *total = tot;
    return base + ex;
}

// Largest value of the threads before this one (-inf for thread 0).
template <int NW>
__device__ __forceinline__ double block_excl_max(double v, double* s_red) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const double incl = wave_incl_max(v);
    if (lane == kWave - 1) s_red[wave] = incl;
    __syncthreads();
    double carry = -INFINITY;
    for (int q = 0; q < wave; ++q) carry = fmax(carry, s_red[q]);
    __syncthreads();
    double ex = wave_shr1(incl, -INFINITY);
    return fmax(ex, carry);
}

// Inclusive running maximum in thread order.
template <int NW>
__device__ __forceinline__ double block_incl_max(double v, double* s_red) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const double incl = wave_incl_max(v);
    if (lane == kWave - 1) s_red[wave] = incl;
    __syncthreads();
    double carry = -INFINITY;
    for (int q = 0; q < wave; ++q) carry = fmax(carry, s_red[q]);
    __syncthreads();
    return fmax(incl, carry);
}

__global__ __launch_bounds__(kScanBlock) void k_scan_chunks(const double* __restrict__ agg,
                                                            int32_t num_tiles,
                                                            double* __restrict__ chunk) {
    constexpr int NW = kScanBlock / kWave;
    __shared__ double s_red[NW];
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x;
    double m = -INFINITY, sb = 0.0;
    if (b < num_tiles) {
        const double2 v = reinterpret_cast<const double2*>(agg)[b];
        m = v.x;
        sb = v.y;
    }
    const double mc = block_max<NW>(m, s_red);
    const double w = (m == -INFINITY) ? 0.0 : sb * exp(m - mc);
    double sc;
    block_excl_sum<NW>(w, s_red, &sc);
    if (threadIdx.x == 0) reinterpret_cast<double2*>(chunk)[blockIdx.x] = make_double2(mc, sc);
}

__global__ __launch_bounds__(kScanBlock) void k_scan_top(const double* __restrict__ chunk,
                                                         int32_t num_chunks, int64_t n,
                                                         double* __restrict__ pref, Totals* tot,
                                                         DevState* st) {
    constexpr int NW = kScanBlock / kWave;
    __shared__ double s_red[NW];
    const int tid = threadIdx.x;
    const int G = num_chunks;
    const int per = (G + kScanBlock - 1) / kScanBlock;
    const int g0 = min(G, tid * per), g1 = min(G, g0 + per);
    double mx = -INFINITY;
    for (int g = g0; g < g1; ++g) mx = fmax(mx, chunk[2 * g]);
    const double M = block_max<NW>(mx, s_red);
    auto weight = [&](int g) {
        const double mg = chunk[2 * g];
        return (mg == -INFINITY || M == -INFINITY) ? 0.0 : chunk[2 * g + 1] * exp(mg - M);
    };
    double part = 0.0;
    for (int g = g0; g < g1; ++g) part += weight(g);
    double total;
    const double excl = block_excl_sum<NW>(part, s_red, &total);
    // this thread's prefixes, made non-decreasing by the largest end of the
    // threads before it
    double run = excl;
    for (int g = g0; g < g1; ++g) run += weight(g);
    const double carry = block_excl_max<NW>(run, s_red);
    run = excl;
    for (int g = g0; g < g1; ++g) {
        pref[g] = fmax(run, carry);
        run += weight(g);
    }
    const double S = block_max<NW>(fmax(run, carry), s_red);
    if (tid == 0) {
        pref[G] = S;
        const bool ok = (S > 0.0) && isfinite(S) && isfinite(M);
        tot->M = M;
        tot->S = S;
        if (st) {
            if (!ok) atomicOr(&st->flags, kDegenerate);
            st->loglik += M + log(S / static_cast<double>(n));
        }
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const double* __restrict__ agg,
                                                           int32_t num_tiles, int64_t n,
                                                           int32_t ts,
                                                           const double* __restrict__ pref,
                                                           const Totals* __restrict__ tot,
                                                           TileAB* __restrict__ ab,
                                                           int32_t* __restrict__ hint,
                                                           const TileAB* __restrict__ pos) {
    constexpr int NW = kScanBlock / kWave;
    __shared__ double s_red[NW];
    __shared__ double s_a[kScanBlock];
    const int tid = threadIdx.x;
    const int T = num_tiles;
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kScanBlock + tid;
    const double M = tot->M, S = tot->S;
    const bool ok = (S > 0.0) && isfinite(S) && isfinite(M);
    const double lo = pref[blockIdx.x], hi = pref[blockIdx.x + 1];
    double m = -INFINITY, sb = 0.0;
    if (b < T) {
        const double2 v = reinterpret_cast<const double2*>(agg)[b];
        m = v.x;
        sb = v.y;
    }
    const double e = (m == -INFINITY || M == -INFINITY) ? 0.0 : exp(m - M);
    double unused;
    const double x = lo + block_excl_sum<NW>(sb * e, s_red, &unused);
    const double a = block_incl_max<NW>(ok ? fmin(x, hi) / S : 0.0, s_red);
    if (b < T) ab[b] = TileAB{a, ok ? e / S : 0.0};
    // hints: tile b owns output tiles ceil(A_b n / ts) <= h < ceil(A_{b+1} n / ts);
    // tile 0 starts at h = 0 and the last tile runs to h = T.  The next
    // chunk's first A equals min(P_{c+1}, P_{c+2}) / S = P_{c+1} / S.
    s_a[tid] = a;
    __syncthreads();
    if (b >= T || !hint) return;
    const HintPos hp{pos, T, static_cast<double>(n) / static_cast<double>(ts)};
    const double a_next = (tid + 1 < kScanBlock) ? s_a[tid + 1] : (ok ? hi / S : 0.0);
    const int64_t h0 = hp.first_h(b, a), h1 = hp.first_h(b + 1, a_next);
    for (int64_t h = h0; h < h1; ++h) hint[h] = static_cast<int32_t>(b);
}

// The chunked scan above, carried out by the one work-group of
// kTileScanBlock threads that scans a batch member of more than
// kTileScanBlock * kTileScanPer tiles: thread tid stands in for the threads
// tid + r * kTileScanBlock (r < kVirt) of those kernels' work-groups of
// kScanBlock threads.  Every wave-level reduction runs over the same 64
// values in the same lanes and every sum over the waves adds them in the
// same order, so the chunk aggregates, the prefixes P_c, M, S, the
// log-likelihood increment, the table and the hints are the same bits as
// the three launches' (a member gets the results it has when stepped
// alone).  chunk: 3G + 1 doubles, as for those launches; agg is only read.
constexpr int kVirt = kScanBlock / kTileScanBlock;
static_assert(kVirt * kTileScanBlock == kScanBlock, "each thread stands in for whole lanes");

struct VirtualBlock {
    static constexpr int NW = kTileScanBlock / kWave;  // waves of this work-group
    static constexpr int NV = kScanBlock / kWave;      // waves of the emulated one
    double* s_red;                                      // NV doubles
    int lane, wave;
    __device__ int vwave(int r) const { return wave + NW * r; }
    // block_max over the emulated work-group
    __device__ double max(const double (&v)[kVirt]) const {
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            const double x = wave_max(v[r]);
            if (lane == 0) s_red[vwave(r)] = x;
        }
        __syncthreads();
        double m = -INFINITY;
        for (int q = 0; q < NV; ++q) m = fmax(m, s_red[q]);
        __syncthreads();
        return m;
    }
    // block_excl_sum: out[r] = the exclusive prefix of virtual thread
    // tid + r * kTileScanBlock; returns the total
    __device__ double excl_sum(const double (&v)[kVirt], double (&out)[kVirt]) const {
        double incl[kVirt];
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            incl[r] = wave_incl_sum(v[r]);
            if (lane == kWave - 1) s_red[vwave(r)] = incl[r];
        }
        __syncthreads();
        double base[kVirt], tot = 0.0;
        for (int q = 0; q < NV; ++q) {
#pragma unroll
            for (int r = 0; r < kVirt; ++r)
                if (q == vwave(r)) base[r] = tot;
            tot += s_red[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            const double ex = wave_shr1(incl[r], 0.0);
            out[r] = base[r] + ex;
        }
        return tot;
    }
    // block_excl_max (incl = false) or block_incl_max (incl = true)
    __device__ void run_max(const double (&v)[kVirt], double (&out)[kVirt], bool inclusive) const {
        double incl[kVirt];
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            incl[r] = wave_incl_max(v[r]);
            if (lane == kWave - 1) s_red[vwave(r)] = incl[r];
        }
        __syncthreads();
        double carry[kVirt];
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            carry[r] = -INFINITY;
            for (int q = 0; q < vwave(r); ++q) carry[r] = fmax(carry[r], s_red[q]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kVirt; ++r)
            out[r] = inclusive ? fmax(incl[r], carry[r])
                               : fmax(wave_shr1(incl[r], -INFINITY), carry[r]);
    }
};

__device__ void scan_tiles_as_chunks(const double* __restrict__ agg, int32_t num_tiles, int64_t n,
                                     int32_t ts, TileAB* __restrict__ ab,
                                     int32_t* __restrict__ hint, Totals* tot, DevState* st,
                                     double* chunk) {
    __shared__ double s_red[VirtualBlock::NV];
    __shared__ double s_a[kScanBlock];
    const int tid = threadIdx.x;
    const VirtualBlock B{s_red, lane_id(), tid / kWave};
    const int T = num_tiles;
    const int G = (T + kScanBlock - 1) / kScanBlock;
    double* pref = chunk + 2 * static_cast<int64_t>(G);
    auto load = [&](int c, double (&m)[kVirt], double (&sb)[kVirt]) {
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            const int64_t b = static_cast<int64_t>(c) * kScanBlock + tid + r * kTileScanBlock;
            m[r] = -INFINITY;
            sb[r] = 0.0;
            if (b < T) {
                const double2 v = reinterpret_cast<const double2*>(agg)[b];
                m[r] = v.x;
                sb[r] = v.y;
            }
        }
    };
    // k_scan_chunks, chunk by chunk (the next chunk's pairs loaded ahead)
    double m[kVirt], sb[kVirt], mn[kVirt], sbn[kVirt];
    load(0, m, sb);
    for (int c = 0; c < G; ++c) {
        if (c + 1 < G) load(c + 1, mn, sbn);
        const double mc = B.max(m);
        double w[kVirt], unused[kVirt];
#pragma unroll
        for (int r = 0; r < kVirt; ++r) w[r] = (m[r] == -INFINITY) ? 0.0 : sb[r] * exp(m[r] - mc);
        const double sc = B.excl_sum(w, unused);
        if (tid == 0) reinterpret_cast<double2*>(chunk)[c] = make_double2(mc, sc);
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            m[r] = mn[r];
            sb[r] = sbn[r];
        }
    }
    __syncthreads();
    // k_scan_top
    const int per = (G + kScanBlock - 1) / kScanBlock;
    int g0[kVirt], g1[kVirt];
    double mx[kVirt];
#pragma unroll
    for (int r = 0; r < kVirt; ++r) {
        g0[r] = min(G, (tid + r * kTileScanBlock) * per);
        g1[r] = min(G, g0[r] + per);
        mx[r] = -INFINITY;
        for (int g = g0[r]; g < g1[r]; ++g) mx[r] = fmax(mx[r], chunk[2 * g]);
    }
    const double M = B.max(mx);
    auto weight = [&](int g) {
        const double mg = chunk[2 * g];
        return (mg == -INFINITY || M == -INFINITY) ? 0.0 : chunk[2 * g + 1] * exp(mg - M);
    };
    double part[kVirt], excl[kVirt], run[kVirt], carry[kVirt], fin[kVirt];
#pragma unroll
    for (int r = 0; r < kVirt; ++r) {
        part[r] = 0.0;
        for (int g = g0[r]; g < g1[r]; ++g) part[r] += weight(g);
    }
    B.excl_sum(part, excl);
#pragma unroll
    for (int r = 0; r < kVirt; ++r) {
        run[r] = excl[r];
        for (int g = g0[r]; g < g1[r]; ++g) run[r] += weight(g);
    }
    B.run_max(run, carry, false);
#pragma unroll
    for (int r = 0; r < kVirt; ++r) {
        run[r] = excl[r];
        for (int g = g0[r]; g < g1[r]; ++g) {
            pref[g] = fmax(run[r], carry[r]);
            run[r] += weight(g);
        }
        fin[r] = fmax(run[r], carry[r]);
    }
    const double S = B.max(fin);
    const bool ok = (S > 0.0) && isfinite(S) && isfinite(M);
    if (tid == 0) {
        pref[G] = S;
        tot->M = M;
        tot->S = S;
        if (st) {
            if (!ok) atomicOr(&st->flags, kDegenerate);
            st->loglik += M + log(S / static_cast<double>(n));
        }
    }
    __syncthreads();
    // k_scan_apply, chunk by chunk
    const HintPos hp{nullptr, T, static_cast<double>(n) / static_cast<double>(ts)};
    load(0, m, sb);
    for (int c = 0; c < G; ++c) {
        if (c + 1 < G) load(c + 1, mn, sbn);
        const double lo = pref[c], hi = pref[c + 1];
        double e[kVirt], pv[kVirt], ex[kVirt], a0[kVirt], a[kVirt];
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            e[r] = (m[r] == -INFINITY || M == -INFINITY) ? 0.0 : exp(m[r] - M);
            pv[r] = sb[r] * e[r];
        }
        B.excl_sum(pv, ex);
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            const double x = lo + ex[r];
            a0[r] = ok ? fmin(x, hi) / S : 0.0;
        }
        B.run_max(a0, a, true);
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            const int v = tid + r * kTileScanBlock;
            const int64_t b = static_cast<int64_t>(c) * kScanBlock + v;
            if (b < T) ab[b] = TileAB{a[r], ok ? e[r] / S : 0.0};
            s_a[v] = a[r];
        }
        __syncthreads();
        if (hint) {
#pragma unroll
            for (int r = 0; r < kVirt; ++r) {
                const int v = tid + r * kTileScanBlock;
                const int64_t b = static_cast<int64_t>(c) * kScanBlock + v;
                if (b < T) {
                    const double a_next = (v + 1 < kScanBlock) ? s_a[v + 1] : (ok ? hi / S : 0.0);
                    const int64_t h0 = hp.first_h(b, a[r]), h1 = hp.first_h(b + 1, a_next);
                    for (int64_t h = h0; h < h1; ++h) hint[h] = static_cast<int32_t>(b);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kVirt; ++r) {
            m[r] = mn[r];
            sb[r] = sbn[r];
        }
    }
}

// The batch's scans: work-group g scans filters g, g + grid, ... (those that
// weighted this step); the last work-group to finish advances the batch's
// step counter.
__global__ __launch_bounds__(kTileScanBlock) void k_scan_batch(const StepArgs* __restrict__ descs,
                                                           BatchState* bs) {
    __shared__ uint32_t s_last;
    const uint64_t step = __hip_atomic_load(&bs->step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t n_filters = bs->n_filters;
    const StepArgs* d = descs + (step % static_cast<uint64_t>(bs->ring)) * bs->capacity;
    __shared__ int64_t s_lo[kTileScanBlock], s_hi[kTileScanBlock];
    __shared__ int32_t s_j[kTileScanBlock];
    __shared__ int s_count;
    for (int32_t f = blockIdx.x; f < n_filters; f += gridDim.x) {
        const StepArgs& A = d[f];
        if ((A.flags & kWeight) && !(A.flags & kFusedScan)) {
            if (A.num_tiles <= kTileScanBlock * kTileScanPer)
                scan_tiles_regs(A.agg_out, A.num_tiles, A.n, A.ts, A.ab_out, A.hint_out, A.tot_out,
                                A.st);
            else
                scan_tiles_as_chunks(A.agg_out, A.num_tiles, A.n, A.ts, A.ab_out, A.hint_out,
                                     A.tot_out, A.st, A.chunk);
        }
        __syncthreads();
        if ((A.flags & kWeight) && A.cut_in) {
            // the cut-point table of the CDF just weighed (the next step's
            // cut_in), built by this work-group
            int32_t* table = const_cast<int32_t*>(A.cut_in);
            const bool fp64 = A.rsz == 8;
            for (int64_t j0 = 0; j0 < A.n; j0 += kTileScanBlock) {
                if (fp64) {
                    const CutEnvelope<double> E{static_cast<const double*>(A.c_out), A.ab_out, A.n,
                                                A.ts, A.num_tiles};
                    cut_table_block<kTileScanBlock>(E, j0, table, s_lo, s_hi, s_j, &s_count);
                } else {
                    const CutEnvelope<float> E{static_cast<const float*>(A.c_out), A.ab_out, A.n,
                                               A.ts, A.num_tiles};
                    cut_table_block<kTileScanBlock>(E, j0, table, s_lo, s_hi, s_j, &s_count);
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        const uint32_t dn = __hip_atomic_fetch_add(&bs->done, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        s_last = (dn == gridDim.x - 1) ? 1u : 0u;
        if (s_last) {
            __hip_atomic_store(&bs->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bs->step, step + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------ initial particles
template <int MODEL, typename R, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_init(StepArgs A) {
    using MD = ModelDef<MODEL>;
    constexpr int F = MD::F, NG = MD::NG;
    constexpr int TS = BLOCK * IPT, NW = BLOCK / kWave;
    __shared__ double red[NW * 16];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * TS;
    R* rout = static_cast<R*>(A.rec_out);
    double pg[NG];
    for (int k = 0; k < NG; ++k) pg[k] = 0.0;
    double cnt = 0.0;
    for (int i = 0; i < IPT; ++i) {
        const int64_t j = j0 + static_cast<int64_t>(i) * BLOCK + tid;
        if (j < A.n) {
            R z[F];
            MD::template init<R>(A.p, A.seed, static_cast<uint32_t>(j), z);
            for (int f = 0; f < F; ++f) rout[f * A.pitch + j] = z[f];
            R g[NG];
            MD::template terms<R>(A.p, 0, z, g);
            for (int k = 0; k < NG; ++k) pg[k] += static_cast<double>(g[k]);
            cnt += 1.0;
            if (A.anc_out) A.anc_out[j] = static_cast<int32_t>(j);
        }
    }
    // status words of this tile start invalid; scalars start at zero
    if (tid < kStatusWords) A.status[static_cast<int64_t>(blockIdx.x) * kStatusWords + tid] = 0;
    if (blockIdx.x == 0 && tid == 0) {
        A.st->loglik = 0.0;
        A.st->ticket = 0;
        A.st->flags = 0;
        A.st->done = 0;
    }
    double vc = wave_sum(cnt);
    double vg[NG];
    for (int k = 0; k < NG; ++k) vg[k] = wave_sum(pg[k]);
    if (lane == 0) {
        red[wave * 16 + 1] = vc;
        for (int k = 0; k < NG; ++k) red[wave * 16 + 3 + k] = vg[k];
    }
    __syncthreads();
    if (tid == 0) {
        double* dst = A.partials + static_cast<int64_t>(blockIdx.x) * kPartialStride;
        double out[3 + NG];
        for (int k = 0; k < 3 + NG; ++k) out[k] = 0.0;
        for (int q = 0; q < NW; ++q) {
            out[1] += red[q * 16 + 1];
            for (int k = 0; k < NG; ++k) out[3 + k] += red[q * 16 + 3 + k];
        }
        for (int k = 0; k < 3 + NG; ++k) dst[k] = out[k];
    }
}

// ------------------------------------------------------------ moment reduction
// One work-group folds the per-tile partials in a fixed order and writes the
// model's moment vector to st->moments.
template <int MODEL>
__global__ __launch_bounds__(256) void k_moments(const double* partials, int32_t num_tiles,
                                                 int64_t n, int32_t weighted, uint32_t t,
                                                 ModelParams p, DevState* st) {
    using MD = ModelDef<MODEL>;
    constexpr int NG = MD::NG, NW = 256 / kWave;
    __shared__ double red[NW * 16];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    double M = -INFINITY;
    if (weighted)
        for (int b = tid; b < num_tiles; b += 256) M = fmax(M, partials[b * kPartialStride]);
    M = wave_max(M);
    if (lane == 0) red[wave] = M;
    __syncthreads();
    M = -INFINITY;
    for (int q = 0; q < NW; ++q) M = fmax(M, red[q]);
    __syncthreads();
    double acc[2 + NG];
    for (int k = 0; k < 2 + NG; ++k) acc[k] = 0.0;
    for (int b = tid; b < num_tiles; b += 256) {
        const double* r = partials + static_cast<int64_t>(b) * kPartialStride;
        const double f = weighted ? (r[0] == -INFINITY ? 0.0 : exp(r[0] - M)) : 1.0;
        acc[0] += r[1] * f;
        acc[1] += r[2] * f * f;
        for (int k = 0; k < NG; ++k) acc[2 + k] += r[3 + k] * f;
    }
    for (int k = 0; k < 2 + NG; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0)
        for (int k = 0; k < 2 + NG; ++k) red[wave * 16 + k] = acc[k];
    __syncthreads();
    if (tid == 0) {
        double s[2 + NG];
        for (int k = 0; k < 2 + NG; ++k) {
            s[k] = 0.0;
            for (int q = 0; q < NW; ++q) s[k] += red[q * 16 + k];
        }
        const double W = weighted ? s[0] : static_cast<double>(n);
        double out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const double ex = s[2] / W, exx = s[3] / W;
        out[0] = ex;
        out[1] = exx - ex * ex;
        const double ess = weighted ? s[0] * s[0] / s[1] : static_cast<double>(n);
        if (MODEL == kLLPF || MODEL == kSVPF) {
            out[2] = ess;
        } else if (MODEL == kLLPL) {
            const double av = p.a_v + 0.5 * t, aw = p.a_w + 0.5 * t;
            out[2] = s[4] / W;
            out[3] = s[5] / W;
            out[4] = s[6] / W / (av - 1.0);
            out[5] = s[7] / W / (aw - 1.0);
        } else {
            out[2] = s[4] / W;
            out[3] = s[5] / W;
            out[4] = s[6] / W;
            out[5] = ess;
            out[6] = s[7] / W;
        }
        for (int k = 0; k < 8; ++k) st->moments[k] = out[k];
    }
}

// ------------------------------------------------------------ search test surface
// anc[j] = min{k : q(k) >= u[j]} (n-1 if none) for a plain double CDF.
__global__ void k_search_binary(PlainCdf cdf, const double* u, int64_t m, int32_t* anc) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < m) anc[j] = static_cast<int32_t>(thread_search(cdf, u[j], 0, cdf.n - 1));
}

// Parallelized cut-point search (Section 3.2): thread j writes its own index
// into the table entries it owns, L_{j-1}+1 .. L_j (1-based), L_j = ceil(n q(j)).
__global__ void k_cutpoint_build(const double* q, int64_t n, int32_t* table) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double dn = static_cast<double>(n);
    const double cj = ceil(dn * q[j]);
    const int64_t Lj = cj < 0.0 ? 0 : (cj > dn ? n : static_cast<int64_t>(cj));
    int64_t Lp = 0;
    if (j > 0) {
        const double cp = ceil(dn * q[j - 1]);
        Lp = cp < 0.0 ? 0 : (cp > dn ? n : static_cast<int64_t>(cp));
    }
    const int64_t top = (j == n - 1) ? n : Lj;
    for (int64_t k = top; k > Lp; --k) table[k - 1] = static_cast<int32_t>(j);
}

// Parallelized cut-point method (Section 3.2): one thread per uniform starts
// at I_{ceil(n u)} and climbs; after 16 climbs it bisects above its position.
__global__ void k_cutpoint_draw(PlainCdf cdf, const int32_t* table, const double* u, int64_t m,
                                int32_t* anc) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int64_t n = cdf.n;
    const double uj = u[j];
    const double ce = ceil(static_cast<double>(n) * uj);
    const int64_t e = !(ce >= 1.0) ? 1 : (ce > static_cast<double>(n) ? n : static_cast<int64_t>(ce));
    // (a table built from a CDF that failed the check may hold anything)
    int64_t k = min(max(static_cast<int64_t>(table[e - 1]), int64_t(0)), n - 1);
    for (int c = 0; c < 16 && k < n - 1 && uj > cdf.q[k]; ++c) ++k;
    if (k < n - 1 && uj > cdf.q[k]) k = thread_search(cdf, uj, k + 1, n - 1);
    anc[j] = static_cast<int32_t>(k);
}

// Merge of a tile of (preferably sorted) uniforms against the CDF staged in
// LDS: the tile's answers lie in [a(min u), a(max u)], walked in windows.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_search_merge(PlainCdf cdf, const double* u, int64_t m,
                                                        int32_t* anc) {
    constexpr int TS = BLOCK * IPT, WIN = 2 * TS, NW = BLOCK / kWave;
    __shared__ double s_q[WIN];
    __shared__ double s_red[NW * 2];
    __shared__ int64_t s_lo, s_hi;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * TS;
    const int64_t n = cdf.n;
    double uu[IPT];
    double umin = INFINITY, umax = -INFINITY;
    for (int i = 0; i < IPT; ++i) {
        const int64_t j = j0 + static_cast<int64_t>(i) * BLOCK + tid;
        uu[i] = j < m ? u[j] : 0.0;
        if (j < m) {
            umin = fmin(umin, uu[i]);
            umax = fmax(umax, uu[i]);
        }
    }
    umin = -wave_max(-umin);
    umax = wave_max(umax);
    if (lane == 0) {
        s_red[wave] = umin;
        s_red[NW + wave] = umax;
    }
    __syncthreads();
    umin = INFINITY;
    umax = -INFINITY;
    for (int q = 0; q < NW; ++q) {
        umin = fmin(umin, s_red[q]);
        umax = fmax(umax, s_red[NW + q]);
    }
    if (wave < 2) {
        const int64_t a = wave_search(cdf, wave == 0 ? umin : umax, 0, n - 1);
        if (lane == 0) {
            if (wave == 0) s_lo = a; else s_hi = a;
        }
    }
    __syncthreads();
    const int64_t a_lo = s_lo, a_hi = max(s_hi, s_lo);
    uint32_t pending = 0;
    for (int i = 0; i < IPT; ++i)
        if (j0 + static_cast<int64_t>(i) * BLOCK + tid < m) pending |= 1u << i;
    if (a_hi - a_lo + 1 > static_cast<int64_t>(kMaxWindows) * WIN) {
        // a bracket of more than kMaxWindows windows: bisection per uniform
        // inside it (exact: every answer lies in [a_lo, a_hi])
        for (int i = 0; i < IPT; ++i)
            if ((pending >> i) & 1u)
                anc[j0 + static_cast<int64_t>(i) * BLOCK + tid] =
                    static_cast<int32_t>(thread_search(cdf, uu[i], a_lo, a_hi));
        return;
    }
    for (int64_t w0 = a_lo; w0 <= a_hi; w0 += WIN) {
        const int cnt = static_cast<int>(min(static_cast<int64_t>(WIN), a_hi - w0 + 1));
        for (int k = tid; k < cnt; k += BLOCK) s_q[k] = cdf.q[w0 + k];
        __syncthreads();
        const bool last = (w0 + cnt - 1 == a_hi);
        const double top = s_q[cnt - 1];
        for (int i = 0; i < IPT; ++i) {
            if ((pending >> i) & 1u) {
                if (last || uu[i] <= top) {
                    int k = lds_lower_bound(s_q, cnt, uu[i]);
                    if (k > cnt - 1) k = cnt - 1;
                    anc[j0 + static_cast<int64_t>(i) * BLOCK + tid] = static_cast<int32_t>(w0 + k);
                    pending &= ~(1u << i);
                }
            }
        }
        __syncthreads();
    }
}

// Non-decreasing and finite check of a plain CDF: sets *bad when violated.
__global__ void k_check_cdf(const double* q, int64_t n, int32_t* bad) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double v = q[k];
    bool b = !isfinite(v);
    if (k > 0 && q[k - 1] > v) b = true;
    if (b) atomicOr(bad, 1);
}

}  // namespace pf

// ------------------------------------------------------------ static scratch
// Device memory of the search entry point that allocates nothing
// (pf_debug_search_noalloc): word 0 is the CDF check flag, the cut-point
// table starts at word kStaticTableOffset (256-byte aligned).  Each GPU the
// library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (static_scratch below), never through the array's name.
static __device__ __align__(256) int32_t scratch[pf::kStaticTableOffset + pf::kStaticCutMax];

// p[0 .. n) = v (clears flags without a memset node, so callers may capture it).
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// ------------------------------------------------------------ launchers
namespace pf {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
hipError_t static_scratch(int32_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

using StepFn = void (*)(StepArgs);

template <int MODEL, typename R, int IPT>
static hipError_t launch_step_t(const StepArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_step<MODEL, R, 256, IPT>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <int MODEL, typename R, int IPT>
static hipError_t launch_init_t(const StepArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_init<MODEL, R, 256, IPT>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int MODEL, typename R>
static hipError_t launch_step_m(const StepArgs& a, int ipt, int grid, hipStream_t s, bool init) {
    switch (ipt) {
    case 1: return init ? launch_init_t<MODEL, R, 1>(a, grid, s) : launch_step_t<MODEL, R, 1>(a, grid, s);
    case 2: return init ? launch_init_t<MODEL, R, 2>(a, grid, s) : launch_step_t<MODEL, R, 2>(a, grid, s);
    case 4: return init ? launch_init_t<MODEL, R, 4>(a, grid, s) : launch_step_t<MODEL, R, 4>(a, grid, s);
    case 8: return init ? launch_init_t<MODEL, R, 8>(a, grid, s) : launch_step_t<MODEL, R, 8>(a, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(int model, bool fp64, int ipt, const StepArgs& a, int grid, hipStream_t s,
                       bool init) {
    switch (model) {
    case kLLPF: return fp64 ? launch_step_m<kLLPF, double>(a, ipt, grid, s, init)
                            : launch_step_m<kLLPF, float>(a, ipt, grid, s, init);
    case kLLPL: return fp64 ? launch_step_m<kLLPL, double>(a, ipt, grid, s, init)
                            : launch_step_m<kLLPL, float>(a, ipt, grid, s, init);
    case kSVPF: return fp64 ? launch_step_m<kSVPF, double>(a, ipt, grid, s, init)
                            : launch_step_m<kSVPF, float>(a, ipt, grid, s, init);
    case kSVPL: return fp64 ? launch_step_m<kSVPL, double>(a, ipt, grid, s, init)
                            : launch_step_m<kSVPL, float>(a, ipt, grid, s, init);
    }
    return hipErrorInvalidValue;
}

template <int MODEL, typename R, int IPT>
static hipError_t launch_batch_t(const StepArgs* descs, const int2* tile_map, BatchState* bs,
                                 int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_step_batch<MODEL, R, 256, IPT>), dim3(grid), dim3(256), 0, s, descs,
                       tile_map, bs);
    return hipGetLastError();
}

template <int MODEL, typename R>
static hipError_t launch_batch_m(int ipt, const StepArgs* descs, const int2* tile_map,
                                 BatchState* bs, int grid, hipStream_t s) {
    switch (ipt) {
    case 1: return launch_batch_t<MODEL, R, 1>(descs, tile_map, bs, grid, s);
    case 2: return launch_batch_t<MODEL, R, 2>(descs, tile_map, bs, grid, s);
    case 4: return launch_batch_t<MODEL, R, 4>(descs, tile_map, bs, grid, s);
    case 8: return launch_batch_t<MODEL, R, 8>(descs, tile_map, bs, grid, s);
    }
    return hipErrorInvalidValue;
}

// One batched cycle: the persistent step kernel over all filters' tiles,
// then the filters' tile scans (capacity bounds the scan grid).
hipError_t launch_batch(int model, bool fp64, int ipt, const StepArgs* descs, const int2* tile_map,
                        int32_t capacity, BatchState* bs, int grid, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    switch (model) {
    case kLLPF: e = fp64 ? launch_batch_m<kLLPF, double>(ipt, descs, tile_map, bs, grid, s)
                         : launch_batch_m<kLLPF, float>(ipt, descs, tile_map, bs, grid, s); break;
    case kLLPL: e = fp64 ? launch_batch_m<kLLPL, double>(ipt, descs, tile_map, bs, grid, s)
                         : launch_batch_m<kLLPL, float>(ipt, descs, tile_map, bs, grid, s); break;
    case kSVPF: e = fp64 ? launch_batch_m<kSVPF, double>(ipt, descs, tile_map, bs, grid, s)
                         : launch_batch_m<kSVPF, float>(ipt, descs, tile_map, bs, grid, s); break;
    case kSVPL: e = fp64 ? launch_batch_m<kSVPL, double>(ipt, descs, tile_map, bs, grid, s)
                         : launch_batch_m<kSVPL, float>(ipt, descs, tile_map, bs, grid, s); break;
    }
    if (e != hipSuccess) return e;
    const int sgrid = capacity < 256 ? (capacity > 0 ? capacity : 1) : 256;
    hipLaunchKernelGGL(k_scan_batch, dim3(sgrid), dim3(kTileScanBlock), 0, s, descs, bs);
    return hipGetLastError();
}

hipError_t launch_batch_map(const int32_t* base, int32_t n_filters, int2* tile_map,
                            hipStream_t s) {
    if (n_filters <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_map, dim3(n_filters), dim3(256), 0, s, base, n_filters, tile_map);
    return hipGetLastError();
}

// Tile counts up to this use the single-work-group scan; above, the chunked
// three-launch scan (chunk buffer: 2 doubles per chunk + G + 1 prefixes).
constexpr int32_t kScanSingleMax = kTileScanBlock * kTileScanPer;

int32_t scan_chunks(int32_t num_tiles) {
    return num_tiles <= kScanSingleMax ? 0 : (num_tiles + kScanBlock - 1) / kScanBlock;
}

hipError_t launch_scan_tiles(double* agg, int32_t num_tiles, int64_t n, int32_t ts, TileAB* ab,
                             int32_t* hint, Totals* tot, DevState* st, double* chunk,
                             const TileAB* pos, hipStream_t s) {
    const int32_t G = scan_chunks(num_tiles);
    if (G == 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kTileScanBlock), 0, s, agg, num_tiles, n, ts,
                           ab, hint, tot, st, pos);
        return hipGetLastError();
    }
    double* pref = chunk + 2 * static_cast<int64_t>(G);
    hipLaunchKernelGGL(k_scan_chunks, dim3(G), dim3(kScanBlock), 0, s,
                       static_cast<const double*>(agg), num_tiles, chunk);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s,
                       static_cast<const double*>(chunk), G, n, pref, tot, st);
    hipLaunchKernelGGL(k_scan_apply, dim3(G), dim3(kScanBlock), 0, s,
                       static_cast<const double*>(agg), num_tiles, n, ts,
                       static_cast<const double*>(pref), static_cast<const Totals*>(tot), ab, hint,
                       pos);
    return hipGetLastError();
}

// The exponential spacings of time t: tile sums, then their tile scan
// (normalised offsets and scale in abE; no hints, no log-likelihood).
hipError_t launch_spacings(int ipt, uint64_t seed, uint32_t t, int64_t n, int32_t num_tiles,
                           double* aggE, TileAB* abE, Totals* totE, double* chunk, hipStream_t s) {
    switch (ipt) {
    case 1: hipLaunchKernelGGL((k_spacing_tiles<256, 1>), dim3(num_tiles), dim3(256), 0, s, seed, t, n, aggE); break;
    case 2: hipLaunchKernelGGL((k_spacing_tiles<256, 2>), dim3(num_tiles), dim3(256), 0, s, seed, t, n, aggE); break;
    case 4: hipLaunchKernelGGL((k_spacing_tiles<256, 4>), dim3(num_tiles), dim3(256), 0, s, seed, t, n, aggE); break;
    default: hipLaunchKernelGGL((k_spacing_tiles<256, 8>), dim3(num_tiles), dim3(256), 0, s, seed, t, n, aggE); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_scan_tiles(aggE, num_tiles, n, 256 * ipt, abE, nullptr, totE, nullptr, chunk,
                             nullptr, s);
}

hipError_t launch_moments(int model, const double* partials, int32_t num_tiles, int64_t n,
                          int32_t weighted, uint32_t t, const ModelParams& p, DevState* st,
                          hipStream_t s) {
    switch (model) {
    case kLLPF: hipLaunchKernelGGL(k_moments<kLLPF>, dim3(1), dim3(256), 0, s, partials, num_tiles, n, weighted, t, p, st); break;
    case kLLPL: hipLaunchKernelGGL(k_moments<kLLPL>, dim3(1), dim3(256), 0, s, partials, num_tiles, n, weighted, t, p, st); break;
    case kSVPF: hipLaunchKernelGGL(k_moments<kSVPF>, dim3(1), dim3(256), 0, s, partials, num_tiles, n, weighted, t, p, st); break;
    case kSVPL: hipLaunchKernelGGL(k_moments<kSVPL>, dim3(1), dim3(256), 0, s, partials, num_tiles, n, weighted, t, p, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cut_table(bool fp64, const void* c, const TileAB* ab, int64_t n, int32_t ts,
                            int32_t tiles, int32_t* table, hipStream_t s) {
    const int64_t grid = (n + 255) / 256;
    if (fp64) {
        CutEnvelope<double> E{static_cast<const double*>(c), ab, n, ts, tiles};
        hipLaunchKernelGGL(k_cut_table<double>, dim3(grid), dim3(256), 0, s, E, table);
    } else {
        CutEnvelope<float> E{static_cast<const float*>(c), ab, n, ts, tiles};
        hipLaunchKernelGGL(k_cut_table<float>, dim3(grid), dim3(256), 0, s, E, table);
    }
    return hipGetLastError();
}

hipError_t launch_search(int strategy, const double* q, int64_t n, const double* u, int64_t m,
                         int32_t* anc, int32_t* table, int32_t* bad, hipStream_t s) {
    const int tb = 256;
    hipLaunchKernelGGL(k_check_cdf, dim3((n + tb - 1) / tb), dim3(tb), 0, s, q, n, bad);
    if (m == 0) return hipGetLastError();
    PlainCdf cdf{q, n};
    if (strategy == kBinary) {
        hipLaunchKernelGGL(k_search_binary, dim3((m + tb - 1) / tb), dim3(tb), 0, s, cdf, u, m, anc);
    } else if (strategy == kCutpoint) {
        hipLaunchKernelGGL(k_cutpoint_build, dim3((n + tb - 1) / tb), dim3(tb), 0, s, q, n, table);
        hipLaunchKernelGGL(k_cutpoint_draw, dim3((m + tb - 1) / tb), dim3(tb), 0, s, cdf, table, u, m, anc);
    } else {
        constexpr int IPT = 4;
        const int64_t grid = (m + 256 * IPT - 1) / (256 * IPT);
        hipLaunchKernelGGL((k_search_merge<256, IPT>), dim3(grid), dim3(256), 0, s, cdf, u, m, anc);
    }
    return hipGetLastError();
}

}  // namespace pf
