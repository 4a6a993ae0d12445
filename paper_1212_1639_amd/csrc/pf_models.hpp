// Device-side random numbers and the per-particle arithmetic of the four
// models: initial draw, propagation (with the particle-learning statistic
// update and parameter draw), log-weight and the per-particle moment terms.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_internal.h"

namespace pf {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products, key bumped by two Weyl constants per round.
struct Words {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox(uint64_t seed, uint32_t index, uint32_t time,
                                        uint32_t stream, uint32_t attempt) {
    uint32_t c0 = index, c1 = time, c2 = stream, c3 = attempt;
    uint32_t key_lo = static_cast<uint32_t>(seed);
    uint32_t key_hi = static_cast<uint32_t>(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32)
        const uint64_t pa = static_cast<uint64_t>(c0) * 0xD2511F53u;
        const uint64_t pb = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
        c0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ key_lo;
        c1 = static_cast<uint32_t>(pb);
        c2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ key_hi;
        c3 = static_cast<uint32_t>(pa);
        key_lo += 0x9E3779B9u;
        key_hi += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Uniform on (0, 1) from one word, in the sampler's precision: 24 bits for
// single precision, 32 bits for double precision.  Both are exact.
template <typename R>
__device__ __forceinline__ R unit(uint32_t w);
template <>
__device__ __forceinline__ float unit<float>(uint32_t w) {
    return (static_cast<float>(w >> 8) + 0.5f) * 0x1p-24f;
}
template <>
__device__ __forceinline__ double unit<double>(uint32_t w) {
    return (static_cast<double>(w) + 0.5) * 0x1p-32;
}
// Resampling uniforms are always formed in double precision.
__device__ __forceinline__ double unit64(uint32_t w) {
    return (static_cast<double>(w) + 0.5) * 0x1p-32;
}

// Arithmetic of the samplers and models in the weights' precision.  Single
// precision uses the hardware's approximate transcendentals and reciprocals
// (a few ulp; the single-precision tolerances are set by the FP32 state
// anyway); double precision keeps correctly rounded division and the
// library's accurate functions, so that it tracks a double-precision
// reference to the last few ulps.
template <typename R>
struct Math;

template <>
struct Math<float> {
    // hardware log2 times ln 2: every argument here is a positive normal
    // number (uniforms are at least 2^-25), which needs none of the
    // denormal scaling of the library's fast log
    __device__ static __forceinline__ float log(float x) {
        return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
    }
    __device__ static __forceinline__ float exp(float x) { return __expf(x); }
    __device__ static __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    __device__ static __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    // sin / cos of 2 pi u for u in [0, 1): the hardware takes revolutions
    __device__ static __forceinline__ void sincos_2pi(float u, float* s, float* c) {
        *s = __builtin_amdgcn_sinf(u);
        *c = __builtin_amdgcn_cosf(u);
    }
};

template <>
struct Math<double> {
    __device__ static __forceinline__ double log(double x) { return ::log(x); }
    __device__ static __forceinline__ double exp(double x) { return ::exp(x); }
    __device__ static __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    __device__ static __forceinline__ double rcp(double x) { return 1.0 / x; }
    __device__ static __forceinline__ double div(double a, double b) { return a / b; }
    __device__ static __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    __device__ static __forceinline__ void sincos_2pi(double u, double* s, double* c) {
        sincospi(2.0 * u, s, c);
    }
};

// Box-Muller pair from two uniforms: r cos(2 pi u2), r sin(2 pi u2).
template <typename R>
__device__ __forceinline__ void box_muller(R u1, R u2, R& z_cos, R& z_sin) {
    const R r = Math<R>::sqrt(R(-2) * Math<R>::log(u1));
    R s, c;
    Math<R>::sincos_2pi(u2, &s, &c);
    z_cos = r * c;
    z_sin = r * s;
}

// Gamma(a, 1), a >= 1, by Marsaglia & Tsang (2000).  The first attempt uses
// the caller's (normal, uniform); attempt k >= 1 draws its own from stream
// kGammaRetry + g at (index, time, ., k): words 0, 1 -> Box-Muller (cosine
// branch), word 2 -> uniform.  After 8 rejections: d = a - 1/3.
template <typename R>
__device__ R gamma_mt(R a, R z, R u, uint64_t seed, uint32_t index, uint32_t time, uint32_t g) {
    using M = Math<R>;
    const R d = a - R(1) / R(3);
    const R c = M::rsqrt(R(9) * d);
    for (uint32_t k = 0; k < 8; ++k) {
        if (k > 0) {
            const Words w = philox(seed, index, time, kGammaRetry + g, k);
            R zs;
            box_muller(unit<R>(w.w0), unit<R>(w.w1), z, zs);
            u = unit<R>(w.w2);
        }
        const R s = R(1) + c * z;
        if (s > R(0)) {
            const R v = s * s * s;
            if (u < R(1) - R(0.0331) * z * z * z * z) return d * v;
            if (M::log(u) < R(0.5) * z * z + d * (R(1) - v + M::log(v))) return d * v;
        }
    }
    return d;
}

template <typename R>
__device__ __forceinline__ R log_norm_pdf(R y, R mean, R var) {
    using M = Math<R>;
    const R e = y - mean;
    return R(-0.5) * M::log(R(6.283185307179586) * var) - R(0.5) * M::div(e * e, var);
}

// ------------------------------------------------------------------ models
// Each model: F record fields, NG per-particle moment terms, WEIGHTED_MOM
// (moments under this step's weights rather than equal weights).
template <int MODEL>
struct ModelDef;

// Local level, known variances; bootstrap filter (Section 2, Algorithm
// "Particle Filtering"; model of Section 4).  Record: x.
template <>
struct ModelDef<kLLPF> {
    static constexpr int F = 1, NG = 2;
    static constexpr bool WEIGHTED_MOM = true;
    template <typename R>
    __device__ static void init(const ModelParams& p, uint64_t seed, uint32_t j, R* z) {
        const Words w = philox(seed, j, 0, kInit, 0);
        R a, b;
        box_muller(unit<R>(w.w0), unit<R>(w.w1), a, b);
        z[0] = R(p.x0_mean) + Math<R>::sqrt(R(p.x0_var)) * a;
    }
    // Step 1: x_t = x~_{t-1} + sqrt(sigma_w2) Z; Z from words 1, 2 of kStep.
    template <typename R>
    __device__ static void propagate(const ModelParams& p, uint64_t, uint32_t, uint32_t, double,
                                     const Words& w, const R* z, R* zn, R* g, bool) {
        R a, b;
        box_muller(unit<R>(w.w1), unit<R>(w.w2), a, b);
        zn[0] = z[0] + Math<R>::sqrt(R(p.sigma_w2)) * a;
        g[0] = zn[0];
        g[1] = zn[0] * zn[0];
    }
    template <typename R>
    __device__ static void terms(const ModelParams&, uint32_t, const R* z, R* g) {
        g[0] = z[0];
        g[1] = z[0] * z[0];
    }
    // Step 2: w proportional to N(y_t; x_t, sigma_v2).
    template <typename R>
    __device__ static R logw(const ModelParams& p, const R* z, double y) {
        return log_norm_pdf(R(y), z[0], R(p.sigma_v2));
    }
};

// Stochastic volatility, known parameters; bootstrap filter.  Record: x.
template <>
struct ModelDef<kSVPF> {
    static constexpr int F = 1, NG = 2;
    static constexpr bool WEIGHTED_MOM = true;
    template <typename R>
    __device__ static void init(const ModelParams& p, uint64_t seed, uint32_t j, R* z) {
        ModelDef<kLLPF>::init(p, seed, j, z);
    }
    template <typename R>
    __device__ static void propagate(const ModelParams& p, uint64_t, uint32_t, uint32_t, double,
                                     const Words& w, const R* z, R* zn, R* g, bool) {
        R a, b;
        box_muller(unit<R>(w.w1), unit<R>(w.w2), a, b);
        zn[0] = R(p.mu) + R(p.phi) * (z[0] - R(p.mu)) + Math<R>::sqrt(R(p.sigma2)) * a;
        g[0] = zn[0];
        g[1] = zn[0] * zn[0];
    }
    template <typename R>
    __device__ static void terms(const ModelParams& p, uint32_t t, const R* z, R* g) {
        ModelDef<kLLPF>::terms(p, t, z, g);
    }
    // y_t ~ N(0, exp(x_t)).
    template <typename R>
    __device__ static R logw(const ModelParams&, const R* z, double y) {
        const R yy = R(y);
        return R(-0.5) * (R(1.8378770664093453) + z[0] + yy * yy * Math<R>::exp(-z[0]));
    }
};

// Local level, unknown variances; particle learning (Section 2, Algorithm
// "Particle Learning"; Section 4).  Record z = (x, b_v, b_w, sigma_v2,
// sigma_w2): the state, the inverse-gamma scales (the shapes a_v + t/2,
// a_w + t/2 are common to all particles) and the parameters drawn at Step 4
// of the previous cycle, which Step 1 weights with.
template <>
struct ModelDef<kLLPL> {
    static constexpr int F = 5, NG = 6;
    static constexpr bool WEIGHTED_MOM = false;
    template <typename R>
    __device__ static void init(const ModelParams& p, uint64_t seed, uint32_t j, R* z) {
        const Words w = philox(seed, j, 0, kInit, 0);
        R zx, zv;
        box_muller(unit<R>(w.w0), unit<R>(w.w1), zx, zv);
        const R uv = unit<R>(w.w2);
        const Words w2 = philox(seed, j, 0, kInit2, 0);
        R zw, unused;
        box_muller(unit<R>(w2.w0), unit<R>(w2.w1), zw, unused);
        const R uw = unit<R>(w2.w2);
        z[0] = R(p.x0_mean) + Math<R>::sqrt(R(p.x0_var)) * zx;
        z[1] = R(p.b_v);
        z[2] = R(p.b_w);
        z[3] = Math<R>::div(R(p.b_v), gamma_mt(R(p.a_v), zv, uv, seed, j, 0, 0));
        z[4] = Math<R>::div(R(p.b_w), gamma_mt(R(p.a_w), zw, uw, seed, j, 0, 1));
    }
    // Steps 2-4 for slot j at time t, from the resampled particle z~ and y_t:
    //   x_t ~ N(V (x~/sigma_w2 + y_t/sigma_v2), V), V = 1/(1/sigma_w2 + 1/sigma_v2);
    //   b_v += (y_t - x_t)^2/2, b_w += (x_t - x~)^2/2;
    //   sigma_v2 ~ IG(a_v + t/2, b_v), sigma_w2 ~ IG(a_w + t/2, b_w).
    // Words: kStep 1,2 -> Box-Muller (x_t, gamma_v normal), 3 -> gamma_v
    // uniform; kStep2 0,1 -> Box-Muller (gamma_w normal), 2 -> gamma_w uniform.
    template <typename R>
    __device__ static void propagate(const ModelParams& p, uint64_t seed, uint32_t j, uint32_t t,
                                     double y, const Words& w, const R* z, R* zn, R* g, bool) {
        R zx, zv;
        box_muller(unit<R>(w.w1), unit<R>(w.w2), zx, zv);
        const R uv = unit<R>(w.w3);
        const Words w2 = philox(seed, j, t, kStep2, 0);
        R zw, unused;
        box_muller(unit<R>(w2.w0), unit<R>(w2.w1), zw, unused);
        const R uw = unit<R>(w2.w2);
        const R yt = R(y);
        const R xp = z[0], sv2 = z[3], sw2 = z[4];
        // V = sv2 sw2 / (sv2 + sw2), m = (sv2 x~ + sw2 y_t) / (sv2 + sw2)
        const R inv = Math<R>::rcp(sv2 + sw2);
        const R V = sv2 * sw2 * inv;
        const R m = (sv2 * xp + sw2 * yt) * inv;
        const R xt = m + Math<R>::sqrt(V) * zx;
        const R bv = z[1] + R(0.5) * (yt - xt) * (yt - xt);
        const R bw = z[2] + R(0.5) * (xt - xp) * (xt - xp);
        const R half_t = R(0.5) * R(t);
        zn[0] = xt;
        zn[1] = bv;
        zn[2] = bw;
        zn[3] = Math<R>::div(bv, gamma_mt(R(p.a_v) + half_t, zv, uv, seed, j, t, 0));
        zn[4] = Math<R>::div(bw, gamma_mt(R(p.a_w) + half_t, zw, uw, seed, j, t, 1));
        terms(p, t, zn, g);
    }
    template <typename R>
    __device__ static void terms(const ModelParams&, uint32_t, const R* z, R* g) {
        g[0] = z[0];
        g[1] = z[0] * z[0];
        g[2] = z[3];
        g[3] = z[4];
        g[4] = z[1];
        g[5] = z[2];
    }
    // Step 1 weight of the next cycle: p(y | z) = N(y; x, sigma_v2 + sigma_w2).
    template <typename R>
    __device__ static R logw(const ModelParams&, const R* z, double y) {
        return log_norm_pdf(R(y), z[0], z[3] + z[4]);
    }
};

// Stochastic volatility, unknown (alpha, beta, sigma^2); propagate, weight,
// resample.  Record z = (x, L01, L11, eta0, eta1, d): the posterior
// precision Lambda = [[L00, L01], [L01, L11]] of (alpha, beta), its
// precision-weighted mean eta, and the inverse-gamma scale d; L00 = p0 + n
// and the shape a_s + n/2 (n transitions seen) are common to all particles.
// The scale is updated by the recursive least-squares identity
//   d' = d + (x_t - z'm)^2 / (2 (1 + z' Lambda^{-1} z)),  z = (1, x~),
// which equals the batch posterior.
template <>
struct ModelDef<kSVPL> {
    static constexpr int F = 6, NG = 6;
    static constexpr bool WEIGHTED_MOM = true;
    template <typename R>
    __device__ static void init(const ModelParams& p, uint64_t seed, uint32_t j, R* z) {
        const Words w = philox(seed, j, 0, kInit, 0);
        R a, b;
        box_muller(unit<R>(w.w0), unit<R>(w.w1), a, b);
        z[0] = R(p.x0_mean) + Math<R>::sqrt(R(p.x0_var)) * a;
        z[1] = R(p.p1);
        z[2] = R(p.p2);
        z[3] = R(p.p0 * p.b0a + p.p1 * p.b0b);
        z[4] = R(p.p1 * p.b0a + p.p2 * p.b0b);
        z[5] = R(p.d_s);
    }
    // Step t for slot j from the resampled particle: sigma^2 ~ IG(a, d);
    // (alpha, beta) = m + sigma L^{-T} (z3, z4), Lambda = L L'; x_t = alpha +
    // beta x~ + sigma z_x; statistics updated with the pair (x~, x_t).
    // Words: kStep 1,2 -> Box-Muller (gamma normal, z_x), 3 -> gamma uniform;
    // kStep2 0,1 -> Box-Muller (z3, z4).  With one_block (single precision
    // under systematic resampling, whose uniform is drawn once per step, so
    // kStep word 0 is free) the five 24-bit uniforms fit one block: the
    // pair for (z3, z4) is word 0 and the low bytes of words 1, 2, 3.
    template <typename R>
    __device__ static void propagate(const ModelParams& p, uint64_t seed, uint32_t j, uint32_t t,
                                     double, const Words& w, const R* z, R* zn, R* g,
                                     bool one_block) {
        R zg, zx;
        box_muller(unit<R>(w.w1), unit<R>(w.w2), zg, zx);
        const R ug = unit<R>(w.w3);
        R z3, z4;
        if (one_block) {
            const uint32_t low = ((w.w1 & 0xffu) << 8) | ((w.w2 & 0xffu) << 16) | ((w.w3 & 0xffu) << 24);
            box_muller(unit<R>(w.w0), unit<R>(low), z3, z4);
        } else {
            const Words w2 = philox(seed, j, t, kStep2, 0);
            box_muller(unit<R>(w2.w0), unit<R>(w2.w1), z3, z4);
        }
        using M = Math<R>;
        const R nprev = R(t) - R(1);
        const R L00 = R(p.p0) + nprev, L01 = z[1], L11 = z[2];
        const R e0 = z[3], e1 = z[4];
        const R idet = M::rcp(L00 * L11 - L01 * L01);
        const R m0 = (L11 * e0 - L01 * e1) * idet;
        const R m1 = (L00 * e1 - L01 * e0) * idet;
        const R a = R(p.a_s) + R(0.5) * nprev;
        const R s2 = M::div(z[5], gamma_mt(a, zg, ug, seed, j, t, 0));
        const R sd = M::sqrt(s2);
        // Lambda = L L' with L = [[l00, 0], [l10, l11]]; solve L' v = (z3, z4)
        const R r00 = M::rsqrt(L00);
        const R l10 = L01 * r00;
        const R r11 = M::rsqrt(L11 - l10 * l10);
        const R v1 = z4 * r11;
        const R v0 = (z3 - l10 * v1) * r00;
        const R alpha = m0 + sd * v0, beta = m1 + sd * v1;
        const R xp = z[0];
        const R xt = alpha + beta * xp + sd * zx;
        // z' Lambda^{-1} z for z = (1, xp), then the recursive update
        const R quad = (L11 - R(2) * L01 * xp + L00 * xp * xp) * idet;
        const R err = xt - (m0 + m1 * xp);
        const R dn = z[5] + R(0.5) * M::div(err * err, R(1) + quad);
        zn[0] = xt;
        zn[1] = L01 + xp;
        zn[2] = L11 + xp * xp;
        zn[3] = e0 + xt;
        zn[4] = e1 + xp * xt;
        zn[5] = dn;
        g[0] = xt;
        g[1] = xt * xt;
        g[2] = alpha;
        g[3] = beta;
        g[4] = s2;
        g[5] = M::div(dn, R(p.a_s) + R(0.5) * R(t) - R(1));
    }
    template <typename R>
    __device__ static void terms(const ModelParams& p, uint32_t t, const R* z, R* g) {
        g[0] = z[0];
        g[1] = z[0] * z[0];
        g[2] = R(0);
        g[3] = R(0);
        g[4] = R(0);
        g[5] = Math<R>::div(z[5], R(p.a_s) + R(0.5) * R(t) - R(1));
    }
    template <typename R>
    __device__ static R logw(const ModelParams& p, const R* z, double y) {
        return ModelDef<kSVPF>::logw(p, z, y);
    }
};

}  // namespace pf
