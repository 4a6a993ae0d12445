/*
 * Plain sequential FP64 oracle for the particle-filter / particle-learning
 * cycle of McAlinn & Nakatsuma, "Parallel Resampling for Fully Parallelized
 * Particle Filters" (arXiv:1212.1639).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load it.  It shares no code, header, table or
 * constant generator with the HIP implementation: the only thing both sides
 * agree on is the *specification* of which random words feed which draw
 * (the counter layout documented beside each model below), and each side
 * implements Philox4x32-10 from its published definition on its own.
 *
 * Everything is computed in IEEE double precision, sequentially, one
 * particle at a time, in the order the paper states the algorithms:
 *   - bootstrap particle filter: Section 2, Algorithm "Particle Filtering";
 *   - particle learning: Section 2, Algorithm "Particle Learning";
 *   - resampling CDF: Section 3.1, equation (resample.cdf);
 *   - multinomial / stratified / systematic uniforms: Section 3.1;
 *   - cut-point method and its parallel table construction: Section 3.2,
 *     Algorithms "Cut-Point Method" and "Parallelized Cut-Point Search",
 *     worked example in Table 1.
 * The stochastic-volatility models are not in the paper; they follow the
 * standard conjugate Normal / inverse-gamma regression posterior and are
 * marked as such where they appear.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Two 32x32->64     */
/* multiplications per round, ten rounds, a Weyl-sequence key schedule.      */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u; /* sqrt(3) - 1  */

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_WEYL_A;
        k1 += PHILOX_WEYL_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Random-word streams.  key = seed; counter = (index, time, stream, attempt). */
enum {
    ST_INIT = 1,      /* initial draws of particle j (time 0)               */
    ST_INIT2 = 5,     /* second block of initial draws                       */
    ST_STEP = 2,      /* main draws of output slot j at time t               */
    ST_STEP2 = 3,     /* second block of draws of slot j at time t           */
    ST_SYSTEMATIC = 4,/* the one offset of systematic resampling at time t   */
    ST_GAMMA0 = 16    /* retries of gamma draw g: stream 16+g, attempt >= 1  */
};

static void words(uint64_t seed, uint32_t j, uint32_t t, uint32_t stream,
                  uint32_t attempt, uint32_t w[4])
{
    uint32_t ctr[4] = {j, t, stream, attempt};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox(ctr, key, w);
}

/* Uniforms on the open interval (0,1).  The 24-bit form is the one a
 * single-precision sampler uses, the 32-bit form the double-precision one;
 * both values are exactly representable, so each side of a comparison can
 * form the same number from the same word. */
double or_u32(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
double or_u24(uint32_t w) { return ((double)(w >> 8) + 0.5) * 0x1p-24; }

static double unif(uint32_t w, int fp32) { return fp32 ? or_u24(w) : or_u32(w); }

/* Box-Muller: two independent standard normals from two uniforms. */
void or_box_muller(double u1, double u2, double z[2])
{
    double r = sqrt(-2.0 * log(u1));
    double a = 2.0 * M_PI * u2;
    z[0] = r * cos(a);
    z[1] = r * sin(a);
}

/* Marsaglia & Tsang (2000), "A simple method for generating gamma
 * variables", for shape a >= 1 and unit scale.  The first attempt uses the
 * (normal, uniform) pair handed in by the caller; attempt k >= 1 takes its
 * pair from stream ST_GAMMA0+g at counter (j, t, 16+g, k): words 0,1 give a
 * Box-Muller normal (cosine branch), word 2 the uniform.  After 8 rejected
 * attempts the draw is d (the value at z = 0). */
#define OR_MT_MAX_ATTEMPTS 8
double or_gamma_mt(double a, double z0, double u0, uint64_t seed, uint32_t j,
                   uint32_t t, uint32_t g, int fp32)
{
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    double z = z0, u = u0;
    for (uint32_t k = 0; k < OR_MT_MAX_ATTEMPTS; ++k) {
        if (k > 0) {
            uint32_t w[4];
            double zz[2];
            words(seed, j, t, ST_GAMMA0 + g, k, w);
            or_box_muller(unif(w[0], fp32), unif(w[1], fp32), zz);
            z = zz[0];
            u = unif(w[2], fp32);
        }
        double s = 1.0 + c * z;
        if (s > 0.0) {
            double v = s * s * s;
            if (u < 1.0 - 0.0331 * z * z * z * z) return d * v;
            if (log(u) < 0.5 * z * z + d * (1.0 - v + log(v))) return d * v;
        }
    }
    return d;
}

/* ------------------------------------------------------------------------ */
/* Resampling (Section 3).                                                   */
/* ------------------------------------------------------------------------ */

/* Resampling CDF, equation (resample.cdf): q(i) proportional to the running
 * sum of the weights, normalised so that q(N) = 1.  The weights are given
 * as log-weights; they are shifted by their maximum M before
 * exponentiation.  Returns M and the shifted total S so that the per-step
 * likelihood estimate (1/N) sum_i p(y|x_i) equals exp(M) * S / N. */
void or_cdf(const double* logw, int64_t n, double* q, double* M_out, double* S_out)
{
    double M = -INFINITY;
    for (int64_t i = 0; i < n; ++i)
        if (logw[i] > M) M = logw[i];
    double run = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        run += exp(logw[i] - M);
        q[i] = run;
    }
    double S = run;
    for (int64_t i = 0; i < n; ++i) q[i] = q[i] / S;
    if (n > 0) q[n - 1] = 1.0;
    *M_out = M;
    *S_out = S;
}

/* Inverse CDF by brute force: the first index whose CDF value reaches u.
 * Indices are 0-based here; if no value reaches u, the last index. */
int64_t or_search_brute(const double* q, int64_t n, double u)
{
    for (int64_t k = 0; k < n; ++k)
        if (q[k] >= u) return k;
    return n - 1;
}

/* Inverse CDF by bisection on a non-decreasing q (same result as brute). */
int64_t or_search_binary(const double* q, int64_t n, double u)
{
    int64_t lo = 0, hi = n - 1; /* answer in [lo, hi]; hi is a fallback */
    if (n <= 0) return -1;
    if (q[n - 1] < u) return n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (q[mid] >= u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Cut-point table (Section 3.2, Chen & Asau): I_k is the smallest i whose
 * CDF value exceeds (k-1)/N.  It is built the way the parallel cut-point
 * search of Section 3.2 builds it: with L_j = ceil(N q(j)) and L_0 = 0,
 * particle j owns the table entries k = L_{j-1}+1 .. L_j and writes its own
 * index into each of them; when L_{j-1} = L_j it owns none.  The loop over
 * j below is what each of the N threads does, run one after the other.
 * The last particle also owns every entry above L_N (they exist only if
 * q(N) < 1).  L and I are 1-based in the paper and 0-based here: entry k
 * of the paper is I[k-1] and holds a 0-based particle index.  The
 * products N q(j) and N u are both formed in double precision, so
 * rounding is monotone and the start index never passes the answer. */
void or_cutpoint_table(const double* q, int64_t n, int64_t* L, int64_t* I)
{
    for (int64_t j = 0; j < n; ++j) {
        double c = ceil((double)n * q[j]);
        int64_t Lj = c < 0.0 ? 0 : (c > (double)n ? n : (int64_t)c);
        L[j] = Lj;
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t prev = j == 0 ? 0 : L[j - 1];
        int64_t top = (j == n - 1) ? n : L[j];
        for (int64_t k = top; k > prev; --k) I[k - 1] = j;
    }
}

/* Cut-point draw (Section 3.2, Algorithm "Cut-Point Method", one uniform):
 * start at the table entry ceil(N u) and move up the CDF while u is still
 * above it.  *climbs receives the number of moves. */
int64_t or_cutpoint_draw(const double* q, const int64_t* I, int64_t n, double u,
                         int64_t* climbs)
{
    double c = ceil((double)n * u);
    int64_t e = c < 1.0 ? 1 : (c > (double)n ? n : (int64_t)c);
    int64_t k = I[e - 1];
    int64_t moves = 0;
    while (k < n - 1 && u > q[k]) { ++k; ++moves; }
    if (climbs) *climbs = moves;
    return k;
}

enum { OR_SEARCH_BINARY = 0, OR_SEARCH_CUTPOINT = 1, OR_SEARCH_BRUTE = 2 };

void or_resample(const double* q, int64_t n, const double* u, int64_t m, int method,
                 int64_t* anc)
{
    if (method == OR_SEARCH_CUTPOINT) {
        int64_t* L = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        int64_t* I = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        or_cutpoint_table(q, n, L, I);
        for (int64_t j = 0; j < m; ++j) anc[j] = or_cutpoint_draw(q, I, n, u[j], NULL);
        free(L);
        free(I);
    } else if (method == OR_SEARCH_BRUTE) {
        for (int64_t j = 0; j < m; ++j) anc[j] = or_search_brute(q, n, u[j]);
    } else {
        for (int64_t j = 0; j < m; ++j) anc[j] = or_search_binary(q, n, u[j]);
    }
}

/* Resampling uniforms for time t (Section 3.1).
 *   multinomial: u_j i.i.d. uniform, word 0 of ST_STEP at (j, t);
 *   stratified:  u_j = (j + U_j)/N with U_j from the same word;
 *   systematic:  u_j = (j + U)/N with the one U from word 0 of
 *                ST_SYSTEMATIC at (0, t);
 *   sorted multinomial: the order statistics of N i.i.d. uniforms, formed
 *                without sorting from exponential spacings: with
 *                E_i = -log U_i (U_i from word 0 of ST_STEP at (i, t),
 *                i = 0..N) and P_j = E_0 + ... + E_j, u_j = P_j / P_N.
 *                The ancestors' counts are multinomial exactly; the slots
 *                receive them in increasing order.
 * j is 0-based, so stratum j is [j/N, (j+1)/N]. */
enum { OR_MULTINOMIAL = 0, OR_STRATIFIED = 1, OR_SYSTEMATIC = 2, OR_SORTED_MULTINOMIAL = 3 };

/* Exponential spacing E_i = -log U_i of index i at time t. */
static double spacing(uint64_t seed, uint32_t t, int64_t i)
{
    uint32_t w[4];
    words(seed, (uint32_t)i, t, ST_STEP, 0, w);
    return -log(or_u32(w[0]));
}

/* Uniform u_j of slot j; U_sys is the systematic offset of time t. */
static double slot_uniform(int scheme, uint64_t seed, uint32_t t, int64_t n, int64_t j,
                           double U_sys)
{
    uint32_t w[4];
    if (scheme == OR_SYSTEMATIC) return ((double)j + U_sys) / (double)n;
    words(seed, (uint32_t)j, t, ST_STEP, 0, w);
    double Uj = or_u32(w[0]);
    return scheme == OR_STRATIFIED ? ((double)j + Uj) / (double)n : Uj;
}

static double systematic_offset(int scheme, uint64_t seed, uint32_t t)
{
    uint32_t w[4];
    if (scheme != OR_SYSTEMATIC) return 0.0;
    words(seed, 0, t, ST_SYSTEMATIC, 0, w);
    return or_u32(w[0]);
}

void or_uniforms(int scheme, uint64_t seed, uint32_t t, int64_t n, double* u)
{
    if (scheme == OR_SORTED_MULTINOMIAL) {
        double P = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            P += spacing(seed, t, j);
            u[j] = P;
        }
        const double PN = P + spacing(seed, t, n);
        for (int64_t j = 0; j < n; ++j) u[j] /= PN;
        return;
    }
    const double U = systematic_offset(scheme, seed, t);
    for (int64_t j = 0; j < n; ++j) u[j] = slot_uniform(scheme, seed, t, n, j, U);
}

/* ------------------------------------------------------------------------ */
/* Models and filters.                                                       */
/* ------------------------------------------------------------------------ */
enum { OR_LL_PF = 0, OR_LL_PL = 1, OR_SV_PF = 2, OR_SV_PL = 3 };

typedef struct or_config {
    int32_t model;      /* OR_LL_PF, OR_LL_PL, OR_SV_PF, OR_SV_PL          */
    int32_t scheme;     /* OR_MULTINOMIAL, OR_STRATIFIED, OR_SYSTEMATIC    */
    int32_t search;     /* OR_SEARCH_*                                     */
    int32_t fp32_words; /* 1: samplers use 24-bit uniforms (single-precision
                           semantics of the random draws); 0: 32-bit       */
    int64_t n;          /* particles                                       */
    uint64_t seed;
    double x0_mean, x0_var;
    double sigma_v2, sigma_w2;     /* local level, known variances         */
    double a_v, b_v, a_w, b_w;     /* local level, IG priors (PL)          */
    double mu, phi, sigma2;        /* stochastic volatility, known (PF)     */
    double prior_mean[2];          /* SV-PL: (alpha, beta) | sigma^2 mean   */
    double prior_prec[3];          /* SV-PL: Lambda0 = [[p0, p1], [p1, p2]] */
    double a_s, d_s;               /* SV-PL: IG prior of sigma^2            */
} or_config;

/* Number of fields each model keeps per particle in the dumps. */
int or_fields(int model)
{
    switch (model) {
    case OR_LL_PF: return 1;  /* x                                             */
    case OR_LL_PL: return 5;  /* x, b_v, b_w, sigma_v^2, sigma_w^2             */
    case OR_SV_PF: return 1;  /* x                                             */
    case OR_SV_PL: return 7;  /* x, n, S1, S11, Sy, S1y, Syy (raw sums)        */
    }
    return 0;
}

#define OR_NMOM 8

static double log_normal_pdf(double y, double mean, double var)
{
    double e = y - mean;
    return -0.5 * log(2.0 * M_PI * var) - 0.5 * e * e / var;
}

/* Output of a run, per step t = 1..T (row t-1):
 *   loglik[t-1]            log of the step's likelihood estimate
 *                          (1/N) sum_i p(y_t | particle i), equation
 *                          (pf.resampling)'s denominator;
 *   mom[(t-1)*OR_NMOM + k] model-dependent moments (see each model);
 *   anc  (optional) [(t-1)*N + j] ancestor chosen for slot j at step t;
 *   state(optional) [((t-1)*F + f)*N + i] field f of particle i after step t;
 *   logw (optional) [(t-1)*N + i] log-weight of particle i at step t.
 * Returns 0, or -1 when every weight of some step is zero or not finite. */

/* Propagation of one output slot j at time t from its resampled
 * ancestor's fields zk[0..F-1] (F = or_fields(model)); writes the slot's new
 * fields to out[0..F-1].  The filters below call these for every slot; the
 * sampled step (or_step_slots) calls them for a few. */

/* Local level, known variances: x_t = x~ + sqrt(sigma_w2) Z, Z from words
 * 1, 2 of ST_STEP (j, t). */
static void ll_pf_slot(const or_config* c, const double* zk, uint32_t j, uint32_t t, double* out)
{
    uint32_t w[4];
    double z[2];
    words(c->seed, j, t, ST_STEP, 0, w);
    or_box_muller(unif(w[1], c->fp32_words), unif(w[2], c->fp32_words), z);
    out[0] = zk[0] + sqrt(c->sigma_w2) * z[0];
}

/* Stochastic volatility, known parameters: x_t = mu + phi (x~ - mu) + sigma Z. */
static void sv_pf_slot(const or_config* c, const double* zk, uint32_t j, uint32_t t, double* out)
{
    uint32_t w[4];
    double z[2];
    const double sd = sqrt(c->sigma2);
    words(c->seed, j, t, ST_STEP, 0, w);
    or_box_muller(unif(w[1], c->fp32_words), unif(w[2], c->fp32_words), z);
    out[0] = c->mu + c->phi * (zk[0] - c->mu) + sd * z[0];
}

/* Local-level bootstrap particle filter (Section 2, Algorithm "Particle
 * Filtering"; model of Section 4, equation (trend+noise), known variances).
 * Step 0: x~_0 ~ N(x0_mean, x0_var).  At t = 1 there is nothing to
 * resample; at t >= 2 the slots are first resampled with the weights of
 * t-1 (this is Step 3 of t-1).  Step 1: x_t = x~_{t-1} + sqrt(sigma_w2) Z.
 * Step 2: w_t proportional to N(y_t; x_t, sigma_v2).
 * Draws: init ST_INIT(j,0) words 0,1 -> Box-Muller, cosine branch;
 * step ST_STEP(j,t) word 0 -> resampling uniform, words 1,2 -> normal.
 * Moments (weights w_t, before resampling): E x, Var x, ESS. */
static int run_ll_pf(const or_config* c, const double* y, int64_t T, double* loglik,
                     double* mom, int64_t* anc_out, double* state_out, double* logw_out,
                     const double* state0, int64_t t0, double y_prev, const int64_t* anc_first)
{
    const int64_t N = c->n;
    const int fp32 = c->fp32_words;
    double* x = (double*)malloc(sizeof(double) * N);
    double* xn = (double*)malloc(sizeof(double) * N);
    double* lw = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    double* u = (double*)malloc(sizeof(double) * N);
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * N);
    uint32_t w[4];
    double z[2];
    int rc = 0;
    for (int64_t i = 0; i < N && !state0; ++i) {
        words(c->seed, (uint32_t)i, 0, ST_INIT, 0, w);
        or_box_muller(unif(w[0], fp32), unif(w[1], fp32), z);
        x[i] = c->x0_mean + sqrt(c->x0_var) * z[0];
    }
    if (state0) {
        /* start from given particles x_{t0}; their weights are those of y_{t0} */
        memcpy(x, state0, sizeof(double) * N);
        if (t0 >= 1) {
            for (int64_t i = 0; i < N; ++i) lw[i] = log_normal_pdf(y_prev, x[i], c->sigma_v2);
            double M0, S0;
            or_cdf(lw, N, q, &M0, &S0);
        }
    }
    for (int64_t t = t0 + 1; t <= t0 + T; ++t) {
        const int64_t r = t - t0 - 1; /* output row */
        if (t == 1) {
            for (int64_t j = 0; j < N; ++j) a[j] = j;
        } else if (r == 0 && anc_first) {
            memcpy(a, anc_first, sizeof(int64_t) * N);
        } else {
            or_uniforms(c->scheme, c->seed, (uint32_t)t, N, u);
            or_resample(q, N, u, N, c->search, a);
        }
        for (int64_t j = 0; j < N; ++j) ll_pf_slot(c, &x[a[j]], (uint32_t)j, (uint32_t)t, &xn[j]);
        memcpy(x, xn, sizeof(double) * N);
        for (int64_t i = 0; i < N; ++i) lw[i] = log_normal_pdf(y[r], x[i], c->sigma_v2);
        double M, S;
        or_cdf(lw, N, q, &M, &S);
        if (!(S > 0.0) || !isfinite(S) || !isfinite(M)) { rc = -1; }
        loglik[r] = M + log(S / (double)N);
        double sw = 0, swx = 0, swxx = 0, sww = 0;
        for (int64_t i = 0; i < N; ++i) {
            double wi = exp(lw[i] - M);
            sw += wi; swx += wi * x[i]; swxx += wi * x[i] * x[i]; sww += wi * wi;
        }
        double* m = mom + r * OR_NMOM;
        for (int k = 0; k < OR_NMOM; ++k) m[k] = 0.0;
        m[0] = swx / sw;
        m[1] = swxx / sw - m[0] * m[0];
        m[2] = sw * sw / sww;
        if (anc_out) for (int64_t j = 0; j < N; ++j) anc_out[r * N + j] = a[j];
        if (state_out) memcpy(state_out + r * N, x, sizeof(double) * N);
        if (logw_out) memcpy(logw_out + r * N, lw, sizeof(double) * N);
    }
    free(x); free(xn); free(lw); free(q); free(u); free(a);
    return rc;
}

/* Stochastic-volatility bootstrap filter with known (mu, phi, sigma2)
 * (not in the paper): x_t = mu + phi (x_{t-1} - mu) + sigma Z,
 * y_t ~ N(0, exp(x_t)).  Same cycle, draws and moments as run_ll_pf. */
static int run_sv_pf(const or_config* c, const double* y, int64_t T, double* loglik,
                     double* mom, int64_t* anc_out, double* state_out, double* logw_out,
                     const double* state0, int64_t t0, double y_prev, const int64_t* anc_first)
{
    const int64_t N = c->n;
    const int fp32 = c->fp32_words;
    double* x = (double*)malloc(sizeof(double) * N);
    double* xn = (double*)malloc(sizeof(double) * N);
    double* lw = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    double* u = (double*)malloc(sizeof(double) * N);
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * N);
    uint32_t w[4];
    double z[2];
    int rc = 0;
    for (int64_t i = 0; i < N && !state0; ++i) {
        words(c->seed, (uint32_t)i, 0, ST_INIT, 0, w);
        or_box_muller(unif(w[0], fp32), unif(w[1], fp32), z);
        x[i] = c->x0_mean + sqrt(c->x0_var) * z[0];
    }
    if (state0) {
        /* start from given particles x_{t0}; their weights are those of y_{t0} */
        memcpy(x, state0, sizeof(double) * N);
        if (t0 >= 1) {
            for (int64_t i = 0; i < N; ++i) lw[i] = log_normal_pdf(y_prev, 0.0, exp(x[i]));
            double M0, S0;
            or_cdf(lw, N, q, &M0, &S0);
        }
    }
    for (int64_t t = t0 + 1; t <= t0 + T; ++t) {
        const int64_t r = t - t0 - 1; /* output row */
        if (t == 1) {
            for (int64_t j = 0; j < N; ++j) a[j] = j;
        } else if (r == 0 && anc_first) {
            memcpy(a, anc_first, sizeof(int64_t) * N);
        } else {
            or_uniforms(c->scheme, c->seed, (uint32_t)t, N, u);
            or_resample(q, N, u, N, c->search, a);
        }
        for (int64_t j = 0; j < N; ++j) sv_pf_slot(c, &x[a[j]], (uint32_t)j, (uint32_t)t, &xn[j]);
        memcpy(x, xn, sizeof(double) * N);
        for (int64_t i = 0; i < N; ++i) lw[i] = log_normal_pdf(y[r], 0.0, exp(x[i]));
        double M, S;
        or_cdf(lw, N, q, &M, &S);
        if (!(S > 0.0) || !isfinite(S) || !isfinite(M)) { rc = -1; }
        loglik[r] = M + log(S / (double)N);
        double sw = 0, swx = 0, swxx = 0, sww = 0;
        for (int64_t i = 0; i < N; ++i) {
            double wi = exp(lw[i] - M);
            sw += wi; swx += wi * x[i]; swxx += wi * x[i] * x[i]; sww += wi * wi;
        }
        double* m = mom + r * OR_NMOM;
        for (int k = 0; k < OR_NMOM; ++k) m[k] = 0.0;
        m[0] = swx / sw;
        m[1] = swxx / sw - m[0] * m[0];
        m[2] = sw * sw / sww;
        if (anc_out) for (int64_t j = 0; j < N; ++j) anc_out[r * N + j] = a[j];
        if (state_out) memcpy(state_out + r * N, x, sizeof(double) * N);
        if (logw_out) memcpy(logw_out + r * N, lw, sizeof(double) * N);
    }
    free(x); free(xn); free(lw); free(q); free(u); free(a);
    return rc;
}

/* Local-level particle learning (Section 2, Algorithm "Particle Learning",
 * with the model and unknown (sigma_v^2, sigma_w^2) of Section 4).  The
 * particle is z = (x, s, theta) with s = (b_v, b_w); the shapes
 * a_v + t/2 and a_w + t/2 are the same for every particle.
 * Step 0: x_0 ~ N(x0_mean, x0_var), s_0 = (b_v, b_w) of the prior,
 *         theta_0 = (sigma_v^2, sigma_w^2) drawn from the IG priors.
 * For t = 1..T:
 *   Step 1: w proportional to p(y_t | z_{t-1}) = N(y_t; x, sigma_v^2 + sigma_w^2);
 *           resample z~_{t-1} with these weights.
 *   Step 2: x_t ~ p(x_t | z~_{t-1}, y_t) = N(m, V) with
 *           V = 1/(1/sigma_w^2 + 1/sigma_v^2), m = V (x~/sigma_w^2 + y_t/sigma_v^2).
 *   Step 3: b_v += (y_t - x_t)^2 / 2, b_w += (x_t - x~_{t-1})^2 / 2.
 *   Step 4: sigma_v^2 ~ IG(a_v + t/2, b_v), sigma_w^2 ~ IG(a_w + t/2, b_w).
 * Draws:
 *   init  ST_INIT(j,0):  words 0,1 -> Box-Muller (z1 -> x_0, z2 -> gamma_v normal),
 *                        word 2 -> gamma_v uniform;
 *         ST_INIT2(j,0): words 0,1 -> Box-Muller (z3 -> gamma_w normal),
 *                        word 2 -> gamma_w uniform;
 *   step  ST_STEP(j,t):  word 0 -> resampling uniform;
 *                        words 1,2 -> Box-Muller (z1 -> x_t, z2 -> gamma_v normal),
 *                        word 3 -> gamma_v uniform;
 *         ST_STEP2(j,t): words 0,1 -> Box-Muller (z3 -> gamma_w normal),
 *                        word 2 -> gamma_w uniform;
 *   gamma retries: g = 0 for sigma_v^2, g = 1 for sigma_w^2.
 * Moments of z_t, equal weights after propagation: E x, Var x,
 *   mean of the drawn sigma_v^2 and sigma_w^2 (Section 2, posterior
 *   statistics from the theta sample), and the Rao-Blackwell means
 *   b/(a - 1) of the two IG posteriors. */
/* Steps 2-4 of particle learning for slot j at time t, from the resampled
 * particle zk = (x~, b_v, b_w, sigma_v^2, sigma_w^2) and y_t. */
static void ll_pl_slot(const or_config* c, const double* zk, uint32_t j, uint32_t t, double yt,
                       double* out)
{
    const int fp32 = c->fp32_words;
    uint32_t w[4];
    double g[2];
    const double av = c->a_v + 0.5 * (double)t, aw = c->a_w + 0.5 * (double)t;
    const double xp = zk[0], sv2 = zk[3], sw2 = zk[4];
    words(c->seed, j, t, ST_STEP, 0, w);
    or_box_muller(unif(w[1], fp32), unif(w[2], fp32), g);
    double z_x = g[0], z_v = g[1], u_v = unif(w[3], fp32);
    words(c->seed, j, t, ST_STEP2, 0, w);
    or_box_muller(unif(w[0], fp32), unif(w[1], fp32), g);
    double z_w = g[0], u_w = unif(w[2], fp32);
    /* Step 2 */
    double V = 1.0 / (1.0 / sw2 + 1.0 / sv2);
    double m = V * (xp / sw2 + yt / sv2);
    double xt = m + sqrt(V) * z_x;
    /* Step 3 */
    double bv = zk[1] + 0.5 * (yt - xt) * (yt - xt);
    double bw = zk[2] + 0.5 * (xt - xp) * (xt - xp);
    /* Step 4 */
    out[0] = xt;
    out[1] = bv;
    out[2] = bw;
    out[3] = bv / or_gamma_mt(av, z_v, u_v, c->seed, j, t, 0, fp32);
    out[4] = bw / or_gamma_mt(aw, z_w, u_w, c->seed, j, t, 1, fp32);
}

static int run_ll_pl(const or_config* c, const double* y, int64_t T, double* loglik,
                     double* mom, int64_t* anc_out, double* state_out, double* logw_out,
                     const double* state0, int64_t t0, double y_prev, const int64_t* anc_first)
{
    const int64_t N = c->n;
    const int fp32 = c->fp32_words;
    const int F = 5;
    double* z = (double*)malloc(sizeof(double) * N * F);  /* [f*N + i] */
    double* zn = (double*)malloc(sizeof(double) * N * F);
    double* lw = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    double* u = (double*)malloc(sizeof(double) * N);
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * N);
    uint32_t w[4];
    double g[2];
    int rc = 0;
    if (state0) memcpy(z, state0, sizeof(double) * N * F); /* z_{t0} given */
    for (int64_t i = 0; i < N && !state0; ++i) {
        words(c->seed, (uint32_t)i, 0, ST_INIT, 0, w);
        or_box_muller(unif(w[0], fp32), unif(w[1], fp32), g);
        double u_v = unif(w[2], fp32);
        z[0 * N + i] = c->x0_mean + sqrt(c->x0_var) * g[0];
        double z_v = g[1];
        words(c->seed, (uint32_t)i, 0, ST_INIT2, 0, w);
        or_box_muller(unif(w[0], fp32), unif(w[1], fp32), g);
        double z_w = g[0], u_w = unif(w[2], fp32);
        z[1 * N + i] = c->b_v;
        z[2 * N + i] = c->b_w;
        z[3 * N + i] = c->b_v / or_gamma_mt(c->a_v, z_v, u_v, c->seed, (uint32_t)i, 0, 0, fp32);
        z[4 * N + i] = c->b_w / or_gamma_mt(c->a_w, z_w, u_w, c->seed, (uint32_t)i, 0, 1, fp32);
    }
    for (int64_t t = t0 + 1; t <= t0 + T; ++t) {
        const int64_t r = t - t0 - 1; /* output row */
        const double yt = y[r];
        /* Step 1 */
        for (int64_t i = 0; i < N; ++i)
            lw[i] = log_normal_pdf(yt, z[0 * N + i], z[3 * N + i] + z[4 * N + i]);
        double M, S;
        or_cdf(lw, N, q, &M, &S);
        if (!(S > 0.0) || !isfinite(S) || !isfinite(M)) { rc = -1; }
        loglik[r] = M + log(S / (double)N);
        if (r == 0 && anc_first) {
            memcpy(a, anc_first, sizeof(int64_t) * N);
        } else {
            or_uniforms(c->scheme, c->seed, (uint32_t)t, N, u);
            or_resample(q, N, u, N, c->search, a);
        }
        const double av = c->a_v + 0.5 * (double)t, aw = c->a_w + 0.5 * (double)t;
        for (int64_t j = 0; j < N; ++j) {
            double zk[5], out[5];
            for (int f = 0; f < F; ++f) zk[f] = z[f * N + a[j]];
            ll_pl_slot(c, zk, (uint32_t)j, (uint32_t)t, yt, out);
            for (int f = 0; f < F; ++f) zn[f * N + j] = out[f];
        }
        memcpy(z, zn, sizeof(double) * N * F);
        double sx = 0, sxx = 0, sv = 0, sw = 0, rv = 0, rw = 0;
        for (int64_t i = 0; i < N; ++i) {
            double xi = z[0 * N + i];
            sx += xi; sxx += xi * xi;
            sv += z[3 * N + i]; sw += z[4 * N + i];
            rv += z[1 * N + i] / (av - 1.0);
            rw += z[2 * N + i] / (aw - 1.0);
        }
        double* mo = mom + r * OR_NMOM;
        for (int k = 0; k < OR_NMOM; ++k) mo[k] = 0.0;
        mo[0] = sx / N;
        mo[1] = sxx / N - mo[0] * mo[0];
        mo[2] = sv / N;
        mo[3] = sw / N;
        mo[4] = rv / N;
        mo[5] = rw / N;
        if (anc_out) for (int64_t j = 0; j < N; ++j) anc_out[r * N + j] = a[j];
        if (state_out) memcpy(state_out + r * N * F, z, sizeof(double) * N * F);
        if (logw_out) memcpy(logw_out + r * N, lw, sizeof(double) * N);
    }
    free(z); free(zn); free(lw); free(q); free(u); free(a);
    return rc;
}

/* Stochastic-volatility particle learning (not in the paper; Storvik-type
 * order: propagate, weight, resample, as in the bootstrap cycle).
 * Transition x_t = alpha + beta x_{t-1} + sigma Z, i.e. alpha = mu (1 - phi),
 * beta = phi; observation y_t ~ N(0, exp(x_t)).  The parameters
 * (alpha, beta, sigma^2) have the conjugate Normal / inverse-gamma prior
 * (alpha, beta) | sigma^2 ~ N(b0, sigma^2 Lambda0^{-1}), sigma^2 ~ IG(a0, d0).
 * Each particle keeps the raw sums of its own path that the regression of
 * x_s on (1, x_{s-1}) needs: n, S1 = sum x_{s-1}, S11 = sum x_{s-1}^2,
 * Sy = sum x_s, S1y = sum x_{s-1} x_s, Syy = sum x_s^2.  The posterior is
 * then, by its definition,
 *   Lambda = Lambda0 + [[n, S1], [S1, S11]],  eta = Lambda0 b0 + (Sy, S1y),
 *   m = Lambda^{-1} eta,  a = a0 + n/2,
 *   d = d0 + (Syy + b0' Lambda0 b0 - m' Lambda m) / 2.
 * Step t: (x~, sums~) = resampled particle (identity at t = 1);
 *   sigma^2 ~ IG(a, d) from sums~;  (alpha, beta) = m + sigma * L^{-T} (z3, z4)
 *   with Lambda = L L' (lower Cholesky factor);
 *   x_t = alpha + beta x~ + sigma z2;  sums += the new pair (x~, x_t);
 *   w_t proportional to N(y_t; 0, exp(x_t)).
 * Draws: init ST_INIT(j,0) words 0,1 -> Box-Muller, z1 -> x_0;
 *   step ST_STEP(j,t): word 0 -> resampling uniform; words 1,2 ->
 *   Box-Muller (z1 -> gamma normal, z2 -> x_t), word 3 -> gamma uniform;
 *   ST_STEP2(j,t): words 0,1 -> Box-Muller (z3, z4) for (alpha, beta);
 *   gamma retries g = 0.
 * Moments (weights w_t, before resampling): E x, Var x, E alpha, E beta,
 *   E sigma^2 of the draws that produced x_t, ESS, and the Rao-Blackwell
 *   mean d/(a-1) of sigma^2 after the update. */
/* Conjugate Normal / inverse-gamma posterior of the regression
 * x_s = alpha + beta x_{s-1} + sigma e_s from the raw sums of one path
 * (definition of the posterior, written out):
 *   Lambda = Lambda0 + [[n, S1], [S1, S11]],  eta = Lambda0 b0 + (Sy, S1y),
 *   m = Lambda^{-1} eta,  a = a0 + n/2,
 *   d = d0 + (Syy + b0' Lambda0 b0 - m' Lambda m) / 2.
 * sums = (n, S1, S11, Sy, S1y, Syy); out = (L00, L01, L11, m0, m1, a, d). */
void or_sv_posterior(const or_config* c, const double sums[6], double out[7])
{
    const double P0 = c->prior_prec[0], P1 = c->prior_prec[1], P2 = c->prior_prec[2];
    const double b0a = c->prior_mean[0], b0b = c->prior_mean[1];
    const double eta0a = P0 * b0a + P1 * b0b, eta0b = P1 * b0a + P2 * b0b;
    const double L00 = P0 + sums[0], L01 = P1 + sums[1], L11 = P2 + sums[2];
    const double ea = eta0a + sums[3], eb = eta0b + sums[4];
    const double det = L00 * L11 - L01 * L01;
    const double ma = (L11 * ea - L01 * eb) / det;
    const double mb = (L00 * eb - L01 * ea) / det;
    out[0] = L00; out[1] = L01; out[2] = L11;
    out[3] = ma; out[4] = mb;
    out[5] = c->a_s + 0.5 * sums[0];
    out[6] = c->d_s + 0.5 * (sums[5] + (b0a * eta0a + b0b * eta0b) - (ma * ea + mb * eb));
}

/* One draw of theta = (alpha, beta, sigma^2) from the posterior `post`
 * (layout of or_sv_posterior): sigma^2 = d / Gamma(a) with the gamma's
 * first attempt on (z_g, u_g), then (alpha, beta) = m + sigma L^{-T} (z3, z4)
 * where Lambda = L L' is the lower Cholesky factor. */
void or_sv_theta(const double post[7], double z_g, double u_g, double z3, double z4,
                 uint64_t seed, uint32_t j, uint32_t t, int fp32, double theta[3])
{
    double s2 = post[6] / or_gamma_mt(post[5], z_g, u_g, seed, j, t, 0, fp32);
    double sd = sqrt(s2);
    double l00 = sqrt(post[0]), l10 = post[1] / l00;
    double l11 = sqrt(post[2] - l10 * l10);
    double v1 = z4 / l11;
    double v0 = (z3 - l10 * v1) / l00;
    theta[0] = post[3] + sd * v0;
    theta[1] = post[4] + sd * v1;
    theta[2] = s2;
}

/* Step t of stochastic-volatility particle learning for slot j from the
 * resampled particle zk = (x~, n, S1, S11, Sy, S1y, Syy): theta from the
 * posterior of the sums, x_t, the sums updated with the pair (x~, x_t).
 * theta[] receives the draw, *rb the Rao-Blackwell mean d/(a-1) of sigma^2
 * after the update. */
static void sv_pl_slot(const or_config* c, const double* zk, uint32_t j, uint32_t t,
                       double* out, double theta[3], double* rb)
{
    const int fp32 = c->fp32_words;
    uint32_t w[4];
    double g[2];
    const double xp = zk[0];
    double sums[6], post[7];
    for (int f = 0; f < 6; ++f) sums[f] = zk[f + 1];
    or_sv_posterior(c, sums, post);
    words(c->seed, j, t, ST_STEP, 0, w);
    or_box_muller(unif(w[1], fp32), unif(w[2], fp32), g);
    double z_g = g[0], z_x = g[1], u_g = unif(w[3], fp32);
    if (fp32 && c->scheme == OR_SYSTEMATIC) {
        /* 24-bit uniforms under systematic resampling, whose uniform is
         * drawn once per step so that word 0 is free: the slot's five
         * uniforms fit one block, the (z3, z4) pair taking word 0 and the
         * low bytes of words 1, 2, 3 (as the high 24 bits of a word) */
        const uint32_t low = ((w[1] & 0xffu) << 8) | ((w[2] & 0xffu) << 16) | ((w[3] & 0xffu) << 24);
        or_box_muller(unif(w[0], fp32), unif(low, fp32), g);
    } else {
        words(c->seed, j, t, ST_STEP2, 0, w);
        or_box_muller(unif(w[0], fp32), unif(w[1], fp32), g);
    }
    or_sv_theta(post, z_g, u_g, g[0], g[1], c->seed, j, t, fp32, theta);
    double xt = theta[0] + theta[1] * xp + sqrt(theta[2]) * z_x;
    sums[0] += 1.0;
    sums[1] += xp;
    sums[2] += xp * xp;
    sums[3] += xt;
    sums[4] += xp * xt;
    sums[5] += xt * xt;
    out[0] = xt;
    for (int f = 0; f < 6; ++f) out[f + 1] = sums[f];
    or_sv_posterior(c, sums, post);
    *rb = post[6] / (post[5] - 1.0);
}

/* Stochastic-volatility particle learning (not in the paper; Storvik-type
 * order: propagate, weight, resample, as in the bootstrap cycle).
 * Transition x_t = alpha + beta x_{t-1} + sigma Z, i.e. alpha = mu (1 - phi),
 * beta = phi; observation y_t ~ N(0, exp(x_t)).  The parameters
 * (alpha, beta, sigma^2) have the conjugate Normal / inverse-gamma prior
 * (alpha, beta) | sigma^2 ~ N(b0, sigma^2 Lambda0^{-1}), sigma^2 ~ IG(a0, d0).
 * Each particle keeps the raw sums of its own path that the regression of
 * x_s on (1, x_{s-1}) needs: n, S1 = sum x_{s-1}, S11 = sum x_{s-1}^2,
 * Sy = sum x_s, S1y = sum x_{s-1} x_s, Syy = sum x_s^2 (or_sv_posterior).
 * Step t: (x~, sums~) = resampled particle (identity at t = 1);
 *   theta ~ p(theta | sums~) (or_sv_theta);
 *   x_t = alpha + beta x~ + sigma z2;  sums += the new pair (x~, x_t);
 *   w_t proportional to N(y_t; 0, exp(x_t)).
 * Draws: init ST_INIT(j,0) words 0,1 -> Box-Muller, z1 -> x_0;
 *   step ST_STEP(j,t): word 0 -> resampling uniform; words 1,2 ->
 *   Box-Muller (z1 -> gamma normal, z2 -> x_t), word 3 -> gamma uniform;
 *   ST_STEP2(j,t): words 0,1 -> Box-Muller (z3, z4) for (alpha, beta);
 *   gamma retries g = 0.  With 24-bit uniforms and systematic resampling
 *   (ST_STEP word 0 unused) the (z3, z4) pair comes from ST_STEP word 0
 *   and the low bytes of words 1-3 instead (see sv_pl_slot).
 * Moments (weights w_t, before resampling): E x, Var x, E alpha, E beta,
 *   E sigma^2 of the draws that produced x_t, ESS, and the Rao-Blackwell
 *   mean d/(a-1) of sigma^2 after the update. */
static int run_sv_pl(const or_config* c, const double* y, int64_t T, double* loglik,
                     double* mom, int64_t* anc_out, double* state_out, double* logw_out,
                     const double* state0, int64_t t0, double y_prev, const int64_t* anc_first)
{
    const int64_t N = c->n;
    const int fp32 = c->fp32_words;
    const int F = 7;
    double* z = (double*)malloc(sizeof(double) * N * F);
    double* zn = (double*)malloc(sizeof(double) * N * F);
    double* th = (double*)malloc(sizeof(double) * N * 3);
    double* rb = (double*)malloc(sizeof(double) * N);
    double* lw = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    double* u = (double*)malloc(sizeof(double) * N);
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * N);
    uint32_t w[4];
    double g[2];
    int rc = 0;
    for (int64_t i = 0; i < N && !state0; ++i) {
        words(c->seed, (uint32_t)i, 0, ST_INIT, 0, w);
        or_box_muller(unif(w[0], fp32), unif(w[1], fp32), g);
        z[0 * N + i] = c->x0_mean + sqrt(c->x0_var) * g[0];
        for (int f = 1; f < F; ++f) z[f * N + i] = 0.0;
    }
    if (state0) {
        /* start from given particles z_{t0}; their weights are those of y_{t0} */
        memcpy(z, state0, sizeof(double) * N * F);
        if (t0 >= 1) {
            for (int64_t i = 0; i < N; ++i) lw[i] = log_normal_pdf(y_prev, 0.0, exp(z[i]));
            double M0, S0;
            or_cdf(lw, N, q, &M0, &S0);
        }
    }
    for (int64_t t = t0 + 1; t <= t0 + T; ++t) {
        const int64_t r = t - t0 - 1; /* output row */
        if (t == 1) {
            for (int64_t j = 0; j < N; ++j) a[j] = j;
        } else if (r == 0 && anc_first) {
            memcpy(a, anc_first, sizeof(int64_t) * N);
        } else {
            or_uniforms(c->scheme, c->seed, (uint32_t)t, N, u);
            or_resample(q, N, u, N, c->search, a);
        }
        for (int64_t j = 0; j < N; ++j) {
            double zk[7], out[7], theta[3];
            for (int f = 0; f < F; ++f) zk[f] = z[f * N + a[j]];
            sv_pl_slot(c, zk, (uint32_t)j, (uint32_t)t, out, theta, &rb[j]);
            for (int f = 0; f < F; ++f) zn[f * N + j] = out[f];
            th[0 * N + j] = theta[0]; th[1 * N + j] = theta[1]; th[2 * N + j] = theta[2];
        }
        memcpy(z, zn, sizeof(double) * N * F);
        for (int64_t i = 0; i < N; ++i) lw[i] = log_normal_pdf(y[r], 0.0, exp(z[i]));
        double M, S;
        or_cdf(lw, N, q, &M, &S);
        if (!(S > 0.0) || !isfinite(S) || !isfinite(M)) { rc = -1; }
        loglik[r] = M + log(S / (double)N);
        double sw = 0, swx = 0, swxx = 0, sww = 0, sa = 0, sb = 0, ss = 0, sr = 0;
        for (int64_t i = 0; i < N; ++i) {
            double wi = exp(lw[i] - M), xi = z[i];
            sw += wi; swx += wi * xi; swxx += wi * xi * xi; sww += wi * wi;
            sa += wi * th[i]; sb += wi * th[N + i]; ss += wi * th[2 * N + i];
            sr += wi * rb[i];
        }
        double* mo = mom + r * OR_NMOM;
        for (int k = 0; k < OR_NMOM; ++k) mo[k] = 0.0;
        mo[0] = swx / sw;
        mo[1] = swxx / sw - mo[0] * mo[0];
        mo[2] = sa / sw;
        mo[3] = sb / sw;
        mo[4] = ss / sw;
        mo[5] = sw * sw / sww;
        mo[6] = sr / sw;
        if (anc_out) for (int64_t j = 0; j < N; ++j) anc_out[r * N + j] = a[j];
        if (state_out) memcpy(state_out + r * N * F, z, sizeof(double) * N * F);
        if (logw_out) memcpy(logw_out + r * N, lw, sizeof(double) * N);
    }
    free(z); free(zn); free(th); free(rb); free(lw); free(q); free(u); free(a);
    return rc;
}

/* Run T steps from the prior (state0 = NULL, t0 = 0) or from given
 * particles `state0` (the model's fields, [f * N + i]) that are the state
 * after step t0; y[0..T-1] are then the observations of steps t0+1..t0+T and,
 * for the models that weight after propagating, y_prev is the observation
 * y_{t0} whose weights the first resampling uses.  Draws use the absolute
 * time index, so a run from the state after t0 steps continues the same
 * random streams. */
int or_run_given(const or_config* c, const double* state0, int64_t t0, double y_prev,
                 const double* y, int64_t T, const int64_t* anc_first, double* loglik,
                 double* mom, int64_t* anc_out, double* state_out, double* logw_out);

int or_run_from(const or_config* c, const double* state0, int64_t t0, double y_prev,
                const double* y, int64_t T, double* loglik, double* mom, int64_t* anc_out,
                double* state_out, double* logw_out)
{
    return or_run_given(c, state0, t0, y_prev, y, T, NULL, loglik, mom, anc_out, state_out,
                        logw_out);
}

/* As or_run_from, except that the first step's resampling is replaced by
 * the given ancestors anc_first[0..N) (0-based; NULL: resample as usual).
 * The rest of that step (propagation, statistics, weights, moments) and
 * every later step are computed as in or_run_from.  This lets a caller
 * hold another implementation's propagation and weighting to this one's
 * arithmetic on exactly the same resampled particles. */
int or_run_given(const or_config* c, const double* state0, int64_t t0, double y_prev,
                 const double* y, int64_t T, const int64_t* anc_first, double* loglik,
                 double* mom, int64_t* anc_out, double* state_out, double* logw_out)
{
    if (!c || c->n < 1 || T < 0 || t0 < 0 || (t0 > 0 && !state0)) return -2;
    if (anc_first)
        for (int64_t j = 0; j < c->n; ++j)
            if (anc_first[j] < 0 || anc_first[j] >= c->n) return -2;
    switch (c->model) {
    case OR_LL_PF: return run_ll_pf(c, y, T, loglik, mom, anc_out, state_out, logw_out, state0, t0, y_prev, anc_first);
    case OR_LL_PL: return run_ll_pl(c, y, T, loglik, mom, anc_out, state_out, logw_out, state0, t0, y_prev, anc_first);
    case OR_SV_PF: return run_sv_pf(c, y, T, loglik, mom, anc_out, state_out, logw_out, state0, t0, y_prev, anc_first);
    case OR_SV_PL: return run_sv_pl(c, y, T, loglik, mom, anc_out, state_out, logw_out, state0, t0, y_prev, anc_first);
    }
    return -2;
}

int or_run(const or_config* c, const double* y, int64_t T, double* loglik, double* mom,
           int64_t* anc_out, double* state_out, double* logw_out)
{
    return or_run_from(c, NULL, 0, 0.0, y, T, loglik, mom, anc_out, state_out, logw_out);
}

/* One step t = t0 + 1 from the particles state0 (the model's fields after
 * t0 steps, [f * N + i]), computed only for the output slots
 * slots[0..k): the resampling CDF over all N particles (weights of y_prev
 * for the models that weight after propagating, of the predictive
 * p(y_t | z) for local-level particle learning), each slot's uniform and
 * ancestor, and the slot's new fields, by the same per-slot arithmetic as
 * or_run_from.  anc_out[i] and state_out[f * k + i] for slot slots[i];
 * with t0 = 0 the models that weight after propagating keep every slot's
 * own particle.  Returns 0, -1 if the weights are degenerate, -2 for bad
 * arguments. */
int or_step_slots(const or_config* c, const double* state0, int64_t t0, double y_prev, double y,
                  const int64_t* slots, int64_t k, int64_t* anc_out, double* state_out)
{
    if (!c || c->n < 1 || !state0 || t0 < 0 || k < 0 || (k > 0 && (!slots || !anc_out || !state_out)))
        return -2;
    const int64_t N = c->n;
    const int F = or_fields(c->model);
    const uint32_t t = (uint32_t)(t0 + 1);
    for (int64_t i = 0; i < k; ++i)
        if (slots[i] < 0 || slots[i] >= N) return -2;
    int rc = 0;
    const int resample = c->model == OR_LL_PL || t0 >= 1;
    if (resample) {
        double* lw = (double*)malloc(sizeof(double) * N);
        double* q = (double*)malloc(sizeof(double) * N);
        double* u = (double*)malloc(sizeof(double) * (k > 0 ? k : 1));
        for (int64_t i = 0; i < N; ++i) {
            const double x = state0[i];
            switch (c->model) {
            case OR_LL_PF: lw[i] = log_normal_pdf(y_prev, x, c->sigma_v2); break;
            case OR_LL_PL: lw[i] = log_normal_pdf(y, x, state0[3 * N + i] + state0[4 * N + i]); break;
            default: lw[i] = log_normal_pdf(y_prev, 0.0, exp(x)); break;
            }
        }
        double M, S;
        or_cdf(lw, N, q, &M, &S);
        if (!(S > 0.0) || !isfinite(S) || !isfinite(M)) rc = -1;
        if (c->scheme == OR_SORTED_MULTINOMIAL) {
            double* all = (double*)malloc(sizeof(double) * N);
            or_uniforms(c->scheme, c->seed, t, N, all);
            for (int64_t i = 0; i < k; ++i) u[i] = all[slots[i]];
            free(all);
        } else {
            const double U = systematic_offset(c->scheme, c->seed, t);
            for (int64_t i = 0; i < k; ++i) u[i] = slot_uniform(c->scheme, c->seed, t, N, slots[i], U);
        }
        or_resample(q, N, u, k, c->search, anc_out);
        free(lw); free(q); free(u);
    } else {
        for (int64_t i = 0; i < k; ++i) anc_out[i] = slots[i];
    }
    for (int64_t i = 0; i < k; ++i) {
        double zk[7], out[7], theta[3], rb;
        for (int f = 0; f < F; ++f) zk[f] = state0[f * N + anc_out[i]];
        const uint32_t j = (uint32_t)slots[i];
        switch (c->model) {
        case OR_LL_PF: ll_pf_slot(c, zk, j, t, out); break;
        case OR_LL_PL: ll_pl_slot(c, zk, j, t, y, out); break;
        case OR_SV_PF: sv_pf_slot(c, zk, j, t, out); break;
        default: sv_pl_slot(c, zk, j, t, out, theta, &rb); break;
        }
        for (int f = 0; f < F; ++f) state_out[f * k + i] = out[f];
    }
    return rc;
}
