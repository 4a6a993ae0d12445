// Internal layout shared by the host runtime (pf_api.cpp) and the HIP
// kernels (pf_kernels.hip) of libpf_mi355x.so.  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace pf {

// Random-word streams: Philox4x32-10 with key = seed and counter
// (index, time, stream, attempt).  Which word feeds which draw is fixed per
// model in pf_models.hpp; a filter's draws therefore do not depend on the
// tiling, the launch shape or the search strategy.
enum Stream : uint32_t {
    kInit = 1, kStep = 2, kStep2 = 3, kSystematic = 4, kInit2 = 5, kGammaRetry = 16
};

enum Model : int32_t { kLLPF = 0, kLLPL = 1, kSVPF = 2, kSVPL = 3 };
enum Scheme : int32_t {
    kMultinomial = 0,
    kStratified = 1,
    kSystematicScheme = 2,
    kSortedMultinomial = 3
};
enum Strategy : int32_t { kAuto = 0, kBinary = 1, kCutpoint = 2, kMerge = 3 };

// How the per-tile sums become the CDF's tile prefixes.
enum Scan : int32_t {
    kScanTiles = 0,    // tiles store their sums; a one-work-group kernel scans them
    kScanLookback = 1  // single pass: decoupled look-back inside the cycle kernel
};

// Step-kernel phase flags.
enum StepFlags : int32_t {
    kResample = 1,   // draw ancestors from the previous step's CDF
    kPropagate = 2,  // move the particles (else they are only re-weighted)
    kWeight = 4,     // compute log-weights, the CDF and the normaliser
    kWeightedMoments = 8,  // moment partials weighted by this step's weights
    kFusedScan = 16        // the cycle's last work-group runs the tile scan
};

// Filters of at most this many tiles scan their tiles inside the cycle
// kernel (the work-group that finishes last), which saves the scan launch;
// for more tiles the work-groups' completion count, one atomic per
// work-group on a single word, costs more than the launch.
constexpr int32_t kFusedScanMax = 16;
// pf_debug_search_noalloc: largest CDF its static cut-point table holds, and
// where the table starts in the static scratch array (after the check flag).
constexpr int64_t kStaticCutMax = int64_t(1) << 20;
constexpr int64_t kStaticTableOffset = 64;

// Per-tile output of the CDF scan.  m_* are log-scale shifts, s_* sums of
// exp(l - m): the tile's exclusive prefix over all earlier tiles (m_ex, s_ex)
// and its own total (m_b, s_b).  The CDF value of element k of tile b is
//   q(k) = (s_ex e^{m_ex - M} + c[k] e^{m_b - M}) / S
// with (M, S) the whole step's shift and sum (Totals) and c[k] the in-tile
// inclusive prefix of exp(l - m_b).
struct TileInfo {
    double m_ex, s_ex, m_b, s_b;
};

struct Totals {
    double M, S;
};

// Normalised affine form of tile b's CDF values: q(k) = a + c[k] * b for k
// in tile b (written by the tile-scan kernel).
struct TileAB {
    double a, b;
};

// Device-resident scalars of one filter.
struct DevState {
    double loglik;       // running sum of M + log(S / N)
    uint32_t ticket;     // dynamic tile ticket of the running step (look-back)
    uint32_t flags;      // bit 0: a step's normaliser was zero or not finite
    double moments[8];   // output of the moment reduction
    uint32_t done;       // work-groups of the running cycle that have finished (fused scan)
    uint32_t pad32;
    double pad[5];
};

// bit 0: a step's normaliser was zero or not finite; bit 1: a fused tile
// scan gave up waiting for a tile's (max, sum)
enum StateFlags : uint32_t { kDegenerate = 1, kScanStall = 2 };

// Parameters of all four models (only the model's own ones are read).
struct ModelParams {
    double x0_mean, x0_var;
    double sigma_v2, sigma_w2;
    double a_v, b_v, a_w, b_w;
    double mu, phi, sigma2;
    double b0a, b0b, p0, p1, p2;
    double a_s, d_s;
};

// CDF samples per tile: the in-tile prefix at the end of each of kSegments
// equal segments, so a consumer can bracket a uniform to one segment with a
// single load (tile-scan form only).
constexpr int kSegments = 64;

// Moment-partial stride (doubles per tile): [m, sum e, sum e^2, g_0..g_5, pad].
constexpr int kPartialStride = 10;
// Look-back status words per tile: aggregate (m lo/hi, s lo/hi), inclusive
// (m lo/hi, s lo/hi); each 64-bit word carries the step's epoch in its upper
// half, so a word is valid only when its tag equals the running epoch.
constexpr int kStatusWords = 8;

struct StepArgs {
    int64_t n;
    int64_t pitch;       // elements between two record fields
    int32_t num_tiles;
    int32_t scheme;
    int32_t strategy;
    int32_t flags;       // StepFlags
    int32_t scan;        // Scan
    int32_t ts;          // particles per tile
    int32_t rsz;         // bytes per record element (4 or 8)
    int32_t test_stall;  // scan waits look for words no tile writes (a test aid)
    uint32_t t;          // time index of this step's draws (1-based)
    uint32_t epoch;      // tag of this launch's look-back words (never 0)
    uint64_t seed;
    double y_prop;       // observation the propagation conditions on
    double y_weight;     // observation the new weights score
    const void* rec_in;  // F arrays of `pitch` elements
    void* rec_out;
    const void* c_in;    // previous step's in-tile prefixes
    const void* samp_in; // previous step's segment samples of c (kSegments per tile)
    const TileInfo* tiles_in;   // look-back form of the previous CDF
    const TileAB* ab_in;        // tile-scan form of the previous CDF
    const int32_t* hint_in;     // source tile of CDF position b*TS/N, b = 0..tiles
    const Totals* tot_in;
    const TileAB* abE;          // sorted multinomial: this step's uniforms as
                                //   u = A_b + (in-tile spacing prefix) B_b
    void* c_out;
    void* samp_out;
    TileInfo* tiles_out;
    Totals* tot_out;
    double* agg_out;            // tile-scan: this step's (m_b, s_b) per tile
    double* chunk;              // chunked tile scan (above 4096 tiles): chunk
                                //   aggregates and prefixes, 3G + 1 doubles
    TileAB* ab_out;             // tile-scan outputs (the arrays ab_in / hint_in
    int32_t* hint_out;          //   point to, read by the next step)
    uint64_t* status;
    DevState* st;
    double* partials;
    int32_t* anc_out;    // ancestors of this step (NULL: not kept)
    const int32_t* cut_in;      // cut-point table I of the previous CDF (global
                                //   cut-point search; NULL otherwise)
    ModelParams p;
};

// Device-side progress of a batch of filters stepped together.
struct BatchState {
    uint64_t step;      // steps completed; selects the argument block of the next step
    uint64_t reserved;  // (unused; keeps the layout the host copies into)
    uint32_t done;      // scan work-groups finished in the running step
    uint32_t ring;      // argument blocks in the ring (steps that can be queued)
    int32_t n_filters;  // current members (argument blocks hold `capacity` entries)
    int32_t capacity;
    int64_t total_tiles;  // tiles of all current members
    uint64_t pad[3];
};

}  // namespace pf
