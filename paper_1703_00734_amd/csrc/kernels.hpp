// Device kernels of the BMF library and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace bmf {

// Arithmetic of a conditional-update launch.
enum Prec : int32_t {
    kP64 = 0,    // FP64 state, gathers and arithmetic
    kP32 = 1,    // FP32 state and gathers, FP32 arithmetic
    kPBF = 2,    // BF16 state and gathers, FP32 arithmetic, FP32 samples
    kPFB32 = 3,  // FP32 state, FP64 arithmetic (pivot fallback of kP32)
    kPFB16 = 4   // BF16 state, FP64 arithmetic (pivot fallback of kPBF)
};

// Capacity (compile-time K) used for a rank K: the register kernel handles
// K <= 16 with capacities {2,4,6,8,10,12,16}; the wave kernel 32 and 64.
int32_t capacity_for(int32_t K);
// Row stride (elements) of a factor array for capacity kc and element size.
int32_t stride_for(int32_t kc, int32_t elem_bytes);

struct UpdArgs {
    const Tile *tiles;        // register kernel: one tile per workgroup
    const int2 *items;        // wave kernel: (side, entity) items ...
    const int32_t *nitems_dev;// ... counted on the device (fallback queue), or
    int32_t nitems;           // ... counted on the host when nitems_dev is null
    const SideDesc *sides;
    const int32_t *ord;       // degree-sorted local ids (register kernel)
    const int64_t *ptr;
    const int32_t *idx;
    const void *val;          // double (kP64) or float
    const void *other;        // gathered factors (the other side's state)
    int32_t ks_other;
    void *self;               // updated factors (state precision)
    int32_t ks_self;
    void *sample;             // this sweep's sample slot (null when not kept), or with
                              // `ss` set: the sample store, slot taken from ss
    int32_t ks_sample;
    const SweepState *ss;     // when set, t and the sample slot come from here
    int32_t K;
    int32_t prow;             // doubles per moment-matched row
    int32_t pfrow;            // floats per prior-factor row (SideDesc::pfac)
    uint32_t t;               // sweep index (Philox c1)
    uint32_t k0, k1;          // Philox key
    float theta;              // FP32 pivot threshold (0 in FP64)
    int32_t *fb_count;        // FP64 fallback queue (null: count as non-PD)
    int2 *fb_list;
    int32_t *fb_total;        // running count of rows sent to the fallback
    int32_t *nonpd;           // FP64 Cholesky failures
    double *sse_col;          // column pass: per column 4 slots of its SSE (null: skip)
    const double *colsq;      // column pass: per column the sum of its squared values
    const int2 *splits;       // per item (first partial slot, count); count 0: not split
    const float *gpart;       // partial Grams + right-hand sides (KP*KP + KP floats each)
    const int32_t *gstart;    // prior groups: group g holds items [gstart[g], gstart[g+1])
    int32_t ngroups;
};

// Partial Grams of heavy-entity segments (BF16 state, MFMA).
struct GramPartArgs {
    const SegItem *segs;
    int32_t nseg;
    const SideDesc *sides;
    const int32_t *idx;
    const void *val;
    const void *other;
    int32_t ks_other;
    float *gpart;
};

// Residual sums of squares per column: SSE_d = sum_n (r_nd - x_n^T w_d)^2
// over the column's observed entries, squares summed in FP64, written to 4
// slots per column (one per wave of a group; unused slots zero).
struct SseArgs {
    const Tile *tiles;        // CSC column tiles
    const SideDesc *sides;    // column sides (self = W, other = X)
    const int32_t *ord;
    const int64_t *ptr;
    const int32_t *idx;
    const void *val;
    const void *X;            // row factors (state precision)
    const void *W;            // column factors (state precision)
    int32_t ks;
    int32_t K;
    double *sse_col;
};

struct StatsArgs {
    const StatsJob *jobs;
    const SideDesc *sides;
    const void *X;            // row factors (sides < nrow_sides)
    const void *W;            // column factors (sides >= nrow_sides)
    int32_t nrow_sides;
    int32_t ks;
    int32_t K;
    double *part;             // njobs x (K + K(K+1)/2)
};

// Fixed-order sum of `count` partial vectors of `width` doubles.
struct ReduceJob {
    const double *src;
    double *dst;
    int32_t count;
    int32_t width;
};

struct HyperArgs {
    const HyperJob *jobs;     // part_begin: slot of the final sums / final SSE
    const double *part;       // NW final sums, per side
    const double *sse_part;   // final SSE, per stage block
    const double *mu0;        // K
    const double *W0inv;      // K x K
    double beta0, nu0, a0, b0;
    int32_t K;
    uint32_t t, k0, k1;
    const SweepState *ss;     // when set, t comes from here
    int32_t *nonpd;
    // when set, the last block to finish advances the sweep state (as k_advance)
    SweepState *advance;
    int32_t *fb_counts;       // the fallback queue counters it resets
    int32_t *done;            // completion counter of the launch (zero between launches)
    // Normal-Wishart noise of job j at noise + j * K(K+3)/2: drawn by the
    // preceding reduction launch when noise_ready, else by this launch
    double *noise;
    int32_t noise_ready;
};

// Noise draws of the Normal-Wishart jobs that a reduction launch makes in
// extra blocks (one per job), for the hyperparameter launch after it.
struct NoiseArgs {
    const HyperJob *jobs;
    int32_t njobs;            // hyper jobs; kinds 0 and 1 get noise
    int32_t K;
    double nu0;
    uint32_t t, k0, k1;
    const SweepState *ss;     // when set, t comes from here
    double *noise;
};

struct InitArgs {
    const int2 *items;        // (side, entity)
    int32_t nitems;
    const SideDesc *sides;
    void *self;
    int32_t ks_self;
    int32_t K, prow;
    uint32_t k0, k1;
};

struct MmArgs {
    const int2 *items;        // (side, entity)
    int32_t nitems;
    const SideDesc *sides;    // sample_off per side
    const void *sample;       // slot 0 of the sample store
    int64_t slot_elems;       // elements per slot
    int32_t ks;
    int32_t S;                // kept samples
    int32_t K, prow;
    double *const *out;       // per side: moment-matched rows
    int32_t *ridged;
    // a subset of the samples per entity (dominant mode, mixture components),
    // or every sample when `labels` is null: sample q of item it is taken
    // when which[it * kMaxComp + comp] is -1 or equals its cluster label
    // (labels[side] + entity * maxS + q); -2 means no component (no output)
    const uint8_t *const *labels;
    const int8_t *which;
    int32_t comp, maxS;
    double *const *aux;       // per side: (pi, log det Lambda) pairs of entity 0, or null
};

// Per-column noise precisions: the row pass's scaled copies (sqrt(tau_d) w_d
// into Wt, sqrt(tau_d) r_nd into vt, in the state / value precision) and the
// per-column Gamma draws, for the blocks of a stage (grid y = job).
struct TauColArgs {
    const TauColJob *jobs;
    int32_t njobs;
    double *tau;              // per column (W-array order)
    const void *W;            // state rows (stride ks)
    void *Wt;
    int32_t ks, K;
    const void *val;          // CSR values
    void *vt;
    const int32_t *idx;       // CSR local column ids
    const int64_t *cptr;      // CSC pointers (global entry offsets)
    const double *sse_col;    // per column 4 partial sums of its residual SSE
    double a0, b0;
    const SweepState *ss;     // sweep index from here when set, else t
    uint32_t t, k0, k1;
};

// Components kept per row by the mixture approximation, at most.
constexpr int kMaxComp = 4;
// lambda-means: clusters per row, rounds, kept samples per row, at most.
constexpr int kLmCmax = 16;
constexpr int kLmMaxit = 32;
constexpr int kLmMaxS = 256;

// lambda-means clustering of each item's kept samples and the choice of its
// components: the largest cluster (ncomp = 1, dominant mode) or the ncomp
// largest with at least two members (mixture), as cluster ids in which[]
// (-1: every sample, -2: none) and size weights in the aux planes.
struct LmeansArgs {
    const int2 *items;        // (side, entity)
    int32_t nitems;
    const SideDesc *sides;
    const void *sample;
    int64_t slot_elems;
    int32_t ks, S, K;
    double lam_scale;
    int32_t ncomp;
    uint8_t *const *labels;   // per side: entity 0's labels (maxS per entity)
    int32_t maxS;
    int8_t *which;            // per item, kMaxComp
    double *const *aux;       // per side: plane 0 (pi, log det) of entity 0
    int64_t aux_plane;        // doubles between component planes
};

// Pooled moments of each item's mixture (eq. marginal_mixture) into its
// moment-matched row.
struct GmmPoolArgs {
    const int2 *items;
    int32_t nitems;
    const int8_t *which;      // per item, kMaxComp
    const double *const *comp;// per side: plane 0 row of entity 0
    const double *const *aux; // per side: plane 0 (pi, log det) of entity 0
    int64_t plane, aux_plane; // doubles between component planes
    double *const *out;       // per side: moment-matched rows
    int32_t K, prow, ncomp;
};

// A side whose prior is a propagated mixture: each sweep every row takes the
// component of largest responsibility at its current value, copied into the
// side's own prior rows (which the update kernels read).
struct GmmSide {
    const double *src;        // plane 0 row of entity 0 of the source block
    const double *aux;        // plane 0 (pi, log det) of entity 0 of the source
    double *dst;              // this side's prior rows (entity 0)
    const void *state;        // this side's state rows (entity 0)
    int32_t n;
    int32_t pad_;
};

struct GmmPickArgs {
    const int2 *items;        // (gmm side, entity)
    int32_t nitems;
    const GmmSide *gsides;
    int64_t plane, aux_plane;
    int32_t ks_state, K, prow, ncomp;
    int32_t force0;           // 1: the largest component (stage begin)
};

// Prior factors of moment-matched rows: for each (side, entity) item the row
// out[side] + entity * prow is factored into pfout[side] + entity * pfrow.
struct PfacArgs {
    const int2 *items;
    int32_t nitems;
    double *const *out;       // per side: moment-matched rows (as MmArgs::out)
    float *const *pfout;      // per side: prior-factor rows, null for none
    int32_t K, prow, pfrow;
};

struct AggArgs {
    const AggJob *jobs;
    const int2 *items;        // (job, row)
    int32_t nitems;
    int32_t K, prow;
    double *out;              // aggregated means, K per slot
    int32_t *corrections;
};

struct PredictArgs {
    const int64_t *xslot;
    const int64_t *wslot;
    int64_t n;
    const double *mux;
    const double *muw;
    int32_t K;
    double ybar;
    float *out;
};

// Predictions for pairs given by original ids: the ids are mapped to slots on
// the device through the position arrays (original id -> position).
struct PredictIdsArgs {
    const int32_t *row;
    const int32_t *col;
    int64_t n;
    const int64_t *row_pos;
    const int64_t *col_pos;
    const double *mux;
    const double *muw;
    int32_t K;
    double ybar;
    float *out;
};

// File-scope device scratch of the allocation-free entry point
// (bmf_predict_noalloc): its pairs' ids and outputs are staged there.
constexpr int64_t kNoallocMaxPairs = (int64_t)1 << 20;
constexpr int64_t kScratchBytes = kNoallocMaxPairs * (4 + 4 + 4);
// Device address of the scratch array on the current device: looked up with
// hipGetSymbolAddress on the first call per device and kept.
hipError_t scratch_address(void **p);

hipError_t launch_update_reg(int32_t kc, int32_t prec, const UpdArgs &a, int32_t ntiles,
                             hipStream_t s);
// Two entities with at most 16 entries per wavefront, 16 < K <= 32, FP32 or
// BF16 state (items in pairs: grid counts pairs).
hipError_t launch_update_duo(int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s, bool mf);
// The copies of propagated rows in the sibling blocks of a stage that have at
// most lowrank_max_nnz() entries, one prior group (copies sharing one stored
// prior factor) per wavefront; a.items holds the copies grouped, sorted within
// a group by entry count (0, 1 .. lowrank_small_nnz(), more).
hipError_t launch_update_group(int32_t kp, int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s);
int32_t lowrank_max_nnz();
int32_t lowrank_small_nnz();
// vgram: BF16 state with K > 16 takes the VALU-Gram kernel instead of the MFMA one
hipError_t launch_update_wave(int32_t kp, int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s,
                              bool vgram = false);
hipError_t launch_sse(int32_t kc, int32_t prec, const SseArgs &a, int32_t ntiles, hipStream_t s);
hipError_t launch_gram_part(int32_t kp, const GramPartArgs &a, hipStream_t s);
hipError_t launch_stats(int32_t prec, const StatsArgs &a, int32_t njobs, hipStream_t s);
// max_width: the largest width among the jobs (blocks cover at most 256
// outputs of a job each).
hipError_t launch_reduce(const ReduceJob *jobs, int32_t njobs, int32_t max_width, hipStream_t s,
                         const NoiseArgs *noise = nullptr);
hipError_t launch_hyper(const HyperArgs &a, int32_t njobs, hipStream_t s);
hipError_t launch_init(int32_t prec, const InitArgs &a, hipStream_t s);
hipError_t launch_mm(int32_t prec, const MmArgs &a, hipStream_t s);
hipError_t launch_lmeans(int32_t prec, const LmeansArgs &a, hipStream_t s);
hipError_t launch_tau_scale(int32_t prec, const TauColArgs &a, hipStream_t s);
hipError_t launch_tau_cols(const TauColArgs &a, hipStream_t s);
hipError_t launch_gmm_pool(const GmmPoolArgs &a, hipStream_t s);
hipError_t launch_gmm_pick(int32_t prec, const GmmPickArgs &a, hipStream_t s);
hipError_t launch_pfac(int32_t kp, const PfacArgs &a, hipStream_t s);
hipError_t launch_agg(const AggArgs &a, hipStream_t s);
hipError_t launch_predict(const PredictArgs &a, hipStream_t s);
hipError_t launch_predict_ids(const PredictIdsArgs &a, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_advance(SweepState *ss, int32_t *fb_counts, hipStream_t s);

}  // namespace bmf
