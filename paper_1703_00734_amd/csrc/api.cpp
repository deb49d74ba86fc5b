// C ABI of the BMF library: context, device layout, stage logic and launches.
//
// The host side validates the problem, centres the values, builds the integer
// plan (ordering, partition, CSR/CSC), the degree-sorted schedules and the
// per-stage work lists, and drives the kernels on one HIP stream.  Every step
// of the sweep runs on the device; the host only enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "bmf.h"
#include "common.hpp"
#include "kernels.hpp"
#include "planner.hpp"

using namespace bmf;

namespace {

constexpr int32_t kStatsRowsPerJob = 512;   // entities per NW statistics job (about)
constexpr int32_t kStatsJobsMax = 256;      // jobs per side at most
constexpr int64_t kPredictChunk = 1 << 20;  // prediction pairs per launch
constexpr int32_t kFallbackGrid = 128;      // workgroups of the FP64 redo pass
constexpr int64_t kLightNnz = 16;           // light entities: VALU-Gram or two-per-wavefront kernels
constexpr int64_t kSegNnz = 2048;           // MFMA path: entities with more entries are split
constexpr int32_t kWaveGridCap = 1 << 20;
constexpr int64_t kMfDuoMin = 32768;            // heavy entities of a stage side for the MFMA duo kernel

enum Counter { kFbRow = 0, kFbCol = 1, kFbTotal = 2, kNonPD = 3, kRidged = 4, kCorr = 5, kHyperDone = 6,
               kNumCounters = 16 };

// Kernel classes for the optional per-launch timing.
enum KClass { kKRows = 0, kKCols, kKGram, kKFallback, kKSse, kKStats, kKReduce, kKHyper, kKInit, kKMM, kKAgg, kKPredict, kKFill, kKPick, kNumK };
const char *kKNames[kNumK] = {"update_rows", "update_cols", "gram_segments", "update_fallback_fp64", "sse", "nw_stats", "reduce",
                              "hyper_draws", "init", "moment_match", "aggregate", "predict", "bookkeeping",
                              "mixture_pick"};

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout;
int64_t kHyPacked(const Layout &L);

// Sizes of everything the device holds, computable from the configuration.
struct Layout {
    int32_t K = 0, kc = 0, prec = 0, ks_m = 0, ks_p = 0, prow = 0, hy = 0, npair = 0, pfrow = 0;
    int64_t nb = 0, E_r = 0, E_c = 0, Emax = 0, Pmax = 0;
    int64_t vs = 0, ss = 0, sp = 0;  // value / state / sample element bytes
    // byte offsets
    int64_t csr_ptr, csr_idx, csr_val, csc_ptr, csc_idx, csc_val, csr_ent, csc_ent, ord, X, W, hyper, tau, mu0,
        W0inv, mm, agg_x, agg_w, sample, probe, sse_col, colsq, sse_final, stats_part, stats_final,
        counters, sweep, fb_list, m_sides, m_tiles, m_reduce, gpart, m_segs, m_splits, nw_noise,
        m_items, m_items2, m_stats, m_hyper, m_mmout, pfac, m_pfout, m_agg_jobs, m_agg_items, p_xslot, p_wslot,
        p_out, rowpos, colpos, m_gitems, m_gstart, lab, which, aux, gmm, m_labptr, m_auxptr, m_gmmout, m_gsides,
        m_pitems, tau_col, Wt, vt, one, m_taujobs, total;
    int32_t ncomp = 1;        // components per row of the propagated fit (mixture: ncomp, else 1)
    int64_t n_tiles_cap, n_items_cap, n_stats_cap, n_sse_cap, n_seg_cap;
    bool mfma = false;
};

// Offset (doubles) of the packed prior row inside a hyperparameter slot.
int64_t kHyPacked(const Layout &L) { return (int64_t)L.K * L.K + 2 * L.K; }

// Components kept per row: the mixture's ncomp (0 => 3), one otherwise.
int32_t ncomp_of(const bmf_config &c) { return c.approx == BMF_APPROX_GMM ? (c.ncomp ? c.ncomp : 3) : 1; }

bool layout_for(const bmf_config &c, Layout &L, std::string &err) {
    L = Layout();
    L.K = c.K;
    L.kc = capacity_for(c.K);
    L.prec = c.precision;
    const bool fp64 = c.precision == BMF_PREC_FP64;
    L.vs = fp64 ? 8 : 4;
    L.ss = fp64 ? 8 : (c.precision == BMF_PREC_BF16 ? 2 : 4);
    L.sp = fp64 ? 8 : 4;
    L.ks_m = stride_for(L.kc, (int32_t)L.ss);
    L.ks_p = stride_for(L.kc, (int32_t)L.sp);
    L.prow = c.K * (c.K + 1) / 2 + 2 * c.K;
    L.hy = c.K * c.K + 2 * c.K + L.prow;   // [Lambda, mu, Lambda mu, packed row]
    L.npair = c.K + c.K * (c.K + 1) / 2;
    L.nb = (int64_t)c.I * c.J;
    L.E_r = (int64_t)c.J * c.N;
    L.E_c = (int64_t)c.I * c.D;
    const int64_t bs_r = (c.N + c.I - 1) / c.I, bs_c = (c.D + c.J - 1) / c.J;
    std::vector<int64_t> R(c.I), C(c.J);
    for (int32_t i = 0; i < c.I; ++i) R[i] = std::min(bs_r, c.N - i * bs_r);
    for (int32_t j = 0; j < c.J; ++j) C[j] = std::min(bs_c, c.D - j * bs_c);
    if (R.back() <= 0 || C.back() <= 0) {
        err = "partition leaves an empty part";
        return false;
    }
    int64_t er[4] = {0, 0, 0, 0}, ec[4] = {0, 0, 0, 0};
    for (int32_t i = 0; i < c.I; ++i)
        for (int32_t j = 0; j < c.J; ++j) {
            const int s = stage_of(i, j);
            er[s] += R[i];
            ec[s] += C[j];
        }
    for (int s = 1; s <= 3; ++s) {
        L.Emax = std::max(L.Emax, er[s] + ec[s]);
        L.Pmax = std::max(L.Pmax, std::max(er[s], ec[s]));
    }
    L.n_tiles_cap = 2 * L.Emax + 8;
    L.n_items_cap = 2 * L.Emax + 8;
    L.n_stats_cap = kStatsJobsMax * 2 * L.nb + 8;
    L.n_sse_cap = L.Emax + 8;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off = align_up(off + std::max<int64_t>(bytes, 1), 256);
        return o;
    };
    const int64_t nnz = c.nnz;
    L.csr_ptr = take(8 * (L.E_r + L.nb));
    L.csr_idx = take(4 * nnz);
    L.csr_val = take(L.vs * nnz);
    L.csc_ptr = take(8 * (L.E_c + L.nb));
    L.csc_idx = take(4 * nnz);
    L.csc_val = take(L.vs * nnz);
    // COO entry of every CSR / CSC position (device planner: the host keeps none)
    L.csr_ent = take(c.plan_on_host ? 0 : 4 * nnz);
    L.csc_ent = take(c.plan_on_host ? 0 : 4 * nnz);
    L.ord = take(4 * (L.E_r + L.E_c));
    L.X = take(L.ss * L.E_r * L.ks_m);
    L.W = take(L.ss * L.E_c * L.ks_m);
    L.hyper = take(8 * L.nb * 2 * L.hy);
    L.tau = take(8 * L.nb);
    L.mu0 = take(8 * c.K);
    L.W0inv = take(8 * c.K * c.K);
    L.mm = take(8 * (L.E_r + L.E_c) * L.prow);
    // prior factors of the moment-matched rows that seed later stages (the rows
    // of blocks (i, 0) and the columns of blocks (0, j): N + D rows), for the
    // empty-entity path of FP32/BF16 passes on the wavefront kernels
    // (not under a mixture prior: a row's prior changes from sweep to sweep)
    if (!fp64 && L.kc >= 32 && L.nb > 1 && c.approx != BMF_APPROX_GMM)
        L.pfrow = (int32_t)align_up(c.K * (c.K + 1) / 2 + 1, 4);
    L.pfac = take(4 * ((int64_t)c.N + c.D) * L.pfrow);
    L.agg_x = take(8 * c.N * c.K);
    L.agg_w = take(8 * c.D * c.K);
    L.sample = take(L.sp * (int64_t)c.max_kept * L.Emax * L.ks_p);
    L.probe = take(L.sp * L.Emax * L.ks_p);
    L.sse_col = take(8 * 4 * L.E_c);
    L.colsq = take(8 * L.E_c);
    L.sse_final = take(8 * L.nb);
    L.nw_noise = take(8 * 3 * L.nb * (c.K * (c.K + 3) / 2));
    L.stats_part = take(8 * L.n_stats_cap * L.npair);
    L.stats_final = take(8 * 2 * L.nb * L.npair);
    L.counters = take(4 * kNumCounters);
    L.sweep = take(sizeof(SweepState));
    L.fb_list = take(8 * (L.Pmax + 8));
    L.m_sides = take(sizeof(SideDesc) * 2 * L.nb);
    L.m_tiles = take(sizeof(Tile) * L.n_tiles_cap);
    L.m_reduce = take(sizeof(ReduceJob) * (3 * L.nb + 8));
    // heavy-entity segments of the MFMA path: at most 2 nnz / kSegNnz per pass
    L.mfma = c.precision == BMF_PREC_BF16 && L.kc >= 32;
    L.n_seg_cap = L.mfma ? 2 * (c.nnz / kSegNnz) + 8 : 0;
    L.gpart = take(4 * L.n_seg_cap * (L.kc * L.kc + L.kc));
    L.m_segs = take(sizeof(SegItem) * 2 * L.n_seg_cap);
    L.m_splits = take(sizeof(int2) * L.n_items_cap);
    L.m_items = take(sizeof(int2) * L.n_items_cap);
    L.m_items2 = take(sizeof(int2) * (L.Emax + 8));
    L.m_stats = take(sizeof(StatsJob) * L.n_stats_cap);
    L.m_hyper = take(sizeof(HyperJob) * 3 * L.nb);
    L.m_mmout = take(sizeof(double *) * 2 * L.nb);
    L.m_pfout = take(sizeof(float *) * 2 * L.nb);
    L.m_agg_jobs = take(sizeof(AggJob) * (c.I + c.J));
    L.m_agg_items = take(sizeof(int2) * (c.N + c.D));
    L.p_xslot = take(8 * kPredictChunk);
    L.p_wslot = take(8 * kPredictChunk);
    L.p_out = take(4 * kPredictChunk);
    L.m_gitems = take(sizeof(int2) * L.n_items_cap);
    L.m_gstart = take(4 * (L.n_items_cap + 8));
    L.rowpos = take(8 * c.N);
    L.colpos = take(8 * c.D);
    // dominant mode / mixture: cluster labels of every row's kept samples, the
    // chosen clusters of the stage's items, per component plane the (weight,
    // log det) pairs and (mixture) the component rows, plus the per-side
    // pointer tables and the mixture-prior pick lists
    {
        const bool clus = c.approx != BMF_APPROX_MM;
        const int64_t Etot = L.E_r + L.E_c;
        L.ncomp = ncomp_of(c);
        L.lab = take(clus ? Etot * c.max_kept : 0);
        L.which = take(clus ? (L.Emax + 8) * kMaxComp : 0);
        L.aux = take(clus ? 8 * 2 * (int64_t)L.ncomp * Etot : 0);
        L.gmm = take(c.approx == BMF_APPROX_GMM ? 8 * (int64_t)L.ncomp * Etot * L.prow : 0);
        L.m_labptr = take(sizeof(void *) * 2 * L.nb);
        L.m_auxptr = take(sizeof(void *) * kMaxComp * 2 * L.nb);
        L.m_gmmout = take(sizeof(void *) * kMaxComp * 2 * L.nb);
        L.m_gsides = take(sizeof(GmmSide) * 2 * L.nb);
        L.m_pitems = take(c.approx == BMF_APPROX_GMM ? sizeof(int2) * (L.Emax + 8) : 0);
    }
    // per-column noise precisions: tau_d of every block column, the row pass's
    // scaled copies of W and of the CSR values, and a constant 1 (the row
    // pass's tau then)
    {
        const bool tc = c.tau_per_column != 0;
        L.tau_col = take(tc ? 8 * L.E_c : 0);
        L.Wt = take(tc ? L.ss * L.E_c * L.ks_m : 0);
        L.vt = take(tc ? L.vs * nnz : 0);
        L.one = take(8);
        L.m_taujobs = take(sizeof(TauColJob) * L.nb);
    }
    L.total = off;
    return true;
}

// Work lists of one stage (host copies of what is uploaded).
struct StageLists {
    std::vector<int32_t> blocks;                    // global block ids in the stage
    std::vector<SideDesc> sides;                    // rows of blocks[k] at k, columns at nbs + k
    // register kernel tiles: [rows grouped by block | rows heavy-first | cols grouped | cols heavy]
    std::vector<Tile> tiles;
    int64_t t_row_blk = 0, t_row_heavy = 0, t_col_blk = 0, t_col_heavy = 0, t_end = 0;
    std::vector<int64_t> row_tile_begin, col_tile_begin;   // per block k, within the grouped lists
    // wave kernel items, same four lists
    std::vector<int2> items;
    int64_t i_row_blk = 0, i_row_heavy = 0, i_col_blk = 0, i_col_heavy = 0, i_end = 0;
    // first item of the heavy-first order with at most kLightNnz entries, and
    // the same per block (block item lists are in decreasing degree order)
    int64_t i_row_light = 0, i_col_light = 0;
    std::vector<int64_t> row_item_light, col_item_light;
    // first item of the heavy-first order (and per block) under a per-row prior
    // with a factor and at most lowrank_max_nnz() entries (these sort after every
    // other item, by decreasing degree; the prior-group kernel takes them)
    int64_t i_row_lowrank = 0, i_col_lowrank = 0;
    std::vector<int64_t> row_item_lowrank, col_item_lowrank;
    // per side: prior-factor rows this stage's moment matching writes (or null)
    std::vector<float *> pfout;
    std::vector<int64_t> row_item_begin, col_item_begin;
    std::vector<int2> ents;                         // every (side, entity) of the stage
    // MFMA path: segments of heavy entities ([rows grouped | cols grouped]) and,
    // parallel to `items`, each item's (first partial slot, segment count)
    std::vector<SegItem> segs;
    std::vector<int2> splits;
    // prior groups (k_update_group): the copies with at most lowrank_max_nnz()
    // entries under a factored per-row prior, grouped by the prior row they
    // share; gstart[g] is group g's first copy in gitems (one more entry ends
    // the last group).  Per block (groups of one copy) and batched (one group
    // per propagated entity across the stage's sibling blocks), per pass.
    std::vector<int2> gitems;
    std::vector<int32_t> gstart;
    std::vector<int64_t> g_row_blk, g_col_blk;      // per stage block: first group (size nbs + 1)
    int64_t g_row_b0 = 0, g_row_b1 = 0, g_col_b0 = 0, g_col_b1 = 0;
    int64_t s_row = 0, s_col = 0, s_end = 0;
    std::vector<int64_t> row_seg_begin, col_seg_begin;   // per stage block, within the pass
    std::vector<std::vector<int32_t>> ord_row, ord_col;   // degree orders per stage block
    int32_t lane_row = 32, lane_col = 32;          // entries per lane of the register kernel
    std::vector<StatsJob> stats;
    std::vector<int64_t> side_stats_begin;          // per side, into stats (size 2*nbs + 1)
    std::vector<HyperJob> hyper;
    std::vector<int32_t> hyper_begin;               // per block k: first hyper job; size nbs + 1
    std::vector<int32_t> hyper_kind;                // kind of each job
    std::vector<int64_t> sse_tile_begin;            // SSE tiles per block (== row tiles grouped)
    int64_t row_ents = 0, col_ents = 0;
    int64_t row_updates = 0, ratings = 0;
    // per-column noise precisions: one job per block
    std::vector<TauColJob> taujobs;
    // mixture priors: the propagated sides and their (side, entity) pick items
    std::vector<GmmSide> gsides;
    std::vector<int2> pitems;
};

}  // namespace

struct bmf_ctx {
    bmf_config cfg{};
    std::string err;
    bool device = false;
    hipStream_t stream = nullptr;      // the caller's stream: all work is ordered on it
    hipStream_t ls = nullptr;          // where launches go (the capture stream while capturing)
    hipStream_t cap_stream = nullptr;  // internal stream used only to capture the sweep graph
    hipGraphExec_t gexec = nullptr;    // one captured sweep of the active stage
    Layout L;
    Plan plan;
    double ybar = 0.0;
    std::vector<double> mu0, W0inv;
    // host offsets per block
    std::vector<int64_t> csr_ptr_off, csc_ptr_off, x_off, w_off, ord_row_off, ord_col_off;
    std::vector<int64_t> nz_off[2];       // first CSR (0) / CSC (1) entry of each block
    // device memory
    char *base = nullptr;
    bool own = false;
    // stage state
    int32_t stage = 0;          // active stage, 0 = none
    int32_t finalized = 0;      // highest stage whose moment matching is done
    int64_t t = 0;              // sweeps run in the active stage
    int32_t kept = 0;
    bool agg_valid = false;
    StageLists S;
    int32_t done_stages[4] = {0, 0, 0, 0};
    // device address of the allocation-free entry point's scratch array on the
    // context's device (looked up once per device at bmf_init)
    char *scratch = nullptr;
    // progress callback (checked before each sweep is enqueued)
    bmf_progress_fn progress = nullptr;
    void *progress_user = nullptr;
    // fingerprint of the training data and settings (checkpoint files)
    uint64_t fingerprint = 0;
    // timing
    bool timing = false;
    struct Pending { int32_t k; hipEvent_t a, b; };
    std::vector<Pending> pending;
    int64_t tlaunch[kNumK] = {0};
    double tms[kNumK] = {0};

    template <typename T> T *dev(int64_t off) { return reinterpret_cast<T *>(base + off); }
    bool bf() const { return cfg.precision == BMF_PREC_BF16; }
    bool fp64() const { return cfg.precision == BMF_PREC_FP64; }
    int32_t prec() const { return cfg.precision == BMF_PREC_FP64 ? kP64 : (bf() ? kPBF : kP32); }
    // register kernel for K <= 16 (FP64: K <= 12), wavefront kernels above
    bool reg() const { return L.kc <= (cfg.precision == BMF_PREC_FP64 ? 12 : 16); }
};

namespace {

bmf_status fail(bmf_ctx *c, bmf_status s, const std::string &m) {
    if (c) c->err = m;
    return s;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(ctx, BMF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

// Timed launch wrapper: records events around the launch when timing is on.
template <typename F>
bmf_status timed(bmf_ctx *c, int32_t k, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        HIPCHK(c, hipEventCreate(&a));
        HIPCHK(c, hipEventCreate(&b));
        HIPCHK(c, hipEventRecord(a, c->stream));
    }
    const hipError_t e = launch();
    if (e != hipSuccess) return fail(c, BMF_EDEVICE, std::string(kKNames[k]) + ": " + hipGetErrorString(e));
    if (c->timing) {
        HIPCHK(c, hipEventRecord(b, c->stream));
        c->pending.push_back({k, a, b});
    }
    return BMF_OK;
}

bool spd_cholesky(int K, const double *A, std::vector<double> &L) {
    L.assign((size_t)K * K, 0.0);
    for (int i = 0; i < K; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * K + j];
            for (int p = 0; p < j; ++p) s -= L[i * K + p] * L[j * K + p];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * K + i] = std::sqrt(s);
            } else {
                L[i * K + j] = s / L[j * K + j];
            }
        }
    return true;
}

// 64-bit fingerprint of the training data and of every setting that the
// chain's values depend on (checkpoint files are only loaded into a context
// with the same one).  Word-wise multiply-xorshift mixing of the raw bytes.
struct Mix64 {
    uint64_t h = 0x9E3779B97F4A7C15ull;
    void word(uint64_t v) {
        h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
    }
    void bytes(const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        size_t i = 0;
        for (; i + 8 <= n; i += 8) {
            uint64_t v;
            std::memcpy(&v, b + i, 8);
            word(v);
        }
        uint64_t t = 0;
        for (size_t k = 0; i + k < n; ++k) t |= (uint64_t)b[i + k] << (8 * k);
        word(t ^ ((uint64_t)n << 56));
    }
    template <typename T> void val(const T &v) { bytes(&v, sizeof(T)); }
};

uint64_t data_fingerprint(const bmf_config &c) {
    Mix64 m;
    m.val(c.N); m.val(c.D); m.val(c.K); m.val(c.nnz); m.val(c.I); m.val(c.J); m.val(c.order);
    m.val(c.beta0); m.val(c.nu0); m.val(c.sample_tau); m.val(c.tau_a0); m.val(c.tau_b0); m.val(c.tau_fixed);
    m.val(c.seed); m.val(c.burnin); m.val(c.thin); m.val(c.max_kept); m.val(c.precision); m.val(c.pivot_theta);
    m.val(c.approx); m.val(c.lambda_scale); m.val(ncomp_of(c)); m.val(c.tau_per_column);
    if (c.mu0) m.bytes(c.mu0, 8 * (size_t)c.K);
    if (c.W0) m.bytes(c.W0, 8 * (size_t)c.K * c.K);
    if (c.nnz > 0) {
        m.bytes(c.row, 4 * (size_t)c.nnz);
        m.bytes(c.col, 4 * (size_t)c.nnz);
        m.bytes(c.val, 4 * (size_t)c.nnz);
    }
    return m.h;
}

bmf_status validate(const bmf_config *cfg, std::string &err) {
    if (!cfg) { err = "null config"; return BMF_EINVAL; }
    const bmf_config &c = *cfg;
    if (c.N <= 0 || c.D <= 0) { err = "N and D must be positive"; return BMF_EINVAL; }
    if (c.N > (int64_t)INT32_MAX || c.D > (int64_t)INT32_MAX) { err = "N, D must fit int32"; return BMF_EUNSUPPORTED; }
    if (c.K < 1) { err = "K must be >= 1"; return BMF_EINVAL; }
    if (c.K > 64) { err = "K > 64 is not supported"; return BMF_EUNSUPPORTED; }
    if (c.nnz < 0 || (c.nnz > 0 && (!c.row || !c.col || !c.val))) { err = "bad COO arrays"; return BMF_EINVAL; }
    if (c.nnz > (int64_t)INT32_MAX) { err = "nnz must fit int32"; return BMF_EUNSUPPORTED; }
    if (c.I < 1 || c.J < 1 || c.I > c.N || c.J > c.D) { err = "bad partition"; return BMF_EINVAL; }
    if (c.I > 65 || c.J > 65) { err = "at most 65 parts per dimension"; return BMF_EUNSUPPORTED; }
    if (c.order < BMF_ORDER_GIVEN || c.order > BMF_ORDER_DECREASING) { err = "bad order"; return BMF_EINVAL; }
    if (!(c.beta0 > 0.0)) { err = "beta0 must be > 0"; return BMF_EINVAL; }
    if (!(c.nu0 > c.K - 1)) { err = "nu0 must be > K - 1"; return BMF_EINVAL; }
    if (c.sample_tau) {
        if (!(c.tau_a0 > 0.0) || !(c.tau_b0 > 0.0)) { err = "tau prior must be positive"; return BMF_EINVAL; }
    } else if (!(c.tau_fixed > 0.0) || !std::isfinite(c.tau_fixed)) {
        err = "tau_fixed must be positive";
        return BMF_EINVAL;
    }
    if (c.burnin < 0 || c.thin < 1 || c.max_kept < 1) { err = "bad burnin/thin/max_kept"; return BMF_EINVAL; }
    if (c.precision < BMF_PREC_FP64 || c.precision > BMF_PREC_BF16) { err = "bad precision"; return BMF_EINVAL; }
    if (c.pivot_theta < 0.0 || c.pivot_theta >= 1.0) { err = "pivot_theta must be in [0, 1)"; return BMF_EINVAL; }
    if (c.lane_nnz < 0) { err = "lane_nnz must be >= 0"; return BMF_EINVAL; }
    if (c.approx < BMF_APPROX_MM || c.approx > BMF_APPROX_GMM) { err = "bad approx"; return BMF_EINVAL; }
    if (!(c.lambda_scale >= 0.0) || !std::isfinite(c.lambda_scale)) { err = "lambda_scale must be >= 0"; return BMF_EINVAL; }
    if (c.ncomp < 0 || c.ncomp > kMaxComp) { err = "ncomp must be in 0..4"; return BMF_EINVAL; }
    if (c.tau_per_column && c.precision == BMF_PREC_BF16) {
        err = "per-column noise precisions need FP32 or FP64 precision";
        return BMF_EUNSUPPORTED;
    }
    if (c.approx != BMF_APPROX_MM && c.K > 32) { err = "dominant-mode and mixture fits need K <= 32"; return BMF_EUNSUPPORTED; }
    if (c.approx != BMF_APPROX_MM && c.max_kept > kLmMaxS) {
        err = "dominant-mode and mixture fits keep at most 256 samples per stage";
        return BMF_EUNSUPPORTED;
    }
    {
        // the gather kernels address a gathered row by a 32-bit byte offset from
        // its block's first row: the largest part times the row stride must fit
        const int64_t ebytes = c.precision == BMF_PREC_FP64 ? 8 : (c.precision == BMF_PREC_BF16 ? 2 : 4);
        const int64_t rowb = (int64_t)stride_for(capacity_for(c.K), (int32_t)ebytes) * ebytes;
        const int64_t part = std::max((c.N + c.I - 1) / c.I, (c.D + c.J - 1) / c.J);
        if (part * rowb >= ((int64_t)1 << 32)) {
            err = "a part of " + std::to_string(part) + " rows at " + std::to_string(rowb) +
                  " bytes per factor row exceeds the 32-bit gather offsets";
            return BMF_EUNSUPPORTED;
        }
    }
    for (int64_t e = 0; e < c.nnz; ++e)
        if (!std::isfinite(c.val[e])) { err = "non-finite value at entry " + std::to_string(e); return BMF_EINVAL; }
    if (c.W0) {
        std::vector<double> L;
        if (!spd_cholesky(c.K, c.W0, L)) { err = "W0 is not SPD"; return BMF_EINVAL; }
    }
    if (c.mu0)
        for (int k = 0; k < c.K; ++k)
            if (!std::isfinite(c.mu0[k])) { err = "mu0 not finite"; return BMF_EINVAL; }
    return BMF_OK;
}

// ---------------------------------------------------------------------------
// schedules
// ---------------------------------------------------------------------------
// Lanes per entity for the register kernel: about `per` entries per lane, a
// power of two in [1, 256] (groups above 64 lanes span several waves).  `per`
// is chosen per pass by the autotuner.
int32_t lanes_for(int64_t deg, int32_t per) {
    int32_t G = 1;
    while (G < 256 && (int64_t)G * per < deg) G <<= 1;
    return G;
}

void side_tiles(int32_t side, int64_t ord_off, const std::vector<int64_t> &ptr, const std::vector<int32_t> &ord,
                int32_t per, std::vector<Tile> &out, std::vector<int64_t> &cost) {
    const int64_t n = (int64_t)ord.size();
    int64_t k = 0;
    while (k < n) {
        const int64_t deg = ptr[ord[k] + 1] - ptr[ord[k]];
        const int32_t G = lanes_for(deg, per);
        const int32_t cap = 256 / G;
        int32_t cnt = 0;
        int64_t cst = 0;
        while (k + cnt < n && cnt < cap) {
            const int64_t d = ptr[ord[k + cnt] + 1] - ptr[ord[k + cnt]];
            if (lanes_for(d, per) != G) break;
            cst += d + 16;
            ++cnt;
        }
        out.push_back(Tile{side, (int32_t)(ord_off + k), cnt, G});
        cost.push_back(cst);
        k += cnt;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// stage construction
// ---------------------------------------------------------------------------
static void build_stage_lists(bmf_ctx *c, int32_t s) {
    StageLists &S = c->S;
    S = StageLists();
    const Plan &P = c->plan;
    const int32_t J = P.J;
    for (int32_t b = 0; b < (int32_t)P.blocks.size(); ++b)
        if (P.blocks[b].stage == s) S.blocks.push_back(b);
    const int32_t nbs = (int32_t)S.blocks.size();
    const Layout &L = c->L;
    double *hyper = c->dev<double>(L.hyper);
    double *mm = c->dev<double>(L.mm);
    double *tau = c->dev<double>(L.tau);
    S.sides.resize(2 * nbs);
    S.pfout.assign(2 * nbs, nullptr);
    // prior-factor row of the first row of row block i (columns: N + first
    // column of column block j)
    float *pf = L.pfrow ? c->dev<float>(L.pfac) : nullptr;
    std::vector<int64_t> pfx(P.I + 1, 0), pfw(P.J + 1, 0);
    for (const PlanBlock &B : P.blocks) {
        if (B.j == 0) pfx[B.i + 1] = B.R;
        if (B.i == 0) pfw[B.j + 1] = B.C;
    }
    for (int32_t i = 0; i < P.I; ++i) pfx[i + 1] += pfx[i];
    pfw[0] = c->cfg.N;
    for (int32_t j = 0; j < P.J; ++j) pfw[j + 1] += pfw[j];
    int64_t soff = 0;
    for (int32_t k = 0; k < nbs; ++k) {
        const int32_t b = S.blocks[k];
        const PlanBlock &B = P.blocks[b];
        const bool xp = B.j > 0, wp = B.i > 0;
        SideDesc r{}, q{};
        r.ptr_off = c->csr_ptr_off[b];
        r.self_off = c->x_off[b];
        r.other_off = c->w_off[b];
        r.sample_off = soff;
        soff += B.R;
        r.prior = xp ? mm + c->x_off[B.i * J + 0] * L.prow : hyper + ((int64_t)b * 2 + 0) * L.hy + kHyPacked(L);
        r.tau = c->cfg.tau_per_column ? c->dev<double>(L.one) : tau + b;
        r.tau_stride = 0;
        r.pfac = xp && pf ? pf + pfx[B.i] * L.pfrow : nullptr;
        r.n = (int32_t)B.R;
        r.per_row = xp;
        r.c2 = counter_word(b, kRow);
        r.c2_init = counter_word(b, kInitX);
        r.block = b;
        q.ptr_off = c->csc_ptr_off[b];
        q.self_off = c->w_off[b];
        q.other_off = c->x_off[b];
        q.sample_off = soff;
        soff += B.C;
        q.prior = wp ? mm + (L.E_r + c->w_off[0 * J + B.j]) * L.prow : hyper + ((int64_t)b * 2 + 1) * L.hy + kHyPacked(L);
        q.tau = c->cfg.tau_per_column ? c->dev<double>(L.tau_col) + c->w_off[b] : tau + b;
        q.tau_stride = c->cfg.tau_per_column ? 1 : 0;
        if (c->cfg.tau_per_column)
            S.taujobs.push_back(TauColJob{b, (int32_t)B.C, c->w_off[b], c->csc_ptr_off[b], c->nz_off[0][b], B.M});
        q.pfac = wp && pf ? pf + pfw[B.j] * L.pfrow : nullptr;
        q.n = (int32_t)B.C;
        q.per_row = wp;
        q.c2 = counter_word(b, kCol);
        q.c2_init = counter_word(b, kInitW);
        q.block = b;
        if (c->cfg.approx == BMF_APPROX_GMM) {
            // a mixture prior: each sweep picks a component per row into the
            // side's own rows, which the update kernels read
            double *gm = c->dev<double>(L.gmm);
            double *ax = c->dev<double>(L.aux);
            char *Xb = c->base + L.X, *Wb = c->base + L.W;
            if (xp) {
                const int64_t src = c->x_off[B.i * J + 0];
                r.prior = mm + c->x_off[b] * L.prow;
                GmmSide g{gm + src * L.prow, ax + src * 2, const_cast<double *>(r.prior),
                          Xb + c->x_off[b] * L.ks_m * L.ss, (int32_t)B.R, 0};
                for (int32_t e = 0; e < (int32_t)B.R; ++e) S.pitems.push_back(make_int2((int32_t)S.gsides.size(), e));
                S.gsides.push_back(g);
            }
            if (wp) {
                const int64_t src = L.E_r + c->w_off[0 * J + B.j];
                q.prior = mm + (L.E_r + c->w_off[b]) * L.prow;
                GmmSide g{gm + src * L.prow, ax + src * 2, const_cast<double *>(q.prior),
                          Wb + c->w_off[b] * L.ks_m * L.ss, (int32_t)B.C, 0};
                for (int32_t e = 0; e < (int32_t)B.C; ++e) S.pitems.push_back(make_int2((int32_t)S.gsides.size(), e));
                S.gsides.push_back(g);
            }
        }
        S.sides[k] = r;
        S.sides[nbs + k] = q;
        if (pf && s < 3 && B.j == 0) S.pfout[k] = pf + pfx[B.i] * L.pfrow;
        if (pf && s < 3 && B.i == 0) S.pfout[nbs + k] = pf + pfw[B.j] * L.pfrow;
        S.row_updates += B.R + B.C;
        S.ratings += B.M;
        S.row_ents += B.R;
        S.col_ents += B.C;
    }
    // degree orders of each side (host copies, same as uploaded at init)
    for (int32_t k = 0; k < nbs; ++k) {
        const PlanBlock &B = P.blocks[S.blocks[k]];
        S.ord_row.push_back(degree_order(B.csr_ptr));
        S.ord_col.push_back(degree_order(B.csc_ptr));
    }
    // wave kernel items: grouped by block, then heavy-first across blocks; on
    // the MFMA path entities above kSegNnz entries are split into segments
    const bool mf = c->L.mfma;
    for (int pass = 0; pass < 2; ++pass) {
        const bool rows = pass == 0;
        std::vector<int2> igrp, sgrp;
        std::vector<int64_t> ideg;
        std::vector<char> ifast;                    // few entries under a factored per-row prior
        const int64_t nlr = lowrank_max_nnz(), nls = lowrank_small_nnz();
        std::vector<int64_t> &ibeg = rows ? S.row_item_begin : S.col_item_begin;
        std::vector<int64_t> &sbeg = rows ? S.row_seg_begin : S.col_seg_begin;
        (rows ? S.s_row : S.s_col) = (int64_t)S.segs.size();
        int32_t slot = 0;
        for (int32_t k = 0; k < nbs; ++k) {
            const int32_t b = S.blocks[k];
            const PlanBlock &B = P.blocks[b];
            const std::vector<int64_t> &ptr = rows ? B.csr_ptr : B.csc_ptr;
            const int32_t side = rows ? k : nbs + k;
            ibeg.push_back((int64_t)igrp.size());
            sbeg.push_back((int64_t)slot);
            std::vector<int64_t> &blight = rows ? S.row_item_light : S.col_item_light;
            std::vector<int64_t> &blowr = rows ? S.row_item_lowrank : S.col_item_lowrank;
            blight.push_back(-1);
            blowr.push_back(-1);
            const bool fast = S.sides[side].pfac != nullptr;
            for (int32_t e : (rows ? S.ord_row[k] : S.ord_col[k])) {
                const int64_t deg = ptr[e + 1] - ptr[e];
                if (blight.back() < 0 && deg <= kLightNnz) blight.back() = (int64_t)igrp.size();
                if (fast && blowr.back() < 0 && deg <= nlr) blowr.back() = (int64_t)igrp.size();
                igrp.push_back(make_int2(side, e));
                ideg.push_back(deg);
                ifast.push_back(fast && deg <= nlr);
                if (mf && deg > kSegNnz) {
                    const int32_t nseg = (int32_t)((deg + kSegNnz - 1) / kSegNnz);
                    sgrp.push_back(make_int2(slot, nseg));
                    // global entry offsets of this entity: the uploaded pointer array
                    // holds block-local offsets shifted by the block's first entry
                    const int64_t g0 = c->nz_off[pass][b] + ptr[e];
                    for (int32_t q = 0; q < nseg; ++q) {
                        SegItem si{};
                        si.side = side;
                        si.ent = e;
                        si.begin = g0 + (int64_t)q * kSegNnz;
                        si.end = std::min(g0 + deg, si.begin + kSegNnz);
                        si.slot = slot++;
                        S.segs.push_back(si);
                    }
                } else {
                    sgrp.push_back(make_int2(0, 0));
                }
            }
        }
        ibeg.push_back((int64_t)igrp.size());
        sbeg.push_back((int64_t)slot);
        {
            std::vector<int64_t> &blight = rows ? S.row_item_light : S.col_item_light;
            std::vector<int64_t> &blowr = rows ? S.row_item_lowrank : S.col_item_lowrank;
            for (int32_t k = 0; k < nbs; ++k) {
                if (blight[k] < 0) blight[k] = ibeg[k + 1];
                if (blowr[k] < 0) blowr[k] = ibeg[k + 1];
            }
        }
        // heavy-first: decreasing degree, the low-rank and empty-entity kernels'
        // items after all others
        std::vector<int64_t> iperm(igrp.size());
        for (size_t q = 0; q < iperm.size(); ++q) iperm[q] = (int64_t)q;
        std::stable_sort(iperm.begin(), iperm.end(), [&](int64_t a2, int64_t b2) {
            if (ifast[a2] != ifast[b2]) return ifast[a2] < ifast[b2];
            return ideg[a2] > ideg[b2];
        });
        (rows ? S.i_row_blk : S.i_col_blk) = (int64_t)S.items.size();
        S.items.insert(S.items.end(), igrp.begin(), igrp.end());
        S.splits.insert(S.splits.end(), sgrp.begin(), sgrp.end());
        (rows ? S.i_row_heavy : S.i_col_heavy) = (int64_t)S.items.size();
        int64_t &light = rows ? S.i_row_light : S.i_col_light;
        int64_t &lowr = rows ? S.i_row_lowrank : S.i_col_lowrank;
        light = -1;
        lowr = -1;
        for (int64_t q : iperm) {
            if (light < 0 && ideg[q] <= kLightNnz) light = (int64_t)S.items.size();
            if (lowr < 0 && ifast[q]) lowr = (int64_t)S.items.size();
            S.items.push_back(igrp[q]);
            S.splits.push_back(sgrp[q]);
        }
        if (light < 0) light = (int64_t)S.items.size();
        if (lowr < 0) lowr = (int64_t)S.items.size();
        // prior groups of this pass: per block, one copy each (the tail of
        // the block's decreasing-degree list); batched, the copies of one
        // propagated entity n of source part p (row part i for X rows, column
        // part j for W columns) across the sibling blocks, ordered by entry
        // count kind (none, one or two, more) and then by block
        {
            std::vector<int64_t> &gblk = rows ? S.g_row_blk : S.g_col_blk;
            const std::vector<int64_t> &blowr = rows ? S.row_item_lowrank : S.col_item_lowrank;
            struct FastCopy {
                int32_t part, n, kind, k;
                int2 item;
            };
            std::vector<FastCopy> fc;
            for (int32_t k = 0; k < nbs; ++k) {
                const PlanBlock &B = P.blocks[S.blocks[k]];
                gblk.push_back((int64_t)S.gstart.size());
                for (int64_t q = blowr[k]; q < ibeg[k + 1]; ++q) {
                    S.gstart.push_back((int32_t)S.gitems.size());
                    S.gitems.push_back(igrp[q]);
                    const int64_t d = ideg[q];
                    fc.push_back(FastCopy{rows ? B.i : B.j, igrp[q].y, d == 0 ? 0 : (d <= nls ? 1 : 2), k, igrp[q]});
                }
            }
            gblk.push_back((int64_t)S.gstart.size());
            std::stable_sort(fc.begin(), fc.end(), [](const FastCopy &x, const FastCopy &y) {
                if (x.part != y.part) return x.part < y.part;
                if (x.n != y.n) return x.n < y.n;
                if (x.kind != y.kind) return x.kind < y.kind;
                return x.k < y.k;
            });
            (rows ? S.g_row_b0 : S.g_col_b0) = (int64_t)S.gstart.size();
            // a group holds at most one wavefront's lanes of copies (the kernel
            // counts their kinds with one ballot); a longer run is split, each
            // piece still sorted by kind
            int32_t in_group = 0;
            for (size_t q = 0; q < fc.size(); ++q) {
                if (q == 0 || fc[q].part != fc[q - 1].part || fc[q].n != fc[q - 1].n || in_group == 64) {
                    S.gstart.push_back((int32_t)S.gitems.size());
                    in_group = 0;
                }
                S.gitems.push_back(fc[q].item);
                ++in_group;
            }
            (rows ? S.g_row_b1 : S.g_col_b1) = (int64_t)S.gstart.size();
        }
    }
    S.gstart.push_back((int32_t)S.gitems.size());
    S.s_end = (int64_t)S.segs.size();
    S.i_end = (int64_t)S.items.size();
    // every entity, for init and moment matching
    for (int32_t side = 0; side < 2 * nbs; ++side)
        for (int32_t e = 0; e < S.sides[side].n; ++e) S.ents.push_back(make_int2(side, e));
    // NW statistics jobs (non-propagated sides only): contiguous entity ranges
    S.side_stats_begin.assign(2 * nbs + 1, 0);
    for (int32_t side = 0; side < 2 * nbs; ++side) {
        S.side_stats_begin[side] = (int64_t)S.stats.size();
        if (S.sides[side].per_row) continue;
        const int32_t n = S.sides[side].n;
        const int32_t nj = std::max(1, std::min(kStatsJobsMax, (n + kStatsRowsPerJob - 1) / kStatsRowsPerJob));
        const int32_t chunk = (n + nj - 1) / nj;
        for (int32_t f = 0; f < n; f += chunk) {
            StatsJob j{side, f, std::min(chunk, n - f), (int32_t)S.stats.size()};
            S.stats.push_back(j);
        }
    }
    S.side_stats_begin[2 * nbs] = (int64_t)S.stats.size();
    // hyperparameter jobs, grouped by block
    for (int32_t k = 0; k < nbs; ++k) {
        const int32_t b = S.blocks[k];
        const PlanBlock &B = P.blocks[b];
        S.hyper_begin.push_back((int32_t)S.hyper.size());
        if (!S.sides[k].per_row) {
            HyperJob h{0, b, k, k + 1, B.R, hyper + ((int64_t)b * 2 + 0) * L.hy};
            S.hyper.push_back(h);
            S.hyper_kind.push_back(0);
        }
        if (!S.sides[nbs + k].per_row) {
            HyperJob h{1, b, nbs + k, nbs + k + 1, B.C, hyper + ((int64_t)b * 2 + 1) * L.hy};
            S.hyper.push_back(h);
            S.hyper_kind.push_back(1);
        }
        if (c->cfg.sample_tau && !c->cfg.tau_per_column) {
            HyperJob h{2, b, k, k + 1, B.M, tau + b};
            S.hyper.push_back(h);
            S.hyper_kind.push_back(2);
        }
    }
    S.hyper_begin.push_back((int32_t)S.hyper.size());
}

// Register-kernel tiles of the active stage for `per_row`/`per_col` entries
// per lane: grouped by block (per-block launches, SSE) and heavy-first
// (batched launches).
static void build_tiles(bmf_ctx *c, int32_t per_row, int32_t per_col) {
    StageLists &S = c->S;
    const Plan &P = c->plan;
    const int32_t nbs = (int32_t)S.blocks.size();
    S.tiles.clear();
    S.row_tile_begin.clear();
    S.col_tile_begin.clear();
    S.lane_row = per_row;
    S.lane_col = per_col;
    for (int pass = 0; pass < 2; ++pass) {
        const bool rows = pass == 0;
        std::vector<Tile> grouped;
        std::vector<int64_t> gcost;
        std::vector<int64_t> &tbeg = rows ? S.row_tile_begin : S.col_tile_begin;
        for (int32_t k = 0; k < nbs; ++k) {
            const int32_t b = S.blocks[k];
            const PlanBlock &B = P.blocks[b];
            const int64_t ooff = rows ? c->ord_row_off[b] : c->ord_col_off[b];
            tbeg.push_back((int64_t)grouped.size());
            side_tiles(rows ? k : nbs + k, ooff, rows ? B.csr_ptr : B.csc_ptr, rows ? S.ord_row[k] : S.ord_col[k],
                       rows ? per_row : per_col, grouped, gcost);
        }
        tbeg.push_back((int64_t)grouped.size());
        std::vector<int64_t> perm(grouped.size());
        for (size_t q = 0; q < perm.size(); ++q) perm[q] = (int64_t)q;
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a2, int64_t b2) { return gcost[a2] > gcost[b2]; });
        (rows ? S.t_row_blk : S.t_col_blk) = (int64_t)S.tiles.size();
        S.tiles.insert(S.tiles.end(), grouped.begin(), grouped.end());
        (rows ? S.t_row_heavy : S.t_col_heavy) = (int64_t)S.tiles.size();
        for (int64_t q : perm) S.tiles.push_back(grouped[q]);
    }
    S.t_end = (int64_t)S.tiles.size();
    S.sse_tile_begin = S.row_tile_begin;
}

static bmf_status upload(bmf_ctx *c, int64_t off, const void *src, size_t bytes) {
    if (bytes == 0) return BMF_OK;
    HIPCHK(c, hipMemcpyAsync(c->base + off, src, bytes, hipMemcpyHostToDevice, c->stream));
    return BMF_OK;
}

static bmf_status upload_tiles(bmf_ctx *c) {
    const Layout &L = c->L;
    StageLists &S = c->S;
    bmf_status st;
    if ((int64_t)S.tiles.size() > L.n_tiles_cap) return fail(c, BMF_ENOMEM, "tile list exceeds its reserved space");
    if ((st = upload(c, L.m_tiles, S.tiles.data(), S.tiles.size() * sizeof(Tile)))) return st;
    // fixed-order reductions: SSE of stage block k at k, NW sums of side q at nbs + q
    const int32_t nbs = (int32_t)S.blocks.size();
    std::vector<ReduceJob> rj;
    for (int32_t k = 0; k < nbs; ++k) {
        const int32_t b = S.blocks[k];
        rj.push_back(ReduceJob{c->dev<double>(L.sse_col) + 4 * c->w_off[b], c->dev<double>(L.sse_final) + k,
                               (int32_t)(4 * c->plan.blocks[b].C), 1});
    }
    for (int32_t q = 0; q < 2 * nbs; ++q)
        rj.push_back(ReduceJob{c->dev<double>(L.stats_part) + S.side_stats_begin[q] * L.npair,
                               c->dev<double>(L.stats_final) + (int64_t)q * L.npair,
                               (int32_t)(S.side_stats_begin[q + 1] - S.side_stats_begin[q]), L.npair});
    if ((st = upload(c, L.m_reduce, rj.data(), rj.size() * sizeof(ReduceJob)))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BMF_OK;
}

static bmf_status upload_stage(bmf_ctx *c) {
    const Layout &L = c->L;
    StageLists &S = c->S;
    bmf_status st;
    if ((int64_t)S.items.size() > L.n_items_cap ||
        (int64_t)S.ents.size() > L.Emax + 8 || (int64_t)S.stats.size() > L.n_stats_cap)
        return fail(c, BMF_ENOMEM, "stage work lists exceed their reserved space");
    if ((st = upload(c, L.m_sides, S.sides.data(), S.sides.size() * sizeof(SideDesc)))) return st;
    if ((st = upload(c, L.m_items, S.items.data(), S.items.size() * sizeof(int2)))) return st;
    if ((int64_t)S.segs.size() > 2 * L.n_seg_cap) return fail(c, BMF_ENOMEM, "segment list exceeds its reserved space");
    if ((st = upload(c, L.m_splits, S.splits.data(), S.splits.size() * sizeof(int2)))) return st;
    if ((st = upload(c, L.m_segs, S.segs.data(), S.segs.size() * sizeof(SegItem)))) return st;
    if ((st = upload(c, L.m_items2, S.ents.data(), S.ents.size() * sizeof(int2)))) return st;
    if ((int64_t)S.gitems.size() > L.n_items_cap || (int64_t)S.gstart.size() > L.n_items_cap + 8)
        return fail(c, BMF_ENOMEM, "prior group lists exceed their reserved space");
    if ((st = upload(c, L.m_gitems, S.gitems.data(), S.gitems.size() * sizeof(int2)))) return st;
    if ((st = upload(c, L.m_gstart, S.gstart.data(), S.gstart.size() * 4))) return st;
    if ((st = upload(c, L.m_stats, S.stats.data(), S.stats.size() * sizeof(StatsJob)))) return st;
    if ((st = upload(c, L.m_hyper, S.hyper.data(), S.hyper.size() * sizeof(HyperJob)))) return st;
    std::vector<double *> outs(S.sides.size());
    const int32_t nbs = (int32_t)S.blocks.size();
    for (int32_t k = 0; k < nbs; ++k) {
        const int32_t b = S.blocks[k];
        outs[k] = c->dev<double>(L.mm) + c->x_off[b] * L.prow;
        outs[nbs + k] = c->dev<double>(L.mm) + (L.E_r + c->w_off[b]) * L.prow;
    }
    if ((st = upload(c, L.m_mmout, outs.data(), outs.size() * sizeof(double *)))) return st;
    if ((st = upload(c, L.m_taujobs, S.taujobs.data(), S.taujobs.size() * sizeof(TauColJob)))) return st;
    if (c->cfg.approx != BMF_APPROX_MM) {
        const int64_t Etot = L.E_r + L.E_c;
        std::vector<uint8_t *> labp(2 * nbs);
        std::vector<double *> auxp(kMaxComp * 2 * nbs, nullptr), gmp(kMaxComp * 2 * nbs, nullptr);
        for (int32_t k = 0; k < nbs; ++k) {
            const int32_t b = S.blocks[k];
            const int64_t e[2] = {c->x_off[b], L.E_r + c->w_off[b]};
            for (int sd = 0; sd < 2; ++sd) {
                const int32_t i = sd * nbs + k;
                labp[i] = c->dev<uint8_t>(L.lab) + e[sd] * c->cfg.max_kept;
                for (int32_t cc = 0; cc < L.ncomp; ++cc) {
                    auxp[cc * 2 * nbs + i] = c->dev<double>(L.aux) + (cc * Etot + e[sd]) * 2;
                    if (c->cfg.approx == BMF_APPROX_GMM)
                        gmp[cc * 2 * nbs + i] = c->dev<double>(L.gmm) + (cc * Etot + e[sd]) * L.prow;
                }
            }
        }
        if ((st = upload(c, L.m_labptr, labp.data(), labp.size() * sizeof(void *)))) return st;
        if ((st = upload(c, L.m_auxptr, auxp.data(), auxp.size() * sizeof(void *)))) return st;
        if ((st = upload(c, L.m_gmmout, gmp.data(), gmp.size() * sizeof(void *)))) return st;
        if ((int64_t)S.pitems.size() > L.Emax + 8) return fail(c, BMF_ENOMEM, "mixture pick list exceeds its space");
        if ((st = upload(c, L.m_gsides, S.gsides.data(), S.gsides.size() * sizeof(GmmSide)))) return st;
        if ((st = upload(c, L.m_pitems, S.pitems.data(), S.pitems.size() * sizeof(int2)))) return st;
        HIPCHK(c, hipStreamSynchronize(c->stream));     // the host tables above are released next
    }
    if ((st = upload(c, L.m_pfout, S.pfout.data(), S.pfout.size() * sizeof(float *)))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BMF_OK;
}

// ---------------------------------------------------------------------------
// kernel drivers
// ---------------------------------------------------------------------------
// Update-pass arguments.  With use_ss the sweep index and the sample slot
// are read on the device from the sweep state (sweeps, graph-capturable);
// otherwise t and sample are taken as given (single steps).
static UpdArgs upd_args(bmf_ctx *c, bool rows, uint32_t t, void *sample, bool use_ss) {
    const Layout &L = c->L;
    UpdArgs a{};
    a.sides = c->dev<SideDesc>(L.m_sides);
    a.ord = c->dev<int32_t>(L.ord);
    a.ptr = c->dev<int64_t>(rows ? L.csr_ptr : L.csc_ptr);
    a.idx = c->dev<int32_t>(rows ? L.csr_idx : L.csc_idx);
    a.val = c->dev<void>(rows ? L.csr_val : L.csc_val);
    a.other = c->dev<void>(rows ? L.W : L.X);
    if (rows && c->cfg.tau_per_column) {
        // the row pass reads sqrt(tau_d) w_d and sqrt(tau_d) r_nd (tau = 1)
        a.val = c->dev<void>(L.vt);
        a.other = c->dev<void>(L.Wt);
    }
    a.ks_other = L.ks_m;
    a.self = c->dev<void>(rows ? L.X : L.W);
    a.ks_self = L.ks_m;
    a.sample = use_ss ? (void *)(c->base + L.sample) : sample;
    a.ss = use_ss ? c->dev<SweepState>(L.sweep) : nullptr;
    a.ks_sample = L.ks_p;
    a.K = c->cfg.K;
    a.prow = L.prow;
    a.pfrow = L.pfrow;
    a.t = t;
    a.k0 = (uint32_t)(c->cfg.seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(c->cfg.seed >> 32);
    int32_t *cnt = c->dev<int32_t>(L.counters);
    a.nonpd = cnt + kNonPD;
    a.fb_total = cnt + kFbTotal;
    if (!c->fp64()) {
        a.theta = (float)(c->cfg.pivot_theta > 0.0 ? c->cfg.pivot_theta : std::ldexp(1.0, -10));
        a.fb_count = cnt + (rows ? kFbRow : kFbCol);
        a.fb_list = c->dev<int2>(L.fb_list);
    }
    return a;
}

// One conditional-update pass over the rows (or columns) of the active stage;
// block k = -1 means every block, else only stage block k.
static bmf_status run_pass(bmf_ctx *c, bool rows, uint32_t t, void *sample, int32_t k, bool use_ss,
                           bool sse = false) {
    const Layout &L = c->L;
    StageLists &S = c->S;
    const int32_t nbs = (int32_t)S.blocks.size();
    UpdArgs a = upd_args(c, rows, t, sample, use_ss);
    if (sse && !rows) {
        a.sse_col = c->dev<double>(L.sse_col);
        a.colsq = c->dev<double>(L.colsq);
    }
    bmf_status st;
    const int32_t kcls = rows ? kKRows : kKCols;
    // the fallback queue counters start every pass at zero: sweeps reset them in
    // the sweep-state advance, single steps around their pass
    if (!c->fp64() && !use_ss) {
        int32_t *fb = a.fb_count;
        if ((st = timed(c, kKFill, [&] { return launch_fill_i32(fb, 0, 1, c->ls); }))) return st;
    }
    // which blocks: one launch for all (batched, heavy-first) or one per block
    std::vector<std::pair<int64_t, int64_t>> ranges;   // tile or item ranges
    const bool batched = c->cfg.batched && k < 0;
    if (c->reg()) {
        if (batched) {
            ranges.push_back(rows ? std::make_pair(S.t_row_heavy, S.t_col_blk) : std::make_pair(S.t_col_heavy, S.t_end));
        } else {
            const std::vector<int64_t> &tb = rows ? S.row_tile_begin : S.col_tile_begin;
            const int64_t base = rows ? S.t_row_blk : S.t_col_blk;
            for (int32_t q = 0; q < nbs; ++q)
                if (k < 0 || q == k) ranges.push_back({base + tb[q], base + tb[q + 1]});
        }
        for (auto &r : ranges) {
            UpdArgs b = a;
            b.tiles = c->dev<Tile>(L.m_tiles) + r.first;
            const int32_t n = (int32_t)(r.second - r.first);
            if ((st = timed(c, kcls, [&] { return launch_update_reg(L.kc, c->prec(), b, n, c->ls); }))) return st;
        }
    } else {
        if (batched) {
            ranges.push_back(rows ? std::make_pair(S.i_row_heavy, S.i_col_blk) : std::make_pair(S.i_col_heavy, S.i_end));
        } else {
            const std::vector<int64_t> &ib = rows ? S.row_item_begin : S.col_item_begin;
            const int64_t base = rows ? S.i_row_blk : S.i_col_blk;
            for (int32_t q = 0; q < nbs; ++q)
                if (k < 0 || q == k) ranges.push_back({base + ib[q], base + ib[q + 1]});
        }
        // segments of heavy entities (MFMA path): partial Grams first
        if (L.mfma) {
            const int64_t sbase = rows ? S.s_row : S.s_col;
            const std::vector<int64_t> &sb = rows ? S.row_seg_begin : S.col_seg_begin;
            const int64_t lo = batched || k < 0 ? sb.front() : sb[k];
            const int64_t hi = batched || k < 0 ? sb.back() : sb[k + 1];
            if (hi > lo) {
                GramPartArgs ga{};
                ga.segs = c->dev<SegItem>(L.m_segs) + sbase + lo;
                ga.nseg = (int32_t)(hi - lo);
                ga.sides = a.sides;
                ga.idx = a.idx;
                ga.val = a.val;
                ga.other = a.other;
                ga.ks_other = a.ks_other;
                ga.gpart = c->dev<float>(L.gpart);
                if ((st = timed(c, kKGram, [&] { return launch_gram_part(L.kc, ga, c->ls); }))) return st;
            }
        }
        // MFMA path: the light entities (at most kLightNnz entries, the tail of
        // each decreasing-degree range) run on the VALU-Gram kernel, which needs
        // fewer registers and so keeps more entities in flight; 16 < K <= 32 in
        // FP32 arithmetic: light entities two per wavefront.  Entities with at
        // most lowrank_max_nnz() entries under a factored per-row prior (the
        // tail) take the low-rank kernel, those without entries (the very tail)
        // the empty-entity kernel.
        const bool duo = L.kc == 32 && (c->prec() == kP32 || c->prec() == kPBF);
        const bool lsplit = L.mfma || duo;
        // heavy entities two per wavefront (MFMA Grams) when the stage's side
        // has enough of them to fill the chip at half as many wavefronts; the
        // count is the stage's, so batched, per-block and single-step passes
        // choose alike
        const int64_t nheavy = rows ? S.i_row_light - S.i_row_heavy : S.i_col_light - S.i_col_heavy;
        const bool mf_duo = nheavy >= kMfDuoMin;
        enum { kWave = 0, kLight = 1, kGroup = 2 };
        std::vector<std::pair<int64_t, int64_t>> split;
        std::vector<int> kind;
        for (size_t ri = 0; ri < ranges.size(); ++ri) {
            int64_t light, lowr;
            if (batched) {
                light = rows ? S.i_row_light : S.i_col_light;
                lowr = rows ? S.i_row_lowrank : S.i_col_lowrank;
            } else {
                const int32_t q = k < 0 ? (int32_t)ri : k;
                const int64_t base = rows ? S.i_row_blk : S.i_col_blk;
                light = base + (rows ? S.row_item_light : S.col_item_light)[q];
                lowr = base + (rows ? S.row_item_lowrank : S.col_item_lowrank)[q];
            }
            const int64_t lo = ranges[ri].first, hi = ranges[ri].second;
            lowr = std::min(std::max(lowr, lo), hi);
            light = lsplit ? std::min(std::max(light, lo), lowr) : lowr;
            split.push_back({lo, light});
            kind.push_back(kWave);
            split.push_back({light, lowr});
            kind.push_back(kLight);
            // the copies under a factored per-row prior with few entries: one
            // launch over their prior groups (range of groups, not of items)
            int64_t g0, g1;
            if (batched) {
                g0 = rows ? S.g_row_b0 : S.g_col_b0;
                g1 = rows ? S.g_row_b1 : S.g_col_b1;
            } else {
                const int32_t q = k < 0 ? (int32_t)ri : k;
                const std::vector<int64_t> &gb = rows ? S.g_row_blk : S.g_col_blk;
                g0 = gb[q];
                g1 = gb[q + 1];
            }
            split.push_back({g0, g1});
            kind.push_back(kGroup);
        }
        for (size_t ri = 0; ri < split.size(); ++ri) {
            const auto &r = split[ri];
            if (r.second <= r.first) continue;
            UpdArgs b = a;
            if (kind[ri] == kGroup) {
                b.items = c->dev<int2>(L.m_gitems);
                b.gstart = c->dev<int32_t>(L.m_gstart) + r.first;
                b.ngroups = (int32_t)(r.second - r.first);
                const int32_t g = (int32_t)std::min<int64_t>(b.ngroups, kWaveGridCap);
                if ((st = timed(c, kcls, [&] { return launch_update_group(L.kc, c->prec(), b, g, c->ls); })))
                    return st;
                continue;
            }
            b.items = c->dev<int2>(L.m_items) + r.first;
            b.nitems = (int32_t)(r.second - r.first);
            if (L.mfma) {
                b.splits = c->dev<int2>(L.m_splits) + r.first;
                b.gpart = c->dev<float>(L.gpart);
            }
            if (duo && (kind[ri] == kLight || (L.mfma && mf_duo))) {
                // two entities per wavefront: light ones with the VALU Gram,
                // with BF16 state the others with two MFMA Grams
                const bool mf = kind[ri] != kLight;
                const int32_t g = (int32_t)std::min<int64_t>((b.nitems + 1) / 2, kWaveGridCap);
                if ((st = timed(c, kcls, [&] { return launch_update_duo(c->prec(), b, g, c->ls, mf); }))) return st;
                continue;
            }
            const bool vgram = kind[ri] == kLight;
            const int32_t g = (int32_t)std::min<int64_t>(b.nitems, kWaveGridCap);
            if ((st = timed(c, kcls, [&] { return launch_update_wave(L.kc, c->prec(), b, g, c->ls, vgram); })))
                return st;
        }
    }
    if (!c->fp64()) {
        UpdArgs f = a;
        f.items = a.fb_list;
        f.nitems_dev = a.fb_count;
        f.fb_list = nullptr;
        f.fb_count = nullptr;
        f.theta = 0.0f;
        const int32_t fp = c->bf() ? kPFB16 : kPFB32;
        if ((st = timed(c, kKFallback, [&] { return launch_update_wave(L.kc, fp, f, kFallbackGrid, c->ls); })))
            return st;
        // the queue holds this pass's entities only: a single step clears it
        // here, a batched sweep (one pass over every block) in the sweep-state
        // advance, and a per-block sweep after each block's pass (else the next
        // block's redo would take this block's queued entities again, with the
        // other side's factors already redrawn)
        if (!use_ss || k >= 0) {
            int32_t *fb = a.fb_count;
            if ((st = timed(c, kKFill, [&] { return launch_fill_i32(fb, 0, 1, c->ls); }))) return st;
        }
    }
    return BMF_OK;
}

// Fixed-order SSE of every stage block (k = -1) or of stage block k from the
// per-column slots.
static bmf_status reduce_sse(bmf_ctx *c, int32_t k) {
    const int32_t nbs = (int32_t)c->S.blocks.size();
    const ReduceJob *rj = c->dev<ReduceJob>(c->L.m_reduce) + (k < 0 ? 0 : k);
    const int32_t nr = k < 0 ? nbs : 1;
    return timed(c, kKReduce, [&] { return launch_reduce(rj, nr, c->L.npair, c->ls); });
}

// Residual SSE of stage block k's columns on their own (a tau step).
static bmf_status run_sse(bmf_ctx *c, int32_t k) {
    const Layout &L = c->L;
    StageLists &S = c->S;
    SseArgs a{};
    a.sides = c->dev<SideDesc>(L.m_sides);
    a.ord = c->dev<int32_t>(L.ord);
    a.ptr = c->dev<int64_t>(L.csc_ptr);
    a.idx = c->dev<int32_t>(L.csc_idx);
    a.val = c->dev<void>(L.csc_val);
    a.X = c->dev<void>(L.X);
    a.W = c->dev<void>(L.W);
    a.ks = L.ks_m;
    a.K = c->cfg.K;
    a.sse_col = c->dev<double>(L.sse_col);
    const int64_t lo = S.col_tile_begin[k], hi = S.col_tile_begin[k + 1];
    a.tiles = c->dev<Tile>(L.m_tiles) + S.t_col_blk + lo;
    const int32_t n = (int32_t)(hi - lo);
    bmf_status st = timed(c, kKSse, [&] { return launch_sse(L.kc, c->prec(), a, n, c->ls); });
    if (st) return st;
    return reduce_sse(c, k);
}

static bmf_status run_stats(bmf_ctx *c, int32_t side_lo, int32_t side_hi, bool reduce = true) {
    const Layout &L = c->L;
    StageLists &S = c->S;
    const int32_t nbs = (int32_t)S.blocks.size();
    const int64_t lo = S.side_stats_begin[side_lo], hi = S.side_stats_begin[side_hi];
    bmf_status st;
    if (hi > lo) {
        StatsArgs a{};
        a.jobs = c->dev<StatsJob>(L.m_stats) + lo;
        a.sides = c->dev<SideDesc>(L.m_sides);
        a.X = c->dev<void>(L.X);
        a.W = c->dev<void>(L.W);
        a.nrow_sides = nbs;
        a.ks = L.ks_m;
        a.K = c->cfg.K;
        a.part = c->dev<double>(L.stats_part);
        const int32_t n = (int32_t)(hi - lo);
        if ((st = timed(c, kKStats, [&] { return launch_stats(c->prec(), a, n, c->ls); }))) return st;
    }
    if (!reduce) return BMF_OK;
    const ReduceJob *rj = c->dev<ReduceJob>(L.m_reduce) + nbs + side_lo;
    return timed(c, kKReduce, [&] { return launch_reduce(rj, side_hi - side_lo, c->L.npair, c->ls); });
}

static bmf_status run_hyper(bmf_ctx *c, int32_t j0, int32_t j1, uint32_t t, bool use_ss, bool advance = false,
                            bool noise_ready = false) {
    if (j1 <= j0) return BMF_OK;
    const Layout &L = c->L;
    HyperArgs a{};
    a.jobs = c->dev<HyperJob>(L.m_hyper) + j0;
    a.part = c->dev<double>(L.stats_final);
    a.sse_part = c->dev<double>(L.sse_final);
    a.mu0 = c->dev<double>(L.mu0);
    a.W0inv = c->dev<double>(L.W0inv);
    a.beta0 = c->cfg.beta0;
    a.nu0 = c->cfg.nu0;
    a.a0 = c->cfg.tau_a0;
    a.b0 = c->cfg.tau_b0;
    a.K = c->cfg.K;
    a.t = t;
    a.ss = use_ss ? c->dev<SweepState>(L.sweep) : nullptr;
    a.k0 = (uint32_t)(c->cfg.seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(c->cfg.seed >> 32);
    a.nonpd = c->dev<int32_t>(L.counters) + kNonPD;
    if (advance) {
        a.advance = c->dev<SweepState>(L.sweep);
        a.fb_counts = c->dev<int32_t>(L.counters) + kFbRow;
        a.done = c->dev<int32_t>(L.counters) + kHyperDone;
    }
    a.noise = c->dev<double>(L.nw_noise) + (int64_t)j0 * (c->cfg.K * (c->cfg.K + 3) / 2);
    a.noise_ready = noise_ready ? 1 : 0;
    return timed(c, kKHyper, [&] { return launch_hyper(a, j1 - j0, c->ls); });
}

// Enqueue one sweep of the active stage on c->ls: rows, columns, SSE, NW
// statistics, hyperparameter and tau draws, then the sweep-state advance.
// Mixture priors (Sec. 5.1): every row under a propagated mixture takes the
// component of largest responsibility at its current value (force0: the
// largest component, for the initial state) into its side's prior rows.
static bmf_status run_gmm_pick(bmf_ctx *c, bool force0) {
    if (c->cfg.approx != BMF_APPROX_GMM || c->S.pitems.empty()) return BMF_OK;
    const Layout &L = c->L;
    GmmPickArgs a{};
    a.items = c->dev<int2>(L.m_pitems);
    a.nitems = (int32_t)c->S.pitems.size();
    a.gsides = c->dev<GmmSide>(L.m_gsides);
    a.plane = (L.E_r + L.E_c) * L.prow;
    a.aux_plane = 2 * (L.E_r + L.E_c);
    a.ks_state = L.ks_m;
    a.K = c->cfg.K;
    a.prow = L.prow;
    a.ncomp = L.ncomp;
    a.force0 = force0 ? 1 : 0;
    return timed(c, kKPick, [&] { return launch_gmm_pick(c->prec(), a, c->ls); });
}

// Per-column noise precisions: the row pass's scaled factors and values from
// the current W and tau_d (every block of the stage, or block k), and the
// tau_d draws after the column pass.
static TauColArgs tau_args(bmf_ctx *c, int32_t k, uint32_t t, bool use_ss) {
    const Layout &L = c->L;
    TauColArgs a{};
    a.jobs = c->dev<TauColJob>(L.m_taujobs) + (k < 0 ? 0 : k);
    a.njobs = k < 0 ? (int32_t)c->S.taujobs.size() : 1;
    a.tau = c->dev<double>(L.tau_col);
    a.W = c->dev<void>(L.W);
    a.Wt = c->dev<void>(L.Wt);
    a.ks = L.ks_m;
    a.K = c->cfg.K;
    a.val = c->dev<void>(L.csr_val);
    a.vt = c->dev<void>(L.vt);
    a.idx = c->dev<int32_t>(L.csr_idx);
    a.cptr = c->dev<int64_t>(L.csc_ptr);
    a.sse_col = c->dev<double>(L.sse_col);
    a.a0 = c->cfg.tau_a0;
    a.b0 = c->cfg.tau_b0;
    a.ss = use_ss ? c->dev<SweepState>(L.sweep) : nullptr;
    a.t = t;
    a.k0 = (uint32_t)(c->cfg.seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(c->cfg.seed >> 32);
    return a;
}

static bmf_status run_tau_scale(bmf_ctx *c, int32_t k) {
    if (!c->cfg.tau_per_column) return BMF_OK;
    const TauColArgs a = tau_args(c, k, 0, false);
    return timed(c, kKFill, [&] { return launch_tau_scale(c->prec(), a, c->ls); });
}

static bmf_status run_tau_cols(bmf_ctx *c, int32_t k, uint32_t t, bool use_ss) {
    if (!c->cfg.tau_per_column || !c->cfg.sample_tau) return BMF_OK;
    const TauColArgs a = tau_args(c, k, t, use_ss);
    return timed(c, kKHyper, [&] { return launch_tau_cols(a, c->ls); });
}

static bmf_status enqueue_sweep(bmf_ctx *c) {
    StageLists &S = c->S;
    bmf_status st;
    if ((st = run_gmm_pick(c, false))) return st;
    if ((st = run_tau_scale(c, -1))) return st;
    const int32_t nbs = (int32_t)S.blocks.size();
    // the column pass always evaluates the residual SSE of every block (the tau
    // statistic when tau is sampled; the training fit, bmf_get_stats, always)
    if (c->cfg.batched) {
        // one launch per step; the SSE and statistics reductions share a launch
        // (their jobs are contiguous), and the hyperparameter launch advances
        // the sweep state in its last block
        if ((st = run_pass(c, true, 0, nullptr, -1, true))) return st;
        if ((st = run_pass(c, false, 0, nullptr, -1, true, true))) return st;
        if ((st = run_stats(c, 0, 2 * nbs, false))) return st;
        const ReduceJob *rj = c->dev<ReduceJob>(c->L.m_reduce);
        const int32_t nr = 3 * nbs;
        // the reduction launch also draws the Normal-Wishart noise of every
        // hyper job (extra blocks), off the hyperparameter launch's path
        NoiseArgs na{};
        na.jobs = c->dev<HyperJob>(c->L.m_hyper);
        na.njobs = S.hyper_begin[nbs];
        na.K = c->cfg.K;
        na.nu0 = c->cfg.nu0;
        na.ss = c->dev<SweepState>(c->L.sweep);
        na.k0 = (uint32_t)(c->cfg.seed & 0xFFFFFFFFu);
        na.k1 = (uint32_t)(c->cfg.seed >> 32);
        na.noise = c->dev<double>(c->L.nw_noise);
        if ((st = timed(c, kKReduce, [&] { return launch_reduce(rj, nr, c->L.npair, c->ls, &na); }))) return st;
        if ((st = run_tau_cols(c, -1, 0, true))) return st;
        if (S.hyper_begin[nbs] > 0) return run_hyper(c, 0, S.hyper_begin[nbs], 0, true, true, true);
    } else {
        for (int32_t k = 0; k < nbs; ++k) {
            if ((st = run_pass(c, true, 0, nullptr, k, true))) return st;
            if ((st = run_pass(c, false, 0, nullptr, k, true, true))) return st;
            if ((st = reduce_sse(c, k))) return st;
            if ((st = run_stats(c, k, k + 1))) return st;
            if ((st = run_stats(c, nbs + k, nbs + k + 1))) return st;
            if ((st = run_tau_cols(c, k, 0, true))) return st;
            if ((st = run_hyper(c, S.hyper_begin[k], S.hyper_begin[k + 1], 0, true))) return st;
        }
    }
    SweepState *ss = c->dev<SweepState>(c->L.sweep);
    int32_t *fbc = c->dev<int32_t>(c->L.counters) + kFbRow;
    return timed(c, kKFill, [&] { return launch_advance(ss, fbc, c->ls); });
}

static void drop_graph(bmf_ctx *c) {
    if (c->gexec) {
        hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
}

// Capture one sweep into a graph (batched mode).  The capture runs on an
// internal stream; the graph is launched on the caller's stream.
static bmf_status capture_sweep(bmf_ctx *c) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    c->ls = c->cap_stream;
    const bool timing = c->timing;
    c->timing = false;
    bmf_status st = enqueue_sweep(c);
    c->timing = timing;
    c->ls = c->stream;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (st) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(c, BMF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
        c->gexec = nullptr;
        return fail(c, BMF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    return BMF_OK;
}

static bmf_status sweep_once(bmf_ctx *c) {
    const bmf_config &g = c->cfg;
    bmf_status st;
    if (g.batched && !c->timing) {
        if (!c->gexec && (st = capture_sweep(c))) return st;
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else {
        if ((st = enqueue_sweep(c))) return st;
    }
    // host mirror of the device sweep state
    const bool keep = c->t >= g.burnin && (c->t - g.burnin) % g.thin == 0 && c->kept < g.max_kept;
    if (keep) c->kept += 1;
    c->t += 1;
    c->agg_valid = false;
    return BMF_OK;
}

// n sweeps of the active stage; the progress callback may stop the loop
// before a sweep is enqueued (BMF_EABORT, state after the previous sweep).
static bmf_status run_sweeps(bmf_ctx *c, int32_t n) {
    for (int32_t q = 0; q < n; ++q) {
        if (c->progress && c->progress(c->progress_user, c->stage, c->t) != 0)
            return fail(c, BMF_EABORT, "stopped by the progress callback before sweep " + std::to_string(c->t) +
                                           " of stage " + std::to_string(c->stage));
        bmf_status st = sweep_once(c);
        if (st) return st;
    }
    return BMF_OK;
}

static bmf_status write_sweep_state(bmf_ctx *c, uint32_t t, int32_t kept) {
    const bmf_config &g = c->cfg;
    SweepState ss{};
    ss.t = t;
    ss.kept = kept;
    ss.burnin = g.burnin;
    ss.thin = g.thin;
    ss.max_kept = g.max_kept;
    ss.slot_bytes = c->L.Emax * c->L.ks_p * c->L.sp;
    const bool keep = (int64_t)t >= g.burnin && ((int64_t)t - g.burnin) % g.thin == 0 && kept < g.max_kept;
    ss.slot = keep ? kept : -1;
    bmf_status st = upload(c, c->L.sweep, &ss, sizeof(ss));
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BMF_OK;
}

// Autotuner of the register kernel's lane groups: for every candidate number
// of entries per lane, rebuild the tiles and time the row and column passes
// on the stage's real data; keep the fastest per pass.  Runs before the
// initial state is written, so it leaves no trace in the chain (the FP32
// fallback counters are restored).
static bmf_status autotune(bmf_ctx *c) {
    const int32_t cand[] = {8, 16, 32, 64, 128, 256};
    const Layout &L = c->L;
    int32_t saved[kNumCounters];
    bmf_status st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(saved, c->base + L.counters, sizeof(saved), hipMemcpyDeviceToHost));
    const bool timing = c->timing;
    c->timing = false;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    double best[2] = {1e30, 1e30};
    int32_t pick[2] = {32, 32};
    for (int32_t v : cand) {
        build_tiles(c, v, v);
        if ((st = upload_tiles(c))) break;
        for (int pass = 0; pass < 2; ++pass) {
            if ((st = run_pass(c, pass == 0, 0, nullptr, -1, false))) break;   // warm-up
            HIPCHK(c, hipEventRecord(e0, c->stream));
            for (int r = 0; r < 2 && !st; ++r) st = run_pass(c, pass == 0, 0, nullptr, -1, false);
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            if (ms < best[pass]) {
                best[pass] = ms;
                pick[pass] = v;
            }
        }
        if (st) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->timing = timing;
    if (st) return st;
    build_tiles(c, pick[0], pick[1]);
    if ((st = upload_tiles(c))) return st;
    HIPCHK(c, hipMemcpy(c->base + L.counters, saved, sizeof(saved), hipMemcpyHostToDevice));
    return BMF_OK;
}

// Initial factors of every side of the active stage.
static bmf_status init_factors(bmf_ctx *c) {
    const Layout &L = c->L;
    StageLists &S = c->S;
    InitArgs a{};
    a.items = c->dev<int2>(L.m_items2);
    a.nitems = (int32_t)S.ents.size();
    a.sides = c->dev<SideDesc>(L.m_sides);
    a.K = c->cfg.K;
    a.prow = L.prow;
    a.k0 = (uint32_t)(c->cfg.seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(c->cfg.seed >> 32);
    // rows and columns live in different arrays: two launches over the entity list halves
    const int64_t nrow_items = S.row_ents;
    bmf_status st;
    for (int pass = 0; pass < 2; ++pass) {
        InitArgs b = a;
        b.items = a.items + (pass == 0 ? 0 : nrow_items);
        b.nitems = (int32_t)(pass == 0 ? nrow_items : (int64_t)S.ents.size() - nrow_items);
        b.self = c->dev<void>(pass == 0 ? L.X : L.W);
        b.ks_self = L.ks_m;
        if ((st = timed(c, kKInit, [&] { return launch_init(c->prec(), b, c->ls); }))) return st;
    }
    return BMF_OK;
}

// Begin stage s: work lists, schedules (autotuned), priors, initial state.
static bmf_status begin_stage(bmf_ctx *c, int32_t s) {
    drop_graph(c);
    build_stage_lists(c, s);
    bmf_status st;
    if ((st = upload_stage(c))) return st;
    const Layout &L = c->L;
    StageLists &S = c->S;
    // hyperparameters (0, I), tau
    const int32_t K = c->cfg.K;
    std::vector<double> hy(L.hy, 0.0);
    for (int k = 0; k < K; ++k) {
        hy[k * K + k] = 1.0;                                    // Lambda = I, mu = 0
        hy[kHyPacked(L) + k * (k + 1) / 2 + k] = 1.0;          // packed Lambda
    }
    const double tau0 = c->cfg.sample_tau ? c->cfg.tau_a0 / c->cfg.tau_b0 : c->cfg.tau_fixed;
    for (int32_t b : S.blocks) {
        if ((st = upload(c, L.hyper + ((int64_t)b * 2 + 0) * L.hy * 8, hy.data(), 8 * L.hy))) return st;
        if ((st = upload(c, L.hyper + ((int64_t)b * 2 + 1) * L.hy * 8, hy.data(), 8 * L.hy))) return st;
        if ((st = upload(c, L.tau + 8 * (int64_t)b, &tau0, 8))) return st;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (c->cfg.tau_per_column) {
        const double one = 1.0;
        if ((st = upload(c, L.one, &one, 8))) return st;
        for (const TauColJob &j : S.taujobs) {
            std::vector<double> tv((size_t)j.C, tau0);
            if ((st = upload(c, L.tau_col + 8 * j.w_off, tv.data(), 8 * tv.size()))) return st;
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    if ((st = run_gmm_pick(c, true))) return st;      // mixture priors: the largest component to start
    if ((st = init_factors(c))) return st;
    if (c->reg() && c->cfg.lane_nnz == 0 && c->cfg.batched) {
        if ((st = autotune(c))) return st;
        if ((st = init_factors(c))) return st;      // the tuning passes overwrote the factors
    } else {
        const int32_t v = c->cfg.lane_nnz > 0 ? c->cfg.lane_nnz : 32;
        build_tiles(c, v, v);
        if ((st = upload_tiles(c))) return st;
    }
    {
        std::vector<double> z(S.blocks.size(), 0.0);
        if ((st = upload(c, L.sse_final, z.data(), 8 * z.size()))) return st;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if ((st = write_sweep_state(c, 0, 0))) return st;
    c->stage = s;
    c->t = 0;
    c->kept = 0;
    c->agg_valid = false;
    return BMF_OK;
}

static bmf_status finalize_stage(bmf_ctx *c) {
    if (c->stage == 0 || c->finalized >= c->stage) return BMF_OK;
    const Layout &L = c->L;
    StageLists &S = c->S;
    if (c->kept < 1) return fail(c, BMF_ESTATE, "no kept sample in the active stage");
    MmArgs a{};
    a.items = c->dev<int2>(L.m_items2);
    a.nitems = (int32_t)S.ents.size();
    a.sides = c->dev<SideDesc>(L.m_sides);
    a.sample = c->base + L.sample;
    a.slot_elems = L.Emax * L.ks_p;
    a.ks = L.ks_p;
    a.S = c->kept;
    a.K = c->cfg.K;
    a.prow = L.prow;
    a.out = c->dev<double *>(L.m_mmout);
    a.ridged = c->dev<int32_t>(L.counters) + kRidged;
    const int32_t sprec = c->fp64() ? kP64 : kP32;
    bmf_status st;
    if (c->cfg.approx == BMF_APPROX_MM) {
        if ((st = timed(c, kKMM, [&] { return launch_mm(sprec, a, c->ls); }))) return st;
    } else {
        // lambda-means per row, then the dominant cluster's or each
        // component's moment matching, then (mixture) the pooled moments
        const int32_t nbs2 = 2 * (int32_t)S.blocks.size();
        const int64_t Etot = L.E_r + L.E_c;
        LmeansArgs la{};
        la.items = a.items;
        la.nitems = a.nitems;
        la.sides = a.sides;
        la.sample = a.sample;
        la.slot_elems = a.slot_elems;
        la.ks = a.ks;
        la.S = a.S;
        la.K = a.K;
        la.lam_scale = c->cfg.lambda_scale;
        la.ncomp = L.ncomp;
        la.labels = c->dev<uint8_t *>(L.m_labptr);
        la.maxS = c->cfg.max_kept;
        la.which = c->dev<int8_t>(L.which);
        la.aux = c->dev<double *>(L.m_auxptr);
        la.aux_plane = 2 * Etot;
        if ((st = timed(c, kKMM, [&] { return launch_lmeans(sprec, la, c->ls); }))) return st;
        a.labels = la.labels;
        a.which = la.which;
        a.maxS = la.maxS;
        const bool gmm = c->cfg.approx == BMF_APPROX_GMM;
        for (int32_t cc = 0; cc < L.ncomp; ++cc) {
            MmArgs m = a;
            m.comp = cc;
            m.aux = c->dev<double *>(L.m_auxptr) + (int64_t)cc * nbs2;
            if (gmm) m.out = c->dev<double *>(L.m_gmmout) + (int64_t)cc * nbs2;
            if ((st = timed(c, kKMM, [&] { return launch_mm(sprec, m, c->ls); }))) return st;
        }
        if (gmm) {
            GmmPoolArgs g{};
            g.items = a.items;
            g.nitems = a.nitems;
            g.which = la.which;
            g.comp = c->dev<double *>(L.m_gmmout);
            g.aux = c->dev<double *>(L.m_auxptr);
            g.plane = Etot * L.prow;
            g.aux_plane = 2 * Etot;
            g.out = c->dev<double *>(L.m_mmout);
            g.K = a.K;
            g.prow = L.prow;
            g.ncomp = L.ncomp;
            if ((st = timed(c, kKMM, [&] { return launch_gmm_pool(g, c->ls); }))) return st;
        }
    }
    if (L.pfrow && c->stage < 3) {
        PfacArgs f{};
        f.items = a.items;
        f.nitems = a.nitems;
        f.out = a.out;
        f.pfout = c->dev<float *>(L.m_pfout);
        f.K = c->cfg.K;
        f.prow = L.prow;
        f.pfrow = L.pfrow;
        if ((st = timed(c, kKMM, [&] { return launch_pfac(L.kc, f, c->ls); }))) return st;
    }
    c->finalized = c->stage;
    c->done_stages[c->stage] = c->kept;
    return BMF_OK;
}

static bool stage_has_blocks(const bmf_ctx *c, int32_t s) {
    for (const PlanBlock &B : c->plan.blocks)
        if (B.stage == s) return true;
    return false;
}

static int32_t last_stage(const bmf_ctx *c) {
    int32_t s = 1;
    for (int32_t q = 2; q <= 3; ++q)
        if (stage_has_blocks(c, q)) s = q;
    return s;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

bmf_status bmf_config_defaults(bmf_config *cfg) {
    if (!cfg) return BMF_EINVAL;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->K = 10;
    cfg->I = 1;
    cfg->J = 1;
    cfg->order = BMF_ORDER_GIVEN;
    cfg->beta0 = 2.0;
    cfg->nu0 = 10.0;
    cfg->sample_tau = 1;
    cfg->tau_a0 = 1.0;
    cfg->tau_b0 = 1.0;
    cfg->tau_fixed = 1.0;
    cfg->burnin = 0;
    cfg->thin = 1;
    cfg->max_kept = 1;
    cfg->precision = BMF_PREC_FP32;
    cfg->pivot_theta = std::ldexp(1.0, -10);
    cfg->batched = 1;
    cfg->approx = BMF_APPROX_MM;
    cfg->lambda_scale = 2.0;
    cfg->ncomp = 3;
    return BMF_OK;
}

const char *bmf_status_string(bmf_status s) {
    switch (s) {
    case BMF_OK: return "BMF_OK";
    case BMF_EINVAL: return "BMF_EINVAL";
    case BMF_ENOMEM: return "BMF_ENOMEM";
    case BMF_EDEVICE: return "BMF_EDEVICE";
    case BMF_ENOTPD: return "BMF_ENOTPD";
    case BMF_ESTATE: return "BMF_ESTATE";
    case BMF_EUNSUPPORTED: return "BMF_EUNSUPPORTED";
    case BMF_EABORT: return "BMF_EABORT";
    }
    return "unknown status";
}

const char *bmf_last_error(const bmf_ctx *c) { return c ? c->err.c_str() : "null context"; }

bmf_status bmf_workspace_size(const bmf_config *cfg, size_t *bytes) {
    std::string err;
    bmf_status st = validate(cfg, err);
    if (st) return st;
    if (!bytes) return BMF_EINVAL;
    Layout L;
    if (!layout_for(*cfg, L, err)) return BMF_EINVAL;
    *bytes = (size_t)L.total;
    return BMF_OK;
}

// Per-block offsets into the pointer, factor and entry arrays.
static void block_offsets(bmf_ctx *c) {
    int64_t pr = 0, pc = 0, xr = 0, wc = 0, nzb = 0;
    for (const PlanBlock &B : c->plan.blocks) {
        c->nz_off[0].push_back(nzb);
        c->nz_off[1].push_back(nzb);
        nzb += B.M;
        c->csr_ptr_off.push_back(pr);
        c->csc_ptr_off.push_back(pc);
        c->x_off.push_back(xr);
        c->w_off.push_back(wc);
        c->ord_row_off.push_back(xr);
        c->ord_col_off.push_back(c->L.E_r + wc);
        pr += B.R + 1;
        pc += B.C + 1;
        xr += B.R;
        wc += B.C;
    }
}

static bmf_status init_common(const bmf_config *cfg, bmf_ctx **out, bool device) {
    if (!out) return BMF_EINVAL;
    *out = nullptr;
    bmf_ctx *c = new (std::nothrow) bmf_ctx();
    if (!c) return BMF_ENOMEM;
    std::string err;
    bmf_status st = validate(cfg, err);
    if (!st && !layout_for(*cfg, c->L, err)) st = BMF_EINVAL;
    if (st) {
        *out = c;
        c->err = err;
        return st;
    }
    c->cfg = *cfg;
    if (c->cfg.lambda_scale == 0.0) c->cfg.lambda_scale = 2.0;
    c->cfg.ncomp = ncomp_of(*cfg);
    c->cfg.row = nullptr;
    c->cfg.col = nullptr;
    c->cfg.val = nullptr;
    c->cfg.mu0 = nullptr;
    c->cfg.W0 = nullptr;
    const int32_t K = cfg->K;
    c->mu0.assign(K, 0.0);
    if (cfg->mu0) std::copy(cfg->mu0, cfg->mu0 + K, c->mu0.begin());
    {
        std::vector<double> W0(K * K, 0.0), Lf;
        if (cfg->W0) std::copy(cfg->W0, cfg->W0 + K * K, W0.begin());
        else
            for (int k = 0; k < K; ++k) W0[k * K + k] = 1.0;
        spd_cholesky(K, W0.data(), Lf);
        // W0^-1 = L^-T L^-1, column by column
        c->W0inv.assign(K * K, 0.0);
        std::vector<double> y(K), x(K);
        for (int col = 0; col < K; ++col) {
            for (int i = 0; i < K; ++i) {
                double s = (i == col) ? 1.0 : 0.0;
                for (int p = 0; p < i; ++p) s -= Lf[i * K + p] * y[p];
                y[i] = s / Lf[i * K + i];
            }
            for (int i = K - 1; i >= 0; --i) {
                double s = y[i];
                for (int p = i + 1; p < K; ++p) s -= Lf[p * K + i] * x[p];
                x[i] = s / Lf[i * K + i];
            }
            for (int r = 0; r < K; ++r) c->W0inv[r * K + col] = x[r];
        }
    }
    // centering: sequential FP64 mean in COO order
    double s = 0.0;
    for (int64_t e = 0; e < cfg->nnz; ++e) s += (double)cfg->val[e];
    c->ybar = cfg->nnz > 0 ? s / (double)cfg->nnz : 0.0;
    c->fingerprint = data_fingerprint(*cfg);
    const bool host_plan = !device || cfg->plan_on_host;
    if (host_plan) {
        st = build_plan(*cfg, c->plan, err);
        if (st) {
            *out = c;
            c->err = err;
            return st;
        }
        block_offsets(c);
    }
    *out = c;
    if (!device) return BMF_OK;

    // ---- device part
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(c, BMF_EDEVICE, "no HIP device");
    c->stream = (hipStream_t)cfg->stream;
    c->ls = c->stream;
    const Layout &L = c->L;
    if (cfg->workspace) {
        if ((int64_t)cfg->workspace_bytes < L.total)
            return fail(c, BMF_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
        if (((uintptr_t)cfg->workspace & 255u) != 0) return fail(c, BMF_EINVAL, "workspace must be 256-byte aligned");
        c->base = (char *)cfg->workspace;
    } else {
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)L.total) != hipSuccess) return fail(c, BMF_ENOMEM, "hipMalloc of the workspace failed");
        c->base = (char *)p;
        c->own = true;
    }
    c->device = true;
    HIPCHK(c, hipMemsetAsync(c->base, 0, (size_t)L.total, c->stream));
    const bool fp64 = cfg->precision == BMF_PREC_FP64;
    if (!host_plan) {
        // the per-entry half of the plan on the GPU, straight into the workspace
        GpuPlanDst dst{};
        dst.csr_ptr = c->dev<int64_t>(L.csr_ptr);
        dst.csc_ptr = c->dev<int64_t>(L.csc_ptr);
        dst.csr_idx = c->dev<int32_t>(L.csr_idx);
        dst.csc_idx = c->dev<int32_t>(L.csc_idx);
        dst.csr_val = c->dev<void>(L.csr_val);
        dst.csc_val = c->dev<void>(L.csc_val);
        dst.csr_ent = c->dev<int32_t>(L.csr_ent);
        dst.csc_ent = c->dev<int32_t>(L.csc_ent);
        dst.colsq = c->dev<double>(L.colsq);
        dst.rowpos = c->dev<int64_t>(L.rowpos);
        dst.colpos = c->dev<int64_t>(L.colpos);
        if ((st = gpu_build_plan(*cfg, c->ybar, fp64, c->plan, dst, c->stream, err))) return fail(c, st, err);
        block_offsets(c);
        std::vector<int32_t> hord;
        for (int pass = 0; pass < 2; ++pass) {
            hord.clear();
            for (const PlanBlock &B : c->plan.blocks) {
                std::vector<int32_t> o = degree_order(pass == 0 ? B.csr_ptr : B.csc_ptr);
                hord.insert(hord.end(), o.begin(), o.end());
            }
            if ((st = upload(c, L.ord + (pass == 0 ? 0 : 4 * L.E_r), hord.data(), hord.size() * 4))) return st;
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    const Plan &P = c->plan;
    const int64_t nb = (int64_t)P.blocks.size();
    // CSR / CSC with centred values, degree orders (host plan)
    if (host_plan) {
    std::vector<int64_t> hptr;
    std::vector<int32_t> hidx;
    std::vector<double> vd;
    std::vector<float> vf;
    std::vector<int32_t> hord;
    std::vector<double> colsq((size_t)L.E_c, 0.0);   // per column: sum of squared stored values
    for (int pass = 0; pass < 2; ++pass) {
        hptr.clear();
        hidx.clear();
        vd.clear();
        vf.clear();
        hord.clear();
        int64_t base_nz = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const PlanBlock &B = P.blocks[b];
            const std::vector<int64_t> &bp = pass == 0 ? B.csr_ptr : B.csc_ptr;
            const std::vector<int32_t> &bi = pass == 0 ? B.csr_idx : B.csc_idx;
            const std::vector<int64_t> &be = pass == 0 ? B.csr_entry : B.csc_entry;
            for (int64_t v : bp) hptr.push_back(base_nz + v);
            hidx.insert(hidx.end(), bi.begin(), bi.end());
            for (int64_t e : be) {
                const double r = (double)cfg->val[e] - c->ybar;
                if (fp64) vd.push_back(r);
                else vf.push_back((float)r);
            }
            if (pass == 1) {
                // per column, the sum of its squared values as stored (for the
                // residual SSE of the column pass)
                for (size_t d = 0; d + 1 < bp.size(); ++d) {
                    double s = 0.0;
                    for (int64_t q = bp[d]; q < bp[d + 1]; ++q) {
                        const double r = (double)cfg->val[be[q]] - c->ybar;
                        const double rs = fp64 ? r : (double)(float)r;
                        s += rs * rs;
                    }
                    colsq[(size_t)(c->w_off[b] + (int64_t)d)] = s;
                }
            }
            std::vector<int32_t> o = degree_order(bp);
            hord.insert(hord.end(), o.begin(), o.end());
            base_nz += B.M;
        }
        const int64_t o_ptr = pass == 0 ? L.csr_ptr : L.csc_ptr;
        const int64_t o_idx = pass == 0 ? L.csr_idx : L.csc_idx;
        const int64_t o_val = pass == 0 ? L.csr_val : L.csc_val;
        if ((st = upload(c, o_ptr, hptr.data(), hptr.size() * 8))) return st;
        if ((st = upload(c, o_idx, hidx.data(), hidx.size() * 4))) return st;
        if (fp64) {
            if ((st = upload(c, o_val, vd.data(), vd.size() * 8))) return st;
        } else {
            if ((st = upload(c, o_val, vf.data(), vf.size() * 4))) return st;
        }
        if ((st = upload(c, L.ord + (pass == 0 ? 0 : 4 * L.E_r), hord.data(), hord.size() * 4))) return st;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if ((st = upload(c, L.colsq, colsq.data(), colsq.size() * 8))) return st;
    if ((st = upload(c, L.rowpos, P.row_pos.data(), 8 * P.row_pos.size()))) return st;
    if ((st = upload(c, L.colpos, P.col_pos.data(), 8 * P.col_pos.size()))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    {
        void *sp = nullptr;
        HIPCHK(c, scratch_address(&sp));
        c->scratch = static_cast<char *>(sp);
    }
    if ((st = upload(c, L.mu0, c->mu0.data(), 8 * K))) return st;
    if ((st = upload(c, L.W0inv, c->W0inv.data(), 8 * K * K))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BMF_OK;
}

bmf_status bmf_init(const bmf_config *cfg, bmf_ctx **out) { return init_common(cfg, out, true); }
bmf_status bmf_init_host(const bmf_config *cfg, bmf_ctx **out) { return init_common(cfg, out, false); }

bmf_status bmf_free(bmf_ctx *c) {
    if (!c) return BMF_OK;
    if (c->device) {
        hipStreamSynchronize(c->stream);
        for (auto &p : c->pending) {
            hipEventDestroy(p.a);
            hipEventDestroy(p.b);
        }
        drop_graph(c);
        if (c->cap_stream) hipStreamDestroy(c->cap_stream);
        if (c->own && c->base) hipFree(c->base);
    }
    delete c;
    return BMF_OK;
}

bmf_status bmf_gibbs_sweep(bmf_ctx *c, int32_t nsweeps) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (nsweeps < 0) return fail(c, BMF_EINVAL, "nsweeps < 0");
    bmf_status st;
    if (c->stage == 0 && (st = begin_stage(c, 1))) return st;
    if (c->finalized >= c->stage) c->finalized = c->stage - 1;   // more samples: redo MM later
    return run_sweeps(c, nsweeps);
}

bmf_status bmf_pp_stage(bmf_ctx *c, int32_t stage, int32_t nsweeps) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (stage < 1 || stage > 3 || nsweeps < 0) return fail(c, BMF_EINVAL, "bad stage or nsweeps");
    if (!stage_has_blocks(c, stage)) return BMF_OK;
    int32_t prev = 0;
    for (int32_t q = stage - 1; q >= 1; --q)
        if (stage_has_blocks(c, q)) { prev = q; break; }
    if (c->stage != prev && !(stage == 1 && c->stage == 0))
        return fail(c, BMF_ESTATE, "stages must be run in order");
    if (prev > 0) {
        bmf_status st = finalize_stage(c);
        if (st) return st;
        if (c->done_stages[prev] < 2)
            return fail(c, BMF_ESTATE, "propagation needs at least 2 kept samples per block");
    }
    bmf_status st = begin_stage(c, stage);
    if (st) return st;
    return run_sweeps(c, nsweeps);
}

bmf_status bmf_aggregate(bmf_ctx *c) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (c->agg_valid) return BMF_OK;
    if (c->stage != last_stage(c)) return fail(c, BMF_ESTATE, "every PP stage must be run before aggregation");
    bmf_status st = finalize_stage(c);
    if (st) return st;
    const Layout &L = c->L;
    const Plan &P = c->plan;
    const int32_t I = P.I, J = P.J;
    if ((I > 1 || J > 1))
        for (int32_t s = 1; s <= 3; ++s)
            if (stage_has_blocks(c, s) && c->done_stages[s] < 2)
                return fail(c, BMF_ESTATE, "aggregation needs at least 2 kept samples per block");
    double *mm = c->dev<double>(L.mm);
    for (int side = 0; side < 2; ++side) {
        std::vector<AggJob> jobs;
        std::vector<int2> items;
        const int32_t nparts = side == 0 ? I : J;
        for (int32_t p = 0; p < nparts; ++p) {
            AggJob jb{};
            if (side == 0) {
                jb.base = mm + c->x_off[p * J + 0] * L.prow;
                for (int32_t j = 1; j < J; ++j) jb.sib[j - 1] = mm + c->x_off[p * J + j] * L.prow;
                jb.nsib = J - 1;
                jb.n = (int32_t)P.R[p];
                jb.out_off = (int64_t)p * P.bs_r;
            } else {
                jb.base = mm + (L.E_r + c->w_off[0 * J + p]) * L.prow;
                for (int32_t i = 1; i < I; ++i) jb.sib[i - 1] = mm + (L.E_r + c->w_off[i * J + p]) * L.prow;
                jb.nsib = I - 1;
                jb.n = (int32_t)P.C[p];
                jb.out_off = (int64_t)p * P.bs_c;
            }
            for (int32_t n = 0; n < jb.n; ++n) items.push_back(make_int2(p, n));
            jobs.push_back(jb);
        }
        if ((st = upload(c, L.m_agg_jobs, jobs.data(), jobs.size() * sizeof(AggJob)))) return st;
        if ((st = upload(c, L.m_agg_items, items.data(), items.size() * sizeof(int2)))) return st;
        AggArgs a{};
        a.jobs = c->dev<AggJob>(L.m_agg_jobs);
        a.items = c->dev<int2>(L.m_agg_items);
        a.nitems = (int32_t)items.size();
        a.K = c->cfg.K;
        a.prow = L.prow;
        a.out = c->dev<double>(side == 0 ? L.agg_x : L.agg_w);
        a.corrections = c->dev<int32_t>(L.counters) + kCorr;
        if ((st = timed(c, kKAgg, [&] { return launch_agg(a, c->ls); }))) return st;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->agg_valid = true;
    return BMF_OK;
}

bmf_status bmf_predict(bmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col, float *out) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (n < 0 || (n > 0 && (!row || !col || !out))) return fail(c, BMF_EINVAL, "bad prediction arrays");
    bmf_status st = bmf_aggregate(c);
    if (st) return st;
    const Layout &L = c->L;
    const Plan &P = c->plan;
    std::vector<int64_t> xs, ws;
    for (int64_t a = 0; a < n; a += kPredictChunk) {
        const int64_t m = std::min(kPredictChunk, n - a);
        xs.resize(m);
        ws.resize(m);
        for (int64_t q = 0; q < m; ++q) {
            const int64_t r = row[a + q], cc = col[a + q];
            if (r < 0 || r >= P.N || cc < 0 || cc >= P.D) return fail(c, BMF_EINVAL, "prediction id out of range");
            xs[q] = P.row_pos[r];
            ws[q] = P.col_pos[cc];
        }
        if ((st = upload(c, L.p_xslot, xs.data(), 8 * m))) return st;
        if ((st = upload(c, L.p_wslot, ws.data(), 8 * m))) return st;
        PredictArgs pa{c->dev<int64_t>(L.p_xslot), c->dev<int64_t>(L.p_wslot), m, c->dev<double>(L.agg_x),
                       c->dev<double>(L.agg_w), c->cfg.K, c->ybar, c->dev<float>(L.p_out)};
        if ((st = timed(c, kKPredict, [&] { return launch_predict(pa, c->ls); }))) return st;
        HIPCHK(c, hipMemcpyAsync(out + a, c->base + L.p_out, 4 * m, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return BMF_OK;
}

bmf_status bmf_predict_noalloc(bmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col, float *out) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (n < 0 || (n > 0 && (!row || !col || !out))) return fail(c, BMF_EINVAL, "bad prediction arrays");
    if (n > kNoallocMaxPairs)
        return fail(c, BMF_EINVAL, "bmf_predict_noalloc takes at most 1048576 pairs per call (its staging "
                                   "array is fixed); split the request");
    if (!c->agg_valid)
        return fail(c, BMF_ESTATE, "bmf_predict_noalloc needs the aggregated means: call bmf_aggregate first");
    const Plan &P = c->plan;
    for (int64_t q = 0; q < n; ++q)
        if (row[q] < 0 || row[q] >= P.N || col[q] < 0 || col[q] >= P.D)
            return fail(c, BMF_EINVAL, "prediction id out of range");
    if (n == 0) return BMF_OK;
    // staging: [row ids | column ids | outputs], kNoallocMaxPairs entries each
    int32_t *srow = reinterpret_cast<int32_t *>(c->scratch);
    int32_t *scol = srow + kNoallocMaxPairs;
    float *sout = reinterpret_cast<float *>(scol + kNoallocMaxPairs);
    const Layout &L = c->L;
    HIPCHK(c, hipMemcpyAsync(srow, row, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(scol, col, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    PredictIdsArgs pa{srow, scol, n, c->dev<int64_t>(L.rowpos), c->dev<int64_t>(L.colpos), c->dev<double>(L.agg_x),
                      c->dev<double>(L.agg_w), c->cfg.K, c->ybar, sout};
    bmf_status st = timed(c, kKPredict, [&] { return launch_predict_ids(pa, c->ls); });
    if (st) return st;
    HIPCHK(c, hipMemcpyAsync(out, sout, 4 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BMF_OK;
}

bmf_status bmf_block_info(const bmf_ctx *c, int32_t b, int64_t *R, int64_t *C, int64_t *M, int32_t *stage) {
    if (!c || b < 0 || b >= (int32_t)c->plan.blocks.size()) return BMF_EINVAL;
    const PlanBlock &B = c->plan.blocks[b];
    if (R) *R = B.R;
    if (C) *C = B.C;
    if (M) *M = B.M;
    if (stage) *stage = B.stage;
    return BMF_OK;
}

bmf_status bmf_global_mean(const bmf_ctx *c, double *ybar) {
    if (!c || !ybar) return BMF_EINVAL;
    *ybar = c->ybar;
    return BMF_OK;
}

bmf_status bmf_get_positions(const bmf_ctx *c, int64_t *pos_row, int64_t *pos_col) {
    if (!c) return BMF_EINVAL;
    if (pos_row) std::copy(c->plan.row_pos.begin(), c->plan.row_pos.end(), pos_row);
    if (pos_col) std::copy(c->plan.col_pos.begin(), c->plan.col_pos.end(), pos_col);
    return BMF_OK;
}

bmf_status bmf_get_block_csr(const bmf_ctx *c, int32_t b, int32_t which, int64_t *ptr, int32_t *idx,
                             int64_t *entry) {
    if (!c || b < 0 || b >= (int32_t)c->plan.blocks.size() || which < 0 || which > 1) return BMF_EINVAL;
    const PlanBlock &B = c->plan.blocks[b];
    const std::vector<int64_t> &p = which == 0 ? B.csr_ptr : B.csc_ptr;
    if (ptr) std::copy(p.begin(), p.end(), ptr);
    if (c->device && !c->cfg.plan_on_host) {
        // the device planner keeps the local ids and entries on the device only
        const Layout &L = c->L;
        const int64_t e0 = c->nz_off[which][b];
        if (idx && B.M > 0 && hipMemcpy(idx, c->base + (which == 0 ? L.csr_idx : L.csc_idx) + 4 * e0, 4 * B.M,
                                        hipMemcpyDeviceToHost) != hipSuccess)
            return BMF_EDEVICE;
        if (entry && B.M > 0) {
            std::vector<int32_t> ent((size_t)B.M);
            if (hipMemcpy(ent.data(), c->base + (which == 0 ? L.csr_ent : L.csc_ent) + 4 * e0, 4 * B.M,
                          hipMemcpyDeviceToHost) != hipSuccess)
                return BMF_EDEVICE;
            std::copy(ent.begin(), ent.end(), entry);
        }
        return BMF_OK;
    }
    const std::vector<int32_t> &i = which == 0 ? B.csr_idx : B.csc_idx;
    const std::vector<int64_t> &e = which == 0 ? B.csr_entry : B.csc_entry;
    if (idx) std::copy(i.begin(), i.end(), idx);
    if (entry) std::copy(e.begin(), e.end(), entry);
    return BMF_OK;
}

// Host conversions between FP64 and the state element type (FP64, FP32, BF16).
static double state_to_double(const bmf_ctx *c, const char *buf, int64_t i) {
    if (c->fp64()) return reinterpret_cast<const double *>(buf)[i];
    if (!c->bf()) return (double)reinterpret_cast<const float *>(buf)[i];
    const uint32_t u = (uint32_t)reinterpret_cast<const uint16_t *>(buf)[i] << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

static void double_to_state(const bmf_ctx *c, char *buf, int64_t i, double v) {
    if (c->fp64()) {
        reinterpret_cast<double *>(buf)[i] = v;
    } else if (!c->bf()) {
        reinterpret_cast<float *>(buf)[i] = (float)v;
    } else {
        const float f = (float)v;
        uint32_t u;
        std::memcpy(&u, &f, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
        reinterpret_cast<uint16_t *>(buf)[i] = (uint16_t)(u >> 16);
    }
}

static int32_t stage_index(const bmf_ctx *c, int32_t b) {
    for (size_t k = 0; k < c->S.blocks.size(); ++k)
        if (c->S.blocks[k] == b) return (int32_t)k;
    return -1;
}

bmf_status bmf_get_state(bmf_ctx *c, int32_t b, double *X, double *W, double *hyper, double *tau) {
    if (!c) return BMF_EINVAL;
    if (!c->device || c->stage == 0) return fail(c, BMF_ESTATE, "no active stage");
    if (stage_index(c, b) < 0) return fail(c, BMF_EINVAL, "block is not in the active stage");
    const Layout &L = c->L;
    const PlanBlock &B = c->plan.blocks[b];
    const int32_t K = c->cfg.K;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int side = 0; side < 2; ++side) {
        double *dst = side == 0 ? X : W;
        if (!dst) continue;
        const int64_t n = side == 0 ? B.R : B.C;
        const int64_t off = side == 0 ? c->x_off[b] : c->w_off[b];
        const int64_t arr = side == 0 ? L.X : L.W;
        std::vector<char> buf((size_t)(n * L.ks_m * L.ss));
        HIPCHK(c, hipMemcpy(buf.data(), c->base + arr + off * L.ks_m * L.ss, buf.size(), hipMemcpyDeviceToHost));
        for (int64_t r = 0; r < n; ++r)
            for (int k = 0; k < K; ++k) dst[r * K + k] = state_to_double(c, buf.data(), r * L.ks_m + k);
    }
    if (hyper) {
        std::vector<double> h(2 * L.hy);
        HIPCHK(c, hipMemcpy(h.data(), c->base + L.hyper + (int64_t)b * 2 * L.hy * 8, 16 * L.hy, hipMemcpyDeviceToHost));
        for (int side = 0; side < 2; ++side) {
            std::copy(h.begin() + side * L.hy, h.begin() + side * L.hy + K * K, hyper + side * (K * K + K));
            std::copy(h.begin() + side * L.hy + K * K, h.begin() + side * L.hy + K * K + K,
                      hyper + side * (K * K + K) + K * K);
        }
    }
    if (tau) HIPCHK(c, hipMemcpy(tau, c->base + L.tau + 8 * (int64_t)b, 8, hipMemcpyDeviceToHost));
    return BMF_OK;
}

bmf_status bmf_set_state(bmf_ctx *c, int32_t b, const double *X, const double *W, const double *hyper,
                         const double *tau) {
    if (!c) return BMF_EINVAL;
    if (!c->device || c->stage == 0) return fail(c, BMF_ESTATE, "no active stage");
    if (stage_index(c, b) < 0) return fail(c, BMF_EINVAL, "block is not in the active stage");
    const Layout &L = c->L;
    const PlanBlock &B = c->plan.blocks[b];
    const int32_t K = c->cfg.K;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int side = 0; side < 2; ++side) {
        const double *src = side == 0 ? X : W;
        if (!src) continue;
        const int64_t n = side == 0 ? B.R : B.C;
        const int64_t off = side == 0 ? c->x_off[b] : c->w_off[b];
        std::vector<char> buf((size_t)(n * L.ks_m * L.ss), 0);
        for (int64_t r = 0; r < n; ++r)
            for (int k = 0; k < K; ++k) double_to_state(c, buf.data(), r * L.ks_m + k, src[r * K + k]);
        HIPCHK(c, hipMemcpy(c->base + (side == 0 ? L.X : L.W) + off * L.ks_m * L.ss, buf.data(), buf.size(),
                            hipMemcpyHostToDevice));
    }
    if (hyper) {
        std::vector<double> h(2 * L.hy, 0.0);
        for (int side = 0; side < 2; ++side) {
            const double *Lam = hyper + side * (K * K + K);
            const double *mu = Lam + K * K;
            std::copy(Lam, Lam + K * K, h.begin() + side * L.hy);
            std::copy(mu, mu + K, h.begin() + side * L.hy + K * K);
            double *pk = h.data() + side * L.hy + kHyPacked(L);
            for (int a = 0; a < K; ++a) {
                double s = 0.0;
                for (int q = 0; q < K; ++q) s += Lam[a * K + q] * mu[q];
                h[side * L.hy + K * K + K + a] = s;
                pk[K * (K + 1) / 2 + a] = s;
                pk[K * (K + 1) / 2 + K + a] = mu[a];
                for (int q = 0; q <= a; ++q) pk[a * (a + 1) / 2 + q] = Lam[a * K + q];
            }
        }
        HIPCHK(c, hipMemcpy(c->base + L.hyper + (int64_t)b * 2 * L.hy * 8, h.data(), 16 * L.hy, hipMemcpyHostToDevice));
    }
    if (tau) HIPCHK(c, hipMemcpy(c->base + L.tau + 8 * (int64_t)b, tau, 8, hipMemcpyHostToDevice));
    c->agg_valid = false;
    return BMF_OK;
}

bmf_status bmf_step(bmf_ctx *c, int32_t b, int32_t which, int64_t t) {
    if (!c) return BMF_EINVAL;
    if (!c->device || c->stage == 0) return fail(c, BMF_ESTATE, "no active stage");
    const int32_t k = stage_index(c, b);
    if (k < 0) return fail(c, BMF_EINVAL, "block is not in the active stage");
    if (t < 0 || t > 0xFFFFFFFELL) return fail(c, BMF_EINVAL, "bad sweep index");
    const uint32_t tt = (uint32_t)t;
    StageLists &S = c->S;
    const int32_t nbs = (int32_t)S.blocks.size();
    bmf_status st;
    // mixture priors follow the current state, as at the start of a sweep;
    // per-column precisions: the row pass's scaled copies of W and the values
    if ((which == 0 || which == 1) && (st = run_gmm_pick(c, false))) return st;
    if (which == 0 && (st = run_tau_scale(c, k))) return st;
    switch (which) {
    case 0: st = run_pass(c, true, tt, c->base + c->L.probe, k, false); break;
    case 1: st = run_pass(c, false, tt, c->base + c->L.probe, k, false); break;
    case 2:
    case 3: {
        const int32_t side = which == 2 ? k : nbs + k;
        if (S.sides[side].per_row) return fail(c, BMF_ESTATE, "side is propagated: no Normal-Wishart draw");
        if ((st = run_stats(c, side, side + 1))) return st;
        int32_t j = -1;
        for (int32_t q = S.hyper_begin[k]; q < S.hyper_begin[k + 1]; ++q)
            if (S.hyper_kind[q] == which - 2) j = q;
        st = run_hyper(c, j, j + 1, tt, false);
        break;
    }
    case 4: {
        if (!c->cfg.sample_tau) return fail(c, BMF_ESTATE, "tau is fixed");
        if ((st = run_sse(c, k))) return st;
        if (c->cfg.tau_per_column) {
            st = run_tau_cols(c, k, tt, false);
            break;
        }
        int32_t j = -1;
        for (int32_t q = S.hyper_begin[k]; q < S.hyper_begin[k + 1]; ++q)
            if (S.hyper_kind[q] == 2) j = q;
        st = run_hyper(c, j, j + 1, tt, false);
        break;
    }
    default: return fail(c, BMF_EINVAL, "bad step kind");
    }
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->agg_valid = false;
    return BMF_OK;
}

bmf_status bmf_get_draw(bmf_ctx *c, int32_t b, int32_t side, double *x) {
    if (!c || !x || side < 0 || side > 1) return BMF_EINVAL;
    if (!c->device || c->stage == 0) return fail(c, BMF_ESTATE, "no active stage");
    const int32_t k = stage_index(c, b);
    if (k < 0) return fail(c, BMF_EINVAL, "block is not in the active stage");
    const Layout &L = c->L;
    const int32_t nbs = (int32_t)c->S.blocks.size();
    const SideDesc &sd = c->S.sides[side == 0 ? k : nbs + k];
    const int32_t K = c->cfg.K;
    std::vector<char> buf((size_t)((int64_t)sd.n * L.ks_p * L.sp));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(buf.data(), c->base + L.probe + sd.sample_off * L.ks_p * L.sp, buf.size(),
                        hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < sd.n; ++r)
        for (int q = 0; q < K; ++q)
            x[r * K + q] = c->fp64() ? reinterpret_cast<double *>(buf.data())[r * L.ks_p + q]
                                     : (double)reinterpret_cast<float *>(buf.data())[r * L.ks_p + q];
    return BMF_OK;
}

bmf_status bmf_get_mm(bmf_ctx *c, int32_t b, int32_t side, double *mu, double *Lam) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (b < 0 || b >= (int32_t)c->plan.blocks.size() || side < 0 || side > 1) return fail(c, BMF_EINVAL, "bad block");
    const PlanBlock &B = c->plan.blocks[b];
    if (c->finalized < B.stage) {
        if (c->stage == B.stage) {
            bmf_status st = finalize_stage(c);
            if (st) return st;
        } else {
            return fail(c, BMF_ESTATE, "the block's stage has not been run");
        }
    }
    const Layout &L = c->L;
    const int32_t K = c->cfg.K;
    const int64_t n = side == 0 ? B.R : B.C;
    const int64_t row0 = side == 0 ? c->x_off[b] : L.E_r + c->w_off[b];
    std::vector<double> buf((size_t)(n * L.prow));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(buf.data(), c->base + L.mm + row0 * L.prow * 8, buf.size() * 8, hipMemcpyDeviceToHost));
    const int32_t kk2 = K * (K + 1) / 2;
    for (int64_t r = 0; r < n; ++r) {
        const double *row = buf.data() + r * L.prow;
        if (mu)
            for (int k = 0; k < K; ++k) mu[r * K + k] = row[kk2 + K + k];
        if (Lam) {
            int q = 0;
            for (int a = 0; a < K; ++a)
                for (int bb = 0; bb <= a; ++bb, ++q) {
                    Lam[(r * K + a) * K + bb] = row[q];
                    Lam[(r * K + bb) * K + a] = row[q];
                }
        }
    }
    return BMF_OK;
}

bmf_status bmf_get_clusters(bmf_ctx *c, int32_t b, int32_t side, int32_t *labels) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (c->cfg.approx == BMF_APPROX_MM) return fail(c, BMF_ESTATE, "moment matching keeps no clusters");
    if (b < 0 || b >= (int32_t)c->plan.blocks.size() || (side != 0 && side != 1) || !labels)
        return fail(c, BMF_EINVAL, "bad block, side or output");
    const PlanBlock &B = c->plan.blocks[b];
    if (B.stage > c->finalized) return fail(c, BMF_ESTATE, "the block's stage is not finalised");
    const int32_t S = c->done_stages[B.stage];
    const int64_t n = side == 0 ? B.R : B.C;
    const int64_t e = side == 0 ? c->x_off[b] : c->L.E_r + c->w_off[b];
    std::vector<uint8_t> buf((size_t)(n * c->cfg.max_kept));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(buf.data(), c->base + c->L.lab + e * c->cfg.max_kept, buf.size(), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < n; ++r)
        for (int32_t q = 0; q < S; ++q) labels[r * S + q] = buf[(size_t)(r * c->cfg.max_kept + q)];
    return BMF_OK;
}

bmf_status bmf_get_component(bmf_ctx *c, int32_t b, int32_t side, int32_t comp, double *pi, double *mu,
                             double *Lam, double *logdet) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    if (c->cfg.approx == BMF_APPROX_MM) return fail(c, BMF_ESTATE, "moment matching keeps no components");
    const Layout &L = c->L;
    if (b < 0 || b >= (int32_t)c->plan.blocks.size() || (side != 0 && side != 1) || comp < 0 || comp >= L.ncomp)
        return fail(c, BMF_EINVAL, "bad block, side or component");
    const PlanBlock &B = c->plan.blocks[b];
    if (B.stage > c->finalized) return fail(c, BMF_ESTATE, "the block's stage is not finalised");
    const int32_t K = c->cfg.K, kk2 = K * (K + 1) / 2;
    const int64_t n = side == 0 ? B.R : B.C;
    const int64_t e = side == 0 ? c->x_off[b] : L.E_r + c->w_off[b];
    const int64_t Etot = L.E_r + L.E_c;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> ax((size_t)(2 * n));
    HIPCHK(c, hipMemcpy(ax.data(), c->base + L.aux + (comp * Etot + e) * 2 * 8, ax.size() * 8, hipMemcpyDeviceToHost));
    // the component's rows: the mixture planes, or (dominant mode) the fitted rows themselves
    const int64_t roff = c->cfg.approx == BMF_APPROX_GMM ? L.gmm + (comp * Etot + e) * L.prow * 8 : L.mm + e * L.prow * 8;
    std::vector<double> rows((size_t)(n * L.prow));
    HIPCHK(c, hipMemcpy(rows.data(), c->base + roff, rows.size() * 8, hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < n; ++r) {
        const double *row = rows.data() + r * L.prow;
        if (pi) pi[r] = ax[(size_t)(2 * r)];
        if (logdet) logdet[r] = ax[(size_t)(2 * r + 1)];
        if (mu)
            for (int k = 0; k < K; ++k) mu[r * K + k] = row[kk2 + K + k];
        if (Lam)
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) Lam[(r * K + i) * K + j] = row[i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i];
    }
    return BMF_OK;
}

bmf_status bmf_get_tau_cols(bmf_ctx *c, int32_t b, double *tau) {
    if (!c) return BMF_EINVAL;
    if (!c->device || c->stage == 0) return fail(c, BMF_ESTATE, "no active stage");
    if (!c->cfg.tau_per_column) return fail(c, BMF_ESTATE, "the noise precision is one per block");
    if (stage_index(c, b) < 0) return fail(c, BMF_EINVAL, "block is not in the active stage");
    if (!tau) return fail(c, BMF_EINVAL, "null output");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(tau, c->base + c->L.tau_col + 8 * c->w_off[b], 8 * (size_t)c->plan.blocks[b].C,
                        hipMemcpyDeviceToHost));
    return BMF_OK;
}

bmf_status bmf_get_aggregate(bmf_ctx *c, int32_t side, double *mu) {
    if (!c || !mu || side < 0 || side > 1) return BMF_EINVAL;
    bmf_status st = bmf_aggregate(c);
    if (st) return st;
    const Layout &L = c->L;
    const Plan &P = c->plan;
    const int32_t K = c->cfg.K;
    const int64_t n = side == 0 ? P.N : P.D;
    std::vector<double> buf((size_t)(n * K));
    HIPCHK(c, hipMemcpy(buf.data(), c->base + (side == 0 ? L.agg_x : L.agg_w), buf.size() * 8, hipMemcpyDeviceToHost));
    const std::vector<int64_t> &pos = side == 0 ? P.row_pos : P.col_pos;
    for (int64_t r = 0; r < n; ++r)
        for (int k = 0; k < K; ++k) mu[r * K + k] = buf[pos[r] * K + k];
    return BMF_OK;
}

bmf_status bmf_get_stats(bmf_ctx *c, int64_t *fallback_rows, int64_t *nonpd_rows, int64_t *mm_ridged,
                         int64_t *agg_corrections, double *train_sse) {
    if (!c) return BMF_EINVAL;
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    int32_t h[kNumCounters];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(h, c->base + c->L.counters, sizeof(h), hipMemcpyDeviceToHost));
    if (train_sse) {
        *train_sse = 0.0;
        const size_t nbs = c->stage > 0 ? c->S.blocks.size() : 0;
        if (nbs > 0) {
            std::vector<double> v(nbs);
            HIPCHK(c, hipMemcpy(v.data(), c->base + c->L.sse_final, 8 * nbs, hipMemcpyDeviceToHost));
            for (double x : v) *train_sse += x;
        }
    }
    if (fallback_rows) *fallback_rows = h[kFbTotal];
    if (nonpd_rows) *nonpd_rows = h[kNonPD];
    if (mm_ridged) *mm_ridged = h[kRidged];
    if (agg_corrections) *agg_corrections = h[kCorr];
    return BMF_OK;
}

bmf_status bmf_enable_timing(bmf_ctx *c, int32_t on) {
    if (!c) return BMF_EINVAL;
    c->timing = on != 0;
    return BMF_OK;
}

bmf_status bmf_kernel_times(bmf_ctx *c, int32_t n, const char **names, int64_t *launches, double *ms,
                            int32_t *count) {
    if (!c) return BMF_EINVAL;
    if (c->device) HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float e = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&e, p.a, p.b));
        c->tlaunch[p.k] += 1;
        c->tms[p.k] += e;
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    c->pending.clear();
    for (int32_t k = 0; k < kNumK && k < n; ++k) {
        if (names) names[k] = kKNames[k];
        if (launches) launches[k] = c->tlaunch[k];
        if (ms) ms[k] = c->tms[k];
    }
    if (count) *count = kNumK;
    return BMF_OK;
}

bmf_status bmf_get_schedule(const bmf_ctx *c, int32_t *lane_nnz_rows, int32_t *lane_nnz_cols) {
    if (!c) return BMF_EINVAL;
    if (lane_nnz_rows) *lane_nnz_rows = c->S.lane_row;
    if (lane_nnz_cols) *lane_nnz_cols = c->S.lane_col;
    return BMF_OK;
}

bmf_status bmf_stage_work(const bmf_ctx *c, int64_t *row_updates, int64_t *ratings) {
    if (!c) return BMF_EINVAL;
    if (row_updates) *row_updates = c->S.row_updates;
    if (ratings) *ratings = c->S.ratings;
    return BMF_OK;
}

bmf_status bmf_get_sample(bmf_ctx *c, int32_t b, int32_t side, int32_t slot, double *x) {
    if (!c || !x || side < 0 || side > 1) return BMF_EINVAL;
    if (!c->device || c->stage == 0) return fail(c, BMF_ESTATE, "no active stage");
    const int32_t k = stage_index(c, b);
    if (k < 0) return fail(c, BMF_EINVAL, "block is not in the active stage");
    if (slot < 0 || slot >= c->kept) return fail(c, BMF_EINVAL, "sample slot not written in this stage");
    const Layout &L = c->L;
    const int32_t nbs = (int32_t)c->S.blocks.size();
    const SideDesc &sd = c->S.sides[side == 0 ? k : nbs + k];
    const int32_t K = c->cfg.K;
    const int64_t slot_bytes = L.Emax * L.ks_p * L.sp;
    std::vector<char> buf((size_t)((int64_t)sd.n * L.ks_p * L.sp));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(buf.data(), c->base + L.sample + slot * slot_bytes + sd.sample_off * L.ks_p * L.sp,
                        buf.size(), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < sd.n; ++r)
        for (int q = 0; q < K; ++q)
            x[r * K + q] = c->fp64() ? reinterpret_cast<double *>(buf.data())[r * L.ks_p + q]
                                     : (double)reinterpret_cast<float *>(buf.data())[r * L.ks_p + q];
    return BMF_OK;
}

bmf_status bmf_set_progress(bmf_ctx *c, bmf_progress_fn fn, void *user) {
    if (!c) return BMF_EINVAL;
    c->progress = fn;
    c->progress_user = user;
    return BMF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// checkpoint files
// ---------------------------------------------------------------------------
namespace {

constexpr char kCkptMagic[8] = {'B', 'M', 'F', 'C', 'K', 'P', 'T', 0};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    int64_t N, D, nnz;
    int32_t K, I, J, order, precision, max_kept;
    uint64_t seed, fingerprint;
    // layout the arrays were written with
    int64_t Emax, ks_m, ss, ks_p, sp, prow, pfrow, hy;
    // stage bookkeeping
    int32_t stage, finalized, kept, lane_row, lane_col, done[4], pad;
    int64_t t;
};

CkptHeader header_of(const bmf_ctx *c) {
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.header_bytes = (uint32_t)sizeof(CkptHeader);
    h.N = c->cfg.N;
    h.D = c->cfg.D;
    h.nnz = c->cfg.nnz;
    h.K = c->cfg.K;
    h.I = c->cfg.I;
    h.J = c->cfg.J;
    h.order = c->cfg.order;
    h.precision = c->cfg.precision;
    h.max_kept = c->cfg.max_kept;
    h.seed = c->cfg.seed;
    h.fingerprint = c->fingerprint;
    h.Emax = c->L.Emax;
    h.ks_m = c->L.ks_m;
    h.ss = c->L.ss;
    h.ks_p = c->L.ks_p;
    h.sp = c->L.sp;
    h.prow = c->L.prow;
    h.pfrow = c->L.pfrow;
    h.hy = c->L.hy;
    return h;
}

// One device byte range, written to or read from the file through a host buffer.
struct Span {
    int64_t off, bytes;
};

// Every device range a checkpoint holds, in file order: counters, sweep state;
// for the active stage per block the X and W rows, the hyperparameter slots,
// tau and the last SSE, then its kept samples; the moment-matched rows of
// every finished stage's blocks; the prior factors.
std::vector<Span> ckpt_spans(const bmf_ctx *c, int32_t stage, int32_t finalized, int32_t kept) {
    const Layout &L = c->L;
    const Plan &P = c->plan;
    std::vector<Span> v;
    v.push_back({L.counters, 4 * (int64_t)kNumCounters});
    v.push_back({L.sweep, (int64_t)sizeof(SweepState)});
    if (stage > 0) {
        int64_t ents = 0;
        int32_t k = 0;
        for (int32_t b = 0; b < (int32_t)P.blocks.size(); ++b) {
            const PlanBlock &B = P.blocks[b];
            if (B.stage != stage) continue;
            v.push_back({L.X + c->x_off[b] * L.ks_m * L.ss, B.R * L.ks_m * L.ss});
            v.push_back({L.W + c->w_off[b] * L.ks_m * L.ss, B.C * L.ks_m * L.ss});
            v.push_back({L.hyper + (int64_t)b * 2 * L.hy * 8, 16 * (int64_t)L.hy});
            v.push_back({L.tau + 8 * (int64_t)b, 8});
            if (c->cfg.tau_per_column) v.push_back({L.tau_col + 8 * c->w_off[b], 8 * B.C});
            v.push_back({L.sse_final + 8 * (int64_t)k, 8});
            ents += B.R + B.C;
            ++k;
        }
        const int64_t slot_bytes = L.Emax * L.ks_p * L.sp;
        for (int32_t q = 0; q < kept; ++q) v.push_back({L.sample + q * slot_bytes, ents * L.ks_p * L.sp});
    }
    for (int32_t b = 0; b < (int32_t)P.blocks.size(); ++b) {
        const PlanBlock &B = P.blocks[b];
        if (B.stage > finalized) continue;
        v.push_back({L.mm + c->x_off[b] * L.prow * 8, B.R * L.prow * 8});
        v.push_back({L.mm + (L.E_r + c->w_off[b]) * L.prow * 8, B.C * L.prow * 8});
    }
    if (L.pfrow) v.push_back({L.pfac, 4 * (P.N + P.D) * (int64_t)L.pfrow});
    if (c->cfg.approx != BMF_APPROX_MM) {
        // the fits of finalised blocks: labels, (weight, log det) planes, mixture components
        const int64_t Etot = L.E_r + L.E_c;
        for (int32_t b = 0; b < (int32_t)P.blocks.size(); ++b) {
            const PlanBlock &B = P.blocks[b];
            if (B.stage > finalized) continue;
            const int64_t e[2] = {c->x_off[b], L.E_r + c->w_off[b]}, n[2] = {B.R, B.C};
            for (int sd = 0; sd < 2; ++sd) {
                v.push_back({L.lab + e[sd] * c->cfg.max_kept, n[sd] * c->cfg.max_kept});
                for (int32_t cc = 0; cc < L.ncomp; ++cc) {
                    v.push_back({L.aux + (cc * Etot + e[sd]) * 2 * 8, n[sd] * 2 * 8});
                    if (c->cfg.approx == BMF_APPROX_GMM)
                        v.push_back({L.gmm + (cc * Etot + e[sd]) * L.prow * 8, n[sd] * L.prow * 8});
                }
            }
        }
    }
    return v;
}

constexpr int64_t kCkptChunk = 64 << 20;

}  // namespace

extern "C" {

bmf_status bmf_save_state(bmf_ctx *c, const char *path) {
    if (!c) return BMF_EINVAL;
    if (!path) return fail(c, BMF_EINVAL, "null path");
    if (!c->device) return fail(c, BMF_ESTATE, "context has no device state");
    CkptHeader h = header_of(c);
    h.stage = c->stage;
    h.finalized = c->finalized;
    h.kept = c->kept;
    h.lane_row = c->S.lane_row;
    h.lane_col = c->S.lane_col;
    for (int q = 0; q < 4; ++q) h.done[q] = c->done_stages[q];
    h.t = c->t;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(c, BMF_EINVAL, std::string("cannot open ") + path + " for writing");
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
    std::vector<char> buf;
    for (const Span &sp : ckpt_spans(c, h.stage, h.finalized, h.kept)) {
        for (int64_t o = 0; ok && o < sp.bytes; o += kCkptChunk) {
            const int64_t n = std::min(kCkptChunk, sp.bytes - o);
            buf.resize((size_t)n);
            if (hipMemcpy(buf.data(), c->base + sp.off + o, (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
                std::fclose(f);
                return fail(c, BMF_EDEVICE, "device read for the checkpoint failed");
            }
            ok = std::fwrite(buf.data(), 1, (size_t)n, f) == (size_t)n;
        }
        if (!ok) break;
    }
    if (std::fclose(f) != 0) ok = false;
    if (!ok) return fail(c, BMF_EINVAL, std::string("write to ") + path + " failed");
    return BMF_OK;
}

bmf_status bmf_load_state(bmf_ctx *c, const char *path) {
    if (!c) return BMF_EINVAL;
    if (!path) return fail(c, BMF_EINVAL, "null path");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(c, BMF_EINVAL, std::string("cannot open ") + path);
    CkptHeader h{};
    const bool got = std::fread(&h, sizeof(h), 1, f) == 1;
    const CkptHeader want = header_of(c);
    std::string why;
    if (!got || std::memcmp(h.magic, kCkptMagic, 8) != 0) why = "not a checkpoint file";
    else if (h.version != kCkptVersion || h.header_bytes != sizeof(CkptHeader)) why = "checkpoint version differs";
    else if (h.N != want.N || h.D != want.D || h.nnz != want.nnz || h.K != want.K || h.I != want.I ||
             h.J != want.J || h.order != want.order || h.precision != want.precision ||
             h.max_kept != want.max_kept || h.seed != want.seed)
        why = "checkpoint was written for another configuration";
    else if (h.fingerprint != want.fingerprint) why = "checkpoint was written for other training data or settings";
    else if (h.Emax != want.Emax || h.ks_m != want.ks_m || h.ss != want.ss || h.ks_p != want.ks_p ||
             h.sp != want.sp || h.prow != want.prow || h.pfrow != want.pfrow || h.hy != want.hy)
        why = "checkpoint layout differs";
    else if (h.stage < 0 || h.stage > 3 || h.finalized < 0 || h.finalized > h.stage || h.kept < 0 ||
             h.kept > want.max_kept || h.t < 0 || (h.stage > 0 && !stage_has_blocks(c, h.stage)))
        why = "checkpoint bookkeeping is out of range";
    if (!why.empty()) {
        std::fclose(f);
        return fail(c, BMF_EINVAL, why + ": " + path);
    }
    if (!c->device) {
        std::fclose(f);
        return fail(c, BMF_ESTATE, "context has no device state");
    }
    bmf_status st = BMF_OK;
    drop_graph(c);
    c->stage = 0;
    c->agg_valid = false;
    if (h.stage > 0) {
        build_stage_lists(c, h.stage);
        if ((st = upload_stage(c)) == BMF_OK) {
            build_tiles(c, h.lane_row > 0 ? h.lane_row : 32, h.lane_col > 0 ? h.lane_col : 32);
            st = upload_tiles(c);
        }
        if (st) {
            std::fclose(f);
            return st;
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<char> buf;
    bool ok = true;
    for (const Span &sp : ckpt_spans(c, h.stage, h.finalized, h.kept)) {
        for (int64_t o = 0; ok && o < sp.bytes; o += kCkptChunk) {
            const int64_t n = std::min(kCkptChunk, sp.bytes - o);
            buf.resize((size_t)n);
            ok = std::fread(buf.data(), 1, (size_t)n, f) == (size_t)n;
            if (ok && hipMemcpy(c->base + sp.off + o, buf.data(), (size_t)n, hipMemcpyHostToDevice) != hipSuccess) {
                std::fclose(f);
                return fail(c, BMF_EDEVICE, "device write from the checkpoint failed");
            }
        }
        if (!ok) break;
    }
    std::fclose(f);
    if (!ok) return fail(c, BMF_EINVAL, std::string("checkpoint is truncated: ") + path);
    c->stage = h.stage;
    c->finalized = h.finalized;
    c->kept = h.kept;
    c->t = h.t;
    for (int q = 0; q < 4; ++q) c->done_stages[q] = h.done[q];
    return BMF_OK;
}

}  // extern "C"
