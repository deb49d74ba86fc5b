// Shared host/device definitions of the BMF library: work descriptors, the
// random-stream layout and Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmf {

// Purpose field of the Philox counter word c2 = (block << 8) | purpose.
enum Purpose : uint32_t {
    kInitX = 0, kInitW = 1, kRow = 2, kCol = 3, kHyperX = 4, kHyperW = 5, kTau = 6,
    kPermRow = 7, kPermCol = 8
};

__host__ __device__ inline uint32_t counter_word(uint32_t block, uint32_t purpose) {
    return ((block & 0xFFFFFFu) << 8) | purpose;
}

// Philox4x32-10: ten rounds of two 32x32->64 multiplies, key bumped by the Weyl
// constants between rounds.
__host__ __device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t k0, uint32_t k1,
                                              uint32_t out[4]) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// One side (rows or columns) of one block inside a launch.
struct SideDesc {
    int64_t ptr_off;     // entity 0 of this side in the global CSR/CSC pointer array
    int64_t self_off;    // entity 0 in the factor array being updated (rows of stride ks)
    int64_t other_off;   // entity 0 of the other side in the gathered factor array
    int64_t sample_off;  // entity 0 in one slot of the sample store
    const double *prior; // shared: [Lambda (K*K), mu (K), Lambda*mu (K)];
                         // per-row: moment-matched rows [Lambda packed, eta, mu]
    const double *tau;   // this block's noise precision, or (tau_stride 1) one per entity
    const float *pfac;   // per-row priors of FP32/BF16 passes: per entity the inverse
                         // factor of its prior precision (rows of stride pfrow), else null
    int32_t n;           // number of entities
    int32_t per_row;     // 0 shared prior, 1 propagated per-row prior
    uint32_t c2;         // Philox counter word of the conditional draws
    uint32_t c2_init;    // Philox counter word of the initial draws
    int32_t block;       // global block id b = i * J + j
    int32_t tau_stride;  // 0: tau[0] for every entity; 1: tau[n] (per-column precisions, column side)
};

// Per-column noise precisions of one block of a stage: the columns' tau_d,
// the row pass's scaled factors sqrt(tau_d) w_d and values sqrt(tau_d) r_nd.
struct TauColJob {
    int32_t block;
    int32_t C;           // columns
    int64_t w_off;       // first column in the W arrays (and in tau_col)
    int64_t cptr_off;    // first column in the global CSC pointer array
    int64_t e0, M;       // the block's CSR entries
};

// Device-side sweep bookkeeping read by every kernel of a sweep, so one
// captured graph serves every sweep of a stage.
struct SweepState {
    uint32_t t;          // sweep index within the stage (Philox c1)
    int32_t slot;        // sample slot of this sweep, -1 when it is not kept
    int32_t kept;        // samples kept so far in the stage
    int32_t burnin;
    int32_t thin;
    int32_t max_kept;
    int64_t slot_bytes;  // bytes per sample slot
};

// A workgroup's share of one pass: `count` entities of side `side`, taken from
// the degree-sorted order array at `start`, each handled by G lanes.
struct Tile {
    int32_t side;
    int32_t start;
    int32_t count;
    int32_t G;
};

// Fixed-order partial sums for the Normal-Wishart statistics of one side.
struct StatsJob {
    int32_t side;
    int32_t first;
    int32_t count;
    int32_t part;        // index of this job's partial sums
};

// Work of the hyperparameter kernel: a Normal-Wishart draw (kind 0 = X side,
// 1 = W side) or a tau draw (kind 2) for one block.
struct HyperJob {
    int32_t kind;
    int32_t block;       // global block id (Philox counter word)
    int32_t part_begin;  // partial sums to reduce, in order
    int32_t part_end;
    int64_t n;           // entities (NW) or training entries (tau)
    double *out;         // NW: [Lambda, mu, Lambda*mu]; tau: the tau slot
};

// Moment matching / initialisation work: entity range of one side.
struct SideRange {
    int32_t side;
    int32_t first;
    int32_t count;
    int32_t pad_;
};

// One segment of a heavy entity's observed entries [begin, end): its partial
// Gram and right-hand side go to partial slot `slot`.
struct SegItem {
    int32_t side;
    int32_t ent;
    int64_t begin;
    int64_t end;
    int32_t slot;
    int32_t pad_;
};

// Aggregation of one row (or column) block: base block and siblings.
struct AggJob {
    const double *base;          // moment-matched rows of the base block
    const double *sib[64];       // of each sibling (up to 64)
    int32_t nsib;
    int32_t n;                   // rows in the block
    int64_t out_off;             // first output row (original-id-independent slot)
};

}  // namespace bmf
