// Host planner: ordering, I x J partition and per-block CSR/CSC (exact integer
// work), plus the degree-sorted schedules the kernels run on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "bmf.h"

namespace bmf {

struct PlanBlock {
    int32_t i = 0, j = 0, stage = 0;
    int64_t R = 0, C = 0, M = 0;
    std::vector<int64_t> csr_ptr, csc_ptr;    // relative to the block, size R+1 / C+1
    std::vector<int32_t> csr_idx, csc_idx;    // local column / local row
    std::vector<int64_t> csr_entry, csc_entry;  // index into the caller's COO arrays
};

struct Plan {
    int64_t N = 0, D = 0;
    int32_t I = 1, J = 1;
    int64_t bs_r = 0, bs_c = 0;               // part sizes ceil(N/I), ceil(D/J)
    std::vector<int64_t> R, C;                // rows per row part, columns per column part
    std::vector<int64_t> row_pos, col_pos;    // position of each id in the chosen order
    std::vector<PlanBlock> blocks;            // b = i * J + j
};

// Stage of block (i, j), 0-based: 1 for (0,0), 2 with exactly one zero index,
// 3 otherwise (eq. stage1, stage2a/b, stage3).
inline int32_t stage_of(int32_t i, int32_t j) {
    if (i == 0 && j == 0) return 1;
    if (i == 0 || j == 0) return 2;
    return 3;
}

// Build the plan.  Returns BMF_OK or BMF_EINVAL with a message (ids out of
// range, duplicate cells, empty part).
bmf_status build_plan(const bmf_config &cfg, Plan &plan, std::string &err);

// The partition's part sizes (N, D, I, J, bs_r, bs_c, R, C of the plan), or
// BMF_EINVAL when a part would be empty.
bmf_status plan_partition(const bmf_config &cfg, Plan &plan, std::string &err);

// pos[e] for every entity: its position in the chosen order (Sec. 5.2), from
// the entities' observation counts.
std::vector<int64_t> make_positions(int64_t n, const std::vector<int64_t> &count, int32_t order, uint64_t seed,
                                    uint32_t purpose);

// Device outputs of the device planner, in the library's layout: global CSR
// and CSC pointer arrays (per block R+1 / C+1 entry offsets), local ids,
// centred values (FP64 or FP32), the COO entry of every sorted position, the
// per-column sums of squared values (W order) and the entities' positions.
struct GpuPlanDst {
    int64_t *csr_ptr, *csc_ptr;
    int32_t *csr_idx, *csc_idx;
    void *csr_val, *csc_val;
    int32_t *csr_ent, *csc_ent;
    double *colsq;
    int64_t *rowpos, *colpos;
};

// The plan with its per-entry work on the GPU (the same plan as build_plan,
// except that the blocks' csr_idx / csr_entry and csc_idx / csc_entry stay on
// the device).  Allocates and frees its own temporary device memory (about
// 40 bytes per entry); work is ordered on s.
bmf_status gpu_build_plan(const bmf_config &cfg, double ybar, bool fp64, Plan &plan, const GpuPlanDst &dst,
                          hipStream_t s, std::string &err);

// Entities of one block side sorted by decreasing degree (ties by local id).
std::vector<int32_t> degree_order(const std::vector<int64_t> &ptr);

}  // namespace bmf
