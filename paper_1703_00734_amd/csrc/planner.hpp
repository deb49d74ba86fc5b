// Host planner: ordering, I x J partition and per-block CSR/CSC (exact integer
// work), plus the degree-sorted schedules the kernels run on.
#pragma once

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

// Entities of one block side sorted by decreasing degree (ties by local id).
std::vector<int32_t> degree_order(const std::vector<int64_t> &ptr);

}  // namespace bmf
