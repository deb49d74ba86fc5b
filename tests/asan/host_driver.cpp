// Exercises the host half of the library (configuration checks, ordering,
// partition, per-block CSR/CSC, workspace sizing, introspection of the plan)
// through bmf_init_host, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure: tests/test_sanitizers.py
// compiles and runs it).  No device call is made.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "bmf.h"

static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint64_t next() {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}

int main() {
    int failures = 0;
    const int64_t N = 211, D = 97;
    std::vector<int32_t> row, col;
    std::vector<float> val;
    for (int64_t r = 0; r < N; ++r)
        for (int64_t c = 0; c < D; ++c)
            if (r % 13 != 5 && next() % 100 < (uint64_t)(3 + 40 * (r % 4 == 0))) {
                row.push_back((int32_t)r);
                col.push_back((int32_t)c);
                val.push_back((float)(next() % 1000) / 250.0f - 2.0f);
            }
    for (int order = 0; order < 3; ++order)
        for (int IJ : {1, 2, 5, 7})
            for (int approx = 0; approx < 3; ++approx) {
                bmf_config c;
                bmf_config_defaults(&c);
                c.N = N;
                c.D = D;
                c.K = 6;
                c.nu0 = 6;
                c.nnz = (int64_t)row.size();
                c.row = row.data();
                c.col = col.data();
                c.val = val.data();
                c.I = IJ;
                c.J = IJ + (IJ > 1);
                c.order = order;
                c.max_kept = 9;
                c.approx = approx;
                size_t ws = 0;
                if (bmf_workspace_size(&c, &ws) != BMF_OK || ws == 0) ++failures;
                bmf_ctx *ctx = nullptr;
                if (bmf_init_host(&c, &ctx) != BMF_OK) {
                    std::printf("init failed: %s\n", bmf_last_error(ctx));
                    ++failures;
                    bmf_free(ctx);
                    continue;
                }
                std::vector<int64_t> pr(N), pc(D);
                if (bmf_get_positions(ctx, pr.data(), pc.data()) != BMF_OK) {
                    std::printf("positions failed: %s\n", bmf_last_error(ctx));
                    ++failures;
                }
                for (int32_t b = 0; b < c.I * c.J; ++b) {
                    int64_t R = 0, C = 0, M = 0;
                    int32_t s = 0;
                    if (bmf_block_info(ctx, b, &R, &C, &M, &s) != BMF_OK) {
                        std::printf("block_info %d failed: %s\n", b, bmf_last_error(ctx));
                        ++failures;
                    }
                    for (int which = 0; which < 2; ++which) {
                        std::vector<int64_t> ptr((which ? C : R) + 1), ent(M > 0 ? M : 1);
                        std::vector<int32_t> idx(M > 0 ? M : 1);
                        if (bmf_get_block_csr(ctx, b, which, ptr.data(), idx.data(), ent.data()) != BMF_OK) {
                            std::printf("block_csr %d failed: %s\n", b, bmf_last_error(ctx));
                            ++failures;
                        }
                    }
                }
                double ybar = 0.0;
                bmf_global_mean(ctx, &ybar);
                // device entry points must refuse a host context without touching memory
                if (bmf_gibbs_sweep(ctx, 1) == BMF_OK) ++failures;
                int32_t lab[4];
                if (bmf_get_clusters(ctx, 0, 0, lab) == BMF_OK) ++failures;
                bmf_free(ctx);
            }
    // refused configurations leave a readable message
    bmf_config bad;
    bmf_config_defaults(&bad);
    bad.N = 10;
    bad.D = 10;
    bad.K = 0;
    bmf_ctx *ctx = nullptr;
    if (bmf_init_host(&bad, &ctx) == BMF_OK) ++failures;
    std::printf("refused: %s\n", bmf_last_error(ctx));
    bmf_free(ctx);
    std::printf("host driver done, %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
