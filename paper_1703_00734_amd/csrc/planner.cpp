// Host planner: ordering (Sec. 5.2), r x c partition (Sec. 3, Sec. 5.2) and the
// observed sets Omega_n / Omega_d of every block as CSR and CSC (Sec. 2.1,
// eq. BMF_likelihood).  All integer; results are exact and deterministic.
#include "planner.hpp"

#include <algorithm>
#include <numeric>

#include "common.hpp"

namespace bmf {

// pos[e] for every entity: its position in the chosen order.
std::vector<int64_t> make_positions(int64_t n, const std::vector<int64_t> &count, int32_t order,
                                    uint64_t seed, uint32_t purpose) {
    std::vector<int64_t> ids(n);
    std::iota(ids.begin(), ids.end(), 0);
    if (order == BMF_ORDER_RANDOM) {
        const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
        const uint32_t c2 = counter_word(0xFFFFFFu, purpose);
        std::vector<uint32_t> key(n);
        for (int64_t e = 0; e < n; ++e) {
            uint32_t o[4];
            philox4x32_10((uint32_t)e, 0u, c2, 0u, k0, k1, o);
            key[e] = o[0];
        }
        std::sort(ids.begin(), ids.end(), [&](int64_t a, int64_t b) {
            return key[a] != key[b] ? key[a] < key[b] : a < b;
        });
    } else if (order == BMF_ORDER_DECREASING) {
        std::sort(ids.begin(), ids.end(), [&](int64_t a, int64_t b) {
            return count[a] != count[b] ? count[a] > count[b] : a < b;
        });
    }
    std::vector<int64_t> pos(n);
    for (int64_t p = 0; p < n; ++p) pos[ids[p]] = p;
    return pos;
}

namespace {

// One stable counting-sort pass of `perm` by key[perm[k]] in [0, range).
void counting_pass(std::vector<int64_t> &perm, const std::vector<int64_t> &key, int64_t range) {
    std::vector<int64_t> start(range + 1, 0);
    for (int64_t e : perm) start[key[e] + 1] += 1;
    for (int64_t r = 0; r < range; ++r) start[r + 1] += start[r];
    std::vector<int64_t> out(perm.size());
    for (int64_t e : perm) out[start[key[e]]++] = e;
    perm.swap(out);
}

}  // namespace

std::vector<int32_t> degree_order(const std::vector<int64_t> &ptr) {
    const int64_t n = (int64_t)ptr.size() - 1;
    std::vector<int32_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return (ptr[a + 1] - ptr[a]) > (ptr[b + 1] - ptr[b]);
    });
    return ord;
}

bmf_status plan_partition(const bmf_config &cfg, Plan &p, std::string &err) {
    p = Plan();
    p.N = cfg.N;
    p.D = cfg.D;
    p.I = cfg.I;
    p.J = cfg.J;
    p.bs_r = (p.N + p.I - 1) / p.I;
    p.bs_c = (p.D + p.J - 1) / p.J;
    for (int32_t i = 0; i < p.I; ++i) p.R.push_back(std::min(p.bs_r, p.N - i * p.bs_r));
    for (int32_t j = 0; j < p.J; ++j) p.C.push_back(std::min(p.bs_c, p.D - j * p.bs_c));
    if (p.R.back() <= 0 || p.C.back() <= 0) {
        err = "partition leaves an empty part";
        return BMF_EINVAL;
    }
    return BMF_OK;
}

bmf_status build_plan(const bmf_config &cfg, Plan &p, std::string &err) {
    p = Plan();
    p.N = cfg.N;
    p.D = cfg.D;
    p.I = cfg.I;
    p.J = cfg.J;
    const int64_t nnz = cfg.nnz;
    std::vector<int64_t> rc(p.N, 0), cc(p.D, 0);
    for (int64_t e = 0; e < nnz; ++e) {
        const int64_t r = cfg.row[e], c = cfg.col[e];
        if (r < 0 || r >= p.N || c < 0 || c >= p.D) {
            err = "COO entry " + std::to_string(e) + " out of range";
            return BMF_EINVAL;
        }
        rc[r] += 1;
        cc[c] += 1;
    }
    {
        Plan q;
        const bmf_status st = plan_partition(cfg, q, err);
        if (st) return st;
        p.bs_r = q.bs_r;
        p.bs_c = q.bs_c;
        p.R = q.R;
        p.C = q.C;
    }
    p.row_pos = make_positions(p.N, rc, cfg.order, cfg.seed, kPermRow);
    p.col_pos = make_positions(p.D, cc, cfg.order, cfg.seed, kPermCol);

    // keys of every entry: block, local row, local column
    std::vector<int64_t> blk(nnz), lr(nnz), lc(nnz);
    for (int64_t e = 0; e < nnz; ++e) {
        const int64_t pr = p.row_pos[cfg.row[e]], pc = p.col_pos[cfg.col[e]];
        blk[e] = (pr / p.bs_r) * p.J + (pc / p.bs_c);
        lr[e] = pr % p.bs_r;
        lc[e] = pc % p.bs_c;
    }
    const int64_t nb = (int64_t)p.I * p.J;

    // CSR order: by (block, local row, local column) = LSD passes
    std::vector<int64_t> csr(nnz);
    std::iota(csr.begin(), csr.end(), 0);
    counting_pass(csr, lc, p.bs_c);
    {
        std::vector<int64_t> key(nnz);
        for (int64_t e = 0; e < nnz; ++e) key[e] = blk[e] * p.bs_r + lr[e];
        counting_pass(csr, key, nb * p.bs_r);
    }
    for (int64_t k = 1; k < nnz; ++k) {
        const int64_t a = csr[k - 1], b = csr[k];
        if (blk[a] == blk[b] && lr[a] == lr[b] && lc[a] == lc[b]) {
            err = "duplicate COO cell at entries " + std::to_string(a) + " and " +
                  std::to_string(b);
            return BMF_EINVAL;
        }
    }
    // CSC order: by (block, local column, local row)
    std::vector<int64_t> csc(nnz);
    std::iota(csc.begin(), csc.end(), 0);
    counting_pass(csc, lr, p.bs_r);
    {
        std::vector<int64_t> key(nnz);
        for (int64_t e = 0; e < nnz; ++e) key[e] = blk[e] * p.bs_c + lc[e];
        counting_pass(csc, key, nb * p.bs_c);
    }

    p.blocks.resize(nb);
    int64_t a = 0, c = 0;
    for (int64_t b = 0; b < nb; ++b) {
        PlanBlock &B = p.blocks[b];
        B.i = (int32_t)(b / p.J);
        B.j = (int32_t)(b % p.J);
        B.stage = stage_of(B.i, B.j);
        B.R = p.R[B.i];
        B.C = p.C[B.j];
        int64_t a_end = a;
        while (a_end < nnz && blk[csr[a_end]] == b) ++a_end;
        int64_t c_end = c;
        while (c_end < nnz && blk[csc[c_end]] == b) ++c_end;
        B.M = a_end - a;
        B.csr_ptr.assign(B.R + 1, 0);
        B.csc_ptr.assign(B.C + 1, 0);
        B.csr_idx.resize(B.M);
        B.csr_entry.resize(B.M);
        B.csc_idx.resize(B.M);
        B.csc_entry.resize(B.M);
        for (int64_t k = 0; k < B.M; ++k) {
            const int64_t e = csr[a + k];
            B.csr_ptr[lr[e] + 1] += 1;
            B.csr_idx[k] = (int32_t)lc[e];
            B.csr_entry[k] = e;
            const int64_t f = csc[c + k];
            B.csc_ptr[lc[f] + 1] += 1;
            B.csc_idx[k] = (int32_t)lr[f];
            B.csc_entry[k] = f;
        }
        for (int64_t r = 0; r < B.R; ++r) B.csr_ptr[r + 1] += B.csr_ptr[r];
        for (int64_t q = 0; q < B.C; ++q) B.csc_ptr[q + 1] += B.csc_ptr[q];
        a = a_end;
        c = c_end;
    }
    return BMF_OK;
}

}  // namespace bmf
