// Device planner: the per-entry half of the plan on the GPU.  The ordering of
// rows and columns (Sec. 5.2: given, random, decreasing number of
// observations) and the r x c partition (Sec. 3, Sec. 5.2) are the host
// planner's; every entry then gets its block, local row and local column, and
// the observed sets Omega_n / Omega_d of every block (Sec. 2.1, eq.
// BMF_likelihood) are laid out by one radix sort of a unique composite key per
// order: (block, local row, local column) for CSR, (block, local column, local
// row) for CSC.  The keys are unique (duplicate cells are an error), so the
// sorted order is the host planner's stable counting-sort order exactly.  The
// degree counts of rows, columns and of each block row and column are device
// atomics; everything else (positions, per-block pointers) is per-entity work
// left to the host.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <string>
#include <vector>

#include "common.hpp"
#include "planner.hpp"

namespace bmf {

namespace {

typedef unsigned long long ull;

__global__ __launch_bounds__(256) void k_plan_count(const int32_t *row, const int32_t *col, int64_t nnz, int64_t N,
                                                    int64_t D, ull *rc, ull *cc, ull *bad) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
        const int64_t r = row[e], c = col[e];
        if (r < 0 || r >= N || c < 0 || c >= D) {
            atomicMin(bad, (ull)e);
        } else {
            atomicAdd(rc + r, 1ull);
            atomicAdd(cc + c, 1ull);
        }
    }
}

__global__ __launch_bounds__(256) void k_plan_keys(const int32_t *row, const int32_t *col, int64_t nnz,
                                                   const int64_t *rpos, const int64_t *cpos, int64_t bs_r,
                                                   int64_t bs_c, int32_t J, ull *kr, ull *kc, int32_t *eid,
                                                   ull *segr, ull *segc) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
        const int64_t pr = rpos[row[e]], pc = cpos[col[e]];
        const int64_t i = pr / bs_r, lr = pr - i * bs_r;
        const int64_t j = pc / bs_c, lc = pc - j * bs_c;
        const int64_t blk = i * J + j;
        kr[e] = (ull)(blk * bs_r + lr) * (ull)bs_c + (ull)lc;
        kc[e] = (ull)(blk * bs_c + lc) * (ull)bs_r + (ull)lr;
        eid[e] = (int32_t)e;
        atomicAdd(segr + blk * bs_r + lr, 1ull);
        atomicAdd(segc + blk * bs_c + lc, 1ull);
    }
}

// The sorted entries' local ids (key mod m) and centred values; the first
// position whose key repeats its predecessor's (a duplicate cell).
template <typename Tv>
__global__ __launch_bounds__(256) void k_plan_fill(const ull *key, const int32_t *ent, int64_t nnz, int64_t m,
                                                   const float *val, double ybar, int32_t *idx, Tv *v, ull *dup) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * 256) {
        const ull kk = key[k];
        idx[k] = (int32_t)(kk % (ull)m);
        v[k] = (Tv)((double)val[ent[k]] - ybar);
        if (k > 0 && key[k - 1] == kk) atomicMin(dup, (ull)k);
    }
}

// Per column (W order), the sum of its squared stored values in CSC order.
template <typename Tv>
__global__ __launch_bounds__(256) void k_plan_colsq(const int64_t *cptr, const int64_t *pidx, const Tv *cval,
                                                    int64_t ncol, double *colsq) {
#pragma clang fp contract(off)
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < ncol; g += (int64_t)gridDim.x * 256) {
        const int64_t q0 = cptr[pidx[g]], q1 = cptr[pidx[g] + 1];
        double s = 0.0;
        for (int64_t q = q0; q < q1; ++q) {
            const double r = (double)cval[q];
            s += r * r;
        }
        colsq[g] = s;
    }
}

int bits_for(ull maxkey) {
    int b = 1;
    while (b < 64 && (maxkey >> b) != 0) ++b;
    return b;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

#define PLAN_CHK(x)                                                                   \
    do {                                                                              \
        const hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess) {                                                       \
            err = std::string("device planner: ") + hipGetErrorString(e_);           \
            return BMF_EDEVICE;                                                       \
        }                                                                             \
    } while (0)

bmf_status gpu_build_plan(const bmf_config &cfg, double ybar, bool fp64, Plan &p, const GpuPlanDst &dst,
                          hipStream_t s, std::string &err) {
    bmf_status st = plan_partition(cfg, p, err);
    if (st) return st;
    const int64_t nnz = cfg.nnz, N = p.N, D = p.D;
    const int64_t nb = (int64_t)p.I * p.J;
    const int64_t nsr = nb * p.bs_r, nsc = nb * p.bs_c;
    // temporaries: the COO arrays, both key arrays and the sorted keys, the
    // entry ids, the degree counts, the radix sort's scratch
    DevBuf b_row, b_col, b_val, b_kr, b_kc, b_ko, b_eid, b_cnt, b_tmp;
    const int64_t ne = std::max<int64_t>(nnz, 1);
    PLAN_CHK(hipMalloc(&b_row.p, 4 * ne));
    PLAN_CHK(hipMalloc(&b_col.p, 4 * ne));
    PLAN_CHK(hipMalloc(&b_val.p, 4 * ne));
    PLAN_CHK(hipMalloc(&b_kr.p, 8 * ne));
    PLAN_CHK(hipMalloc(&b_kc.p, 8 * ne));
    PLAN_CHK(hipMalloc(&b_ko.p, 8 * ne));
    PLAN_CHK(hipMalloc(&b_eid.p, 4 * ne));
    const int64_t ncnt = N + D + nsr + nsc + 2;
    PLAN_CHK(hipMalloc(&b_cnt.p, 8 * ncnt));
    ull *rc = static_cast<ull *>(b_cnt.p), *cc = rc + N, *segr = cc + D, *segc = segr + nsr, *flags = segc + nsc;
    PLAN_CHK(hipMemsetAsync(b_cnt.p, 0, 8 * (ncnt - 2), s));
    const ull none = ~0ull;
    const ull none2[2] = {none, none};
    PLAN_CHK(hipMemcpy(flags, none2, 16, hipMemcpyHostToDevice));
    if (nnz > 0) {
        PLAN_CHK(hipMemcpyAsync(b_row.p, cfg.row, 4 * nnz, hipMemcpyHostToDevice, s));
        PLAN_CHK(hipMemcpyAsync(b_col.p, cfg.col, 4 * nnz, hipMemcpyHostToDevice, s));
        PLAN_CHK(hipMemcpyAsync(b_val.p, cfg.val, 4 * nnz, hipMemcpyHostToDevice, s));
    }
    const int32_t *drow = static_cast<int32_t *>(b_row.p), *dcol = static_cast<int32_t *>(b_col.p);
    const dim3 grid((unsigned)std::min<int64_t>((nnz + 255) / 256 + 1, 16384));
    hipLaunchKernelGGL(k_plan_count, grid, dim3(256), 0, s, drow, dcol, nnz, N, D, rc, cc, flags);
    PLAN_CHK(hipGetLastError());
    // ordering on the host from the degree counts
    std::vector<ull> hc((size_t)(N + D));
    ull bad = 0;
    PLAN_CHK(hipMemcpyAsync(hc.data(), rc, 8 * (N + D), hipMemcpyDeviceToHost, s));
    PLAN_CHK(hipMemcpyAsync(&bad, flags, 8, hipMemcpyDeviceToHost, s));
    PLAN_CHK(hipStreamSynchronize(s));
    if (bad != none) {
        err = "COO entry " + std::to_string(bad) + " out of range";
        return BMF_EINVAL;
    }
    std::vector<int64_t> rcount(hc.begin(), hc.begin() + N), ccount(hc.begin() + N, hc.end());
    p.row_pos = make_positions(N, rcount, cfg.order, cfg.seed, kPermRow);
    p.col_pos = make_positions(D, ccount, cfg.order, cfg.seed, kPermCol);
    PLAN_CHK(hipMemcpyAsync(dst.rowpos, p.row_pos.data(), 8 * N, hipMemcpyHostToDevice, s));
    PLAN_CHK(hipMemcpyAsync(dst.colpos, p.col_pos.data(), 8 * D, hipMemcpyHostToDevice, s));
    // keys, then one sort per order
    ull *kr = static_cast<ull *>(b_kr.p), *kc = static_cast<ull *>(b_kc.p), *ko = static_cast<ull *>(b_ko.p);
    int32_t *eid = static_cast<int32_t *>(b_eid.p);
    hipLaunchKernelGGL(k_plan_keys, grid, dim3(256), 0, s, drow, dcol, nnz, dst.rowpos, dst.colpos, p.bs_r, p.bs_c,
                       p.J, kr, kc, eid, segr, segc);
    PLAN_CHK(hipGetLastError());
    const int bits = bits_for((ull)nsr * (ull)p.bs_c);
    size_t tmp = 0;
    PLAN_CHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kr, ko, eid, dst.csr_ent, (int)nnz, 0, bits, s));
    PLAN_CHK(hipMalloc(&b_tmp.p, std::max<size_t>(tmp, 8)));
    const float *dval = static_cast<float *>(b_val.p);
    for (int pass = 0; pass < 2; ++pass) {
        const bool csr = pass == 0;
        size_t t2 = tmp;
        PLAN_CHK(hipcub::DeviceRadixSort::SortPairs(b_tmp.p, t2, csr ? kr : kc, ko, eid, csr ? dst.csr_ent : dst.csc_ent,
                                                    (int)nnz, 0, bits, s));
        const int64_t m = csr ? p.bs_c : p.bs_r;
        int32_t *idx = csr ? dst.csr_idx : dst.csc_idx;
        void *v = csr ? dst.csr_val : dst.csc_val;
        const int32_t *ent = csr ? dst.csr_ent : dst.csc_ent;
        if (fp64)
            hipLaunchKernelGGL(k_plan_fill<double>, grid, dim3(256), 0, s, ko, ent, nnz, m, dval, ybar, idx,
                               static_cast<double *>(v), flags + 1);
        else
            hipLaunchKernelGGL(k_plan_fill<float>, grid, dim3(256), 0, s, ko, ent, nnz, m, dval, ybar, idx,
                               static_cast<float *>(v), flags + 1);
        PLAN_CHK(hipGetLastError());
        if (csr) {
            ull dup = 0;
            PLAN_CHK(hipMemcpyAsync(&dup, flags + 1, 8, hipMemcpyDeviceToHost, s));
            PLAN_CHK(hipStreamSynchronize(s));
            if (dup != none) {
                int32_t pair[2] = {0, 0};
                PLAN_CHK(hipMemcpy(pair, dst.csr_ent + dup - 1, 8, hipMemcpyDeviceToHost));
                err = "duplicate COO cell at entries " + std::to_string(pair[0]) + " and " + std::to_string(pair[1]);
                return BMF_EINVAL;
            }
        }
    }
    // per-block pointers on the host from the block-row and block-column counts
    std::vector<ull> hs((size_t)(nsr + nsc));
    PLAN_CHK(hipMemcpyAsync(hs.data(), segr, 8 * (nsr + nsc), hipMemcpyDeviceToHost, s));
    PLAN_CHK(hipStreamSynchronize(s));
    p.blocks.assign(nb, PlanBlock());
    std::vector<int64_t> hptr[2];
    std::vector<int64_t> pidx;
    int64_t nz = 0;
    for (int64_t b = 0; b < nb; ++b) {
        PlanBlock &B = p.blocks[b];
        B.i = (int32_t)(b / p.J);
        B.j = (int32_t)(b % p.J);
        B.stage = stage_of(B.i, B.j);
        B.R = p.R[B.i];
        B.C = p.C[B.j];
        for (int pass = 0; pass < 2; ++pass) {
            const int64_t n = pass == 0 ? B.R : B.C;
            const ull *cnt = pass == 0 ? hs.data() + b * p.bs_r : hs.data() + nsr + b * p.bs_c;
            std::vector<int64_t> &bp = pass == 0 ? B.csr_ptr : B.csc_ptr;
            bp.assign(n + 1, 0);
            for (int64_t q = 0; q < n; ++q) bp[q + 1] = bp[q] + (int64_t)cnt[q];
            for (int64_t v : bp) hptr[pass].push_back(nz + v);
        }
        B.M = B.csr_ptr[B.R];
        nz += B.M;
    }
    PLAN_CHK(hipMemcpyAsync(dst.csr_ptr, hptr[0].data(), 8 * hptr[0].size(), hipMemcpyHostToDevice, s));
    PLAN_CHK(hipMemcpyAsync(dst.csc_ptr, hptr[1].data(), 8 * hptr[1].size(), hipMemcpyHostToDevice, s));
    // each column's first pointer in the global CSC pointer array (W order)
    {
        int64_t off = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t C = p.blocks[b].C;
            for (int64_t q = 0; q < C; ++q) pidx.push_back(off + q);
            off += C + 1;
        }
    }
    DevBuf b_pidx;
    PLAN_CHK(hipMalloc(&b_pidx.p, 8 * std::max<size_t>(pidx.size(), 1)));
    PLAN_CHK(hipMemcpyAsync(b_pidx.p, pidx.data(), 8 * pidx.size(), hipMemcpyHostToDevice, s));
    const int64_t ncol = (int64_t)pidx.size();
    const dim3 gc((unsigned)std::min<int64_t>((ncol + 255) / 256 + 1, 16384));
    if (fp64)
        hipLaunchKernelGGL(k_plan_colsq<double>, gc, dim3(256), 0, s, dst.csc_ptr, static_cast<int64_t *>(b_pidx.p),
                           static_cast<const double *>(dst.csc_val), ncol, dst.colsq);
    else
        hipLaunchKernelGGL(k_plan_colsq<float>, gc, dim3(256), 0, s, dst.csc_ptr, static_cast<int64_t *>(b_pidx.p),
                           static_cast<const float *>(dst.csc_val), ncol, dst.colsq);
    PLAN_CHK(hipGetLastError());
    PLAN_CHK(hipStreamSynchronize(s));
    return BMF_OK;
}

}  // namespace bmf
