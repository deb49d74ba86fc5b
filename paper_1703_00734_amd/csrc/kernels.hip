// HIP kernels (gfx950) of the BPMF Gibbs sweep under posterior propagation.
//
// Conditional update of one side of a block (Sec. 2.1 model; Gibbs sampler of
// Salakhutdinov & Mnih 2008b as used in Sec. 5.1): for entity n with observed
// set Omega_n,
//     A = P_n + tau * sum_{d in Omega_n} w_d w_d^T,
//     h = P_n m_n + tau * sum_{d in Omega_n} r_nd w_d,
//     L L^T = A,  x_n = L^-T (L^-1 h + z),  z ~ N(0, I)  (Philox counter (n, t, c2, g)).
// (P_n, P_n m_n) is the side's shared Normal-Wishart-drawn prior, or the
// propagated moment-matched per-row prior of PP stages 2-3 (eq. stage2a-stage3).
//
// Two update kernels:
//   * k_update_reg<KC>: K <= 16.  G lanes per entity (G a power of two <= 256,
//     chosen per degree), each lane accumulating the full packed Gram and
//     right-hand side in registers over a strided share of Omega_n; a
//     butterfly reduction (DPP and lane swaps) leaves the exact same sums in
//     every lane of the group, which then factor and solve redundantly in
//     registers.
//   * k_update_wave<KP>: K <= 64, one wavefront per entity.  The Gram is
//     accumulated on MFMA (BF16 state, KP >= 32) or as an 8x8 lane grid of
//     register tiles; the Cholesky factor and both triangular solves run in
//     registers, one matrix row per lane, with lane broadcasts.  Also runs the
//     FP64 redo of rows whose FP32 pivot test failed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <math.h>

#include "kernels.hpp"

namespace bmf {

// --------------------------------------------------------------------------
// scalar helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

// uniform on (0,1): (m + 1/2) 2^-23 from the top 23 bits; exact in FP32 and FP64
__device__ __forceinline__ float unif_f(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 1.1920928955078125e-7f; }
__device__ __forceinline__ double unif_d(uint32_t x) { return ((double)(x >> 9) + 0.5) * 1.1920928955078125e-7; }

// Four standard normals of counter (c0, c1, c2, g) by two Box-Muller transforms.
// FP32: the hardware transcendentals (v_log_f32 is log2, v_sin_f32 / v_cos_f32
// take the angle in turns, so 2 pi u needs no range reduction), each within a
// few ulp.
__device__ __forceinline__ void normals4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t g,
                                         uint32_t k0, uint32_t k1, float z[4]) {
    uint32_t o[4];
    philox4x32_10(c0, c1, c2, g, k0, k1, o);
    constexpr float kM2Ln2 = -1.38629436111989061883f;   // -2 ln 2
    const float r1 = __builtin_amdgcn_sqrtf(kM2Ln2 * __builtin_amdgcn_logf(unif_f(o[0])));
    const float r2 = __builtin_amdgcn_sqrtf(kM2Ln2 * __builtin_amdgcn_logf(unif_f(o[2])));
    const float u1 = unif_f(o[1]), u3 = unif_f(o[3]);
    z[0] = r1 * __builtin_amdgcn_cosf(u1); z[1] = r1 * __builtin_amdgcn_sinf(u1);
    z[2] = r2 * __builtin_amdgcn_cosf(u3); z[3] = r2 * __builtin_amdgcn_sinf(u3);
}
__device__ __forceinline__ void normals4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t g,
                                         uint32_t k0, uint32_t k1, double z[4]) {
    uint32_t o[4];
    philox4x32_10(c0, c1, c2, g, k0, k1, o);
    const double two_pi = 6.283185307179586476925286766559;
    const double r1 = sqrt(-2.0 * log(unif_d(o[0])));
    const double r2 = sqrt(-2.0 * log(unif_d(o[2])));
    const double t1 = two_pi * unif_d(o[1]), t2 = two_pi * unif_d(o[3]);
    z[0] = r1 * cos(t1); z[1] = r1 * sin(t1); z[2] = r2 * cos(t2); z[3] = r2 * sin(t2);
}

// Gamma(shape, 1), Marsaglia & Tsang (2000); attempt k on counter (c0,c1,c2,k);
// shape < 1 boosted by U^(1/shape) with U from counter (c0,c1,c2,0xFFFFFFFF).
__device__ double gamma_draw(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                             double shape) {
    double boost = 1.0, a = shape;
    if (a < 1.0) {
        uint32_t o[4];
        philox4x32_10(c0, c1, c2, 0xFFFFFFFFu, k0, k1, o);
        boost = pow(unif_d(o[0]), 1.0 / a);
        a += 1.0;
    }
    const double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
    const double two_pi = 6.283185307179586476925286766559;
    for (uint32_t k = 0; k < 64u; ++k) {
        uint32_t o[4];
        philox4x32_10(c0, c1, c2, k, k0, k1, o);
        const double z = sqrt(-2.0 * log(unif_d(o[0]))) * cos(two_pi * unif_d(o[1]));
        double v = 1.0 + c * z;
        if (v <= 0.0) continue;
        v = v * v * v;
        if (log(unif_d(o[2])) < 0.5 * z * z + d - d * v + d * log(v)) return d * v * boost;
    }
    return d * boost;
}

// End of a sweep: the fallback queues of the row and column passes start
// empty, the sweep index moves on, and the next sweep's sample slot (or none).
__device__ __forceinline__ void sweep_advance(SweepState *ss, int32_t *fb_counts) {
    fb_counts[0] = 0;
    fb_counts[1] = 0;
    SweepState s = *ss;
    if (s.slot >= 0) s.kept += 1;
    s.t += 1;
    const bool keep = (int64_t)s.t >= s.burnin && ((int64_t)s.t - s.burnin) % s.thin == 0 && s.kept < s.max_kept;
    s.slot = keep ? s.kept : -1;
    *ss = s;
}

// --------------------------------------------------------------------------
// butterfly sums inside a wavefront without the LDS crossbar
// --------------------------------------------------------------------------
// Step M of a butterfly over aligned groups of 2M lanes, for groups of M lanes
// that already hold one value each: M = 1, 2 pair lanes inside a quad (DPP
// quad_perm), M = 4, 8 mirror the 8- or 16-lane row (DPP row_half_mirror,
// row_mirror: lane i meets lane 2M-1-i, which holds what lane i^M holds), and
// M = 16, 32 swap rows between two registers (v_permlane16_swap /
// v_permlane32_swap).  Every lane of a group ends with the same two addends, so
// the group holds bitwise identical sums: the tree is that of the xor
// butterfly.
template <int M> __device__ __forceinline__ int dpp_partner(int v) {
    if constexpr (M == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    else if constexpr (M == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    else if constexpr (M == 4) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);
    else return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);
}
template <int M> __device__ __forceinline__ float bfly_step(float v) {
    const int b = __float_as_int(v);
    if constexpr (M < 16) {
        return v + __int_as_float(dpp_partner<M>(b));
    } else {
        const auto s = M == 16 ? __builtin_amdgcn_permlane16_swap(b, b, false, false)
                               : __builtin_amdgcn_permlane32_swap(b, b, false, false);
        return __int_as_float(s[0]) + __int_as_float(s[1]);
    }
}
template <int M> __device__ __forceinline__ double bfly_step(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xFFFFFFFFll), hi = (int)(b >> 32);
    auto join = [](int l, int h) { return __longlong_as_double(((long long)h << 32) | (unsigned int)l); };
    if constexpr (M < 16) {
        return v + join(dpp_partner<M>(lo), dpp_partner<M>(hi));
    } else {
        const auto sl = M == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                                : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto sh = M == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                                : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return join(sl[0], sh[0]) + join(sl[1], sh[1]);
    }
}
// Sums over aligned groups of Gw lanes (Gw a power of two <= 64, uniform over
// the wavefront); every lane of a group ends with the group's sum.
template <typename T, int N>
__device__ __forceinline__ void group_sum(T (&v)[N], int Gw) {
#define BMF_BFLY_STEP(M)                                          \
    if (Gw > M) {                                                 \
        _Pragma("unroll") for (int q = 0; q < N; ++q) v[q] = bfly_step<M>(v[q]); \
    }
    BMF_BFLY_STEP(1) BMF_BFLY_STEP(2) BMF_BFLY_STEP(4) BMF_BFLY_STEP(8) BMF_BFLY_STEP(16) BMF_BFLY_STEP(32)
#undef BMF_BFLY_STEP
}
template <typename T> __device__ __forceinline__ T group_sum1(T v, int Gw) {
    T a[1] = {v};
    group_sum(a, Gw);
    return a[0];
}

// --------------------------------------------------------------------------
// precision traits and vector row loads/stores
// --------------------------------------------------------------------------
// acc: arithmetic; w: gathered factors (= the other side's state); v: values;
// s: state written; p: kept samples.
template <int P> struct PrecT;
template <> struct PrecT<kP64> { using acc = double; using w = double; using v = double; using s = double; using p = double; };
template <> struct PrecT<kP32> { using acc = float; using w = float; using v = float; using s = float; using p = float; };
template <> struct PrecT<kPBF> { using acc = float; using w = uint16_t; using v = float; using s = uint16_t; using p = float; };
template <> struct PrecT<kPFB32> { using acc = double; using w = float; using v = float; using s = float; using p = float; };
template <> struct PrecT<kPFB16> { using acc = double; using w = uint16_t; using v = float; using s = uint16_t; using p = float; };

template <typename T> __host__ __device__ constexpr int vec_of() { return 16 / (int)sizeof(T); }
template <typename T> __host__ __device__ constexpr int ks_of(int kc) {
    return kc >= 32 ? kc : ((kc + vec_of<T>() - 1) / vec_of<T>()) * vec_of<T>();
}

template <typename Tacc, int KS>
__device__ __forceinline__ void load_row(const float *p, Tacc (&w)[KS]) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int v = 0; v < KS / 4; ++v) {
        const float4 f = q[v];
        w[4 * v] = (Tacc)f.x; w[4 * v + 1] = (Tacc)f.y; w[4 * v + 2] = (Tacc)f.z; w[4 * v + 3] = (Tacc)f.w;
    }
}
template <typename Tacc, int KS>
__device__ __forceinline__ void load_row(const double *p, Tacc (&w)[KS]) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int v = 0; v < KS / 2; ++v) {
        const double2 f = q[v];
        w[2 * v] = (Tacc)f.x; w[2 * v + 1] = (Tacc)f.y;
    }
}
template <typename Tacc, int KS>
__device__ __forceinline__ void load_row(const uint16_t *p, Tacc (&w)[KS]) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int v = 0; v < KS / 8; ++v) {
        const uint4 u = q[v];
        const uint32_t x[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            w[8 * v + 2 * c] = (Tacc)__uint_as_float(x[c] << 16);
            w[8 * v + 2 * c + 1] = (Tacc)__uint_as_float(x[c] & 0xFFFF0000u);
        }
    }
}

// Store K values (zero padded to the stride) of x into a storage row.
template <int KC, typename Tacc>
__device__ __forceinline__ void store_row(float *p, const Tacc (&x)[KC], int K) {
    constexpr int KS = ks_of<float>(KC);
    float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int v = 0; v < KS / 4; ++v) {
        float e[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k = 4 * v + c;
            e[c] = (k < KC && k < K) ? (float)x[k < KC ? k : 0] : 0.0f;
        }
        q[v] = make_float4(e[0], e[1], e[2], e[3]);
    }
}
template <int KC, typename Tacc>
__device__ __forceinline__ void store_row(double *p, const Tacc (&x)[KC], int K) {
    constexpr int KS = ks_of<double>(KC);
    double2 *q = reinterpret_cast<double2 *>(p);
#pragma unroll
    for (int v = 0; v < KS / 2; ++v) {
        const int k0 = 2 * v, k1 = 2 * v + 1;
        const double e0 = (k0 < KC && k0 < K) ? (double)x[k0 < KC ? k0 : 0] : 0.0;
        const double e1 = (k1 < KC && k1 < K) ? (double)x[k1 < KC ? k1 : 0] : 0.0;
        q[v] = make_double2(e0, e1);
    }
}
template <int KC, typename Tacc>
__device__ __forceinline__ void store_row_bf16(uint16_t *p, const Tacc (&x)[KC], int K) {
    constexpr int KS = ks_of<uint16_t>(KC);
    uint4 *q = reinterpret_cast<uint4 *>(p);
#pragma unroll
    for (int v = 0; v < KS / 8; ++v) {
        uint32_t e[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int ka = 8 * v + 2 * c, kb = ka + 1;
            const uint32_t lo = (ka < KC && ka < K) ? f32_to_bf16((float)x[ka < KC ? ka : 0]) : 0u;
            const uint32_t hi = (kb < KC && kb < K) ? f32_to_bf16((float)x[kb < KC ? kb : 0]) : 0u;
            e[c] = lo | (hi << 16);
        }
        q[v] = make_uint4(e[0], e[1], e[2], e[3]);
    }
}

// The first NW dwords of a factor row (16-byte aligned) in as few loads as
// possible, kept raw until the FMAs convert them: rows of a later pair can be
// in flight while the current pair is used.
template <int NW>
__device__ __forceinline__ void load_raw(const void *p, uint32_t (&r)[NW]) {
    const uint4 *q4 = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int v = 0; v < NW / 4; ++v) {
        const uint4 u = q4[v];
        r[4 * v] = u.x; r[4 * v + 1] = u.y; r[4 * v + 2] = u.z; r[4 * v + 3] = u.w;
    }
    constexpr int R = NW % 4, B = NW - R;
    const uint32_t *q1 = reinterpret_cast<const uint32_t *>(p) + B;
    if constexpr (R >= 2) {
        const uint2 u = *reinterpret_cast<const uint2 *>(q1);
        r[B] = u.x; r[B + 1] = u.y;
    }
    if constexpr (R == 1 || R == 3) r[NW - 1] = q1[R - 1];
}
template <typename Tw> __host__ __device__ constexpr int raw_words(int kc) {
    return (kc * (int)sizeof(Tw) + 3) / 4;
}
// Element k of a raw row as the arithmetic type.
template <typename Tacc, typename Tw, int NW>
__device__ __forceinline__ Tacc raw_elem(const uint32_t (&r)[NW], int k) {
    if constexpr (sizeof(Tw) == 2) {
        const uint32_t x = r[k >> 1];
        return (Tacc)__uint_as_float((k & 1) ? (x & 0xFFFF0000u) : (x << 16));
    } else if constexpr (sizeof(Tw) == 4) {
        return (Tacc)__uint_as_float(r[k]);
    } else {
        return (Tacc)__hiloint2double((int)r[2 * k + 1], (int)r[2 * k]);
    }
}

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }


template <typename T> __device__ __forceinline__ double elem_to_d(T v) { return (double)v; }
template <> __device__ __forceinline__ double elem_to_d<uint16_t>(uint16_t v) { return (double)bf16_to_f32(v); }
template <typename T> __device__ __forceinline__ T elem_from(double v) { return (T)v; }
template <> __device__ __forceinline__ uint16_t elem_from<uint16_t>(double v) { return f32_to_bf16((float)v); }

template <int KC, typename Tacc>
__device__ __forceinline__ void store_row(uint16_t *p, const Tacc (&x)[KC], int K) { store_row_bf16<KC>(p, x, K); }

// Pivot of a Cholesky step: l = sqrt(d) and 1 / l.  FP32 takes v_rsq_f32
// (about 1 ulp); FP64 keeps the correctly rounded operations.
__device__ __forceinline__ void pivot_of(float d, float &l, float &inv) {
    inv = __builtin_amdgcn_rsqf(d);
    l = d * inv;
}
__device__ __forceinline__ void pivot_of(double d, double &l, double &inv) {
    l = sqrt(d);
    inv = 1.0 / l;
}

// --------------------------------------------------------------------------
// k_update_reg: K <= KC <= 16, G lanes per entity, Gram in registers.
// --------------------------------------------------------------------------
// SSE: the column pass also writes each column's residual sum of squares
// (a.sse_col), for the tau draw of the same sweep.
template <int KC, int P, bool SSE>
__global__ __launch_bounds__(256) void k_update_reg(const UpdArgs a) {
    using Tacc = typename PrecT<P>::acc;
    using Tw = typename PrecT<P>::w;
    using Tv = typename PrecT<P>::v;
    using Ts = typename PrecT<P>::s;
    using Tp = typename PrecT<P>::p;
    constexpr int NT = KC * (KC + 1) / 2;
    constexpr int KSW = ks_of<Tw>(KC);
    constexpr int KSS = ks_of<Ts>(KC);
    constexpr int KSP = ks_of<Tp>(KC);
    constexpr bool kFP32 = sizeof(Tacc) == 4;

    uint32_t t_sw = a.t;
    void *sample = a.sample;
    if (a.ss) {
        t_sw = a.ss->t;
        sample = a.ss->slot >= 0 ? reinterpret_cast<char *>(a.sample) + a.ss->slot * a.ss->slot_bytes : nullptr;
    }
    const Tile tl = a.tiles[blockIdx.x];
    const int G = tl.G;                    // lanes per entity: 1..64, or 128/256 (several waves)
    const int grp = threadIdx.x / G;
    const bool wide = G > 64;              // uniform per tile
    // groups of at least four lanes hand their sums to one lane each for the
    // factorization (through LDS, after a barrier): empty groups stay until then
    constexpr bool kPackable = sizeof(Tacc) == 4;
    const bool pack = kPackable && G >= 4;
    if (!wide && !pack && grp >= tl.count) return;  // whole groups only: shuffles stay inside a group
    const bool active = grp < tl.count;
    int gl = threadIdx.x & (G - 1);
    const SideDesc &sd = a.sides[tl.side];
    const int K = a.K;
    int n = active ? a.ord[tl.start + grp] : 0;
    const int64_t p0 = active ? a.ptr[sd.ptr_off + n] : 0;
    const int64_t p1 = active ? a.ptr[sd.ptr_off + n + 1] : 0;
    const Tw *other = reinterpret_cast<const Tw *>(a.other) + sd.other_off * KSW;
    const Tv *val = reinterpret_cast<const Tv *>(a.val);

    Tacc g[NT];
    Tacc hs[KC];
#pragma unroll
    for (int q = 0; q < NT; ++q) g[q] = 0;
#pragma unroll
    for (int i = 0; i < KC; ++i) hs[i] = 0;

    // Pairs of entries (e, e + G): the factor rows of the next pair are
    // requested before the FMAs of the current one, the indices and values two
    // pairs ahead; the FMAs take the entries in order.
    constexpr int NW = raw_words<Tw>(KC);
    auto fma_entry = [&](const uint32_t (&wr)[NW], Tacc r) {
        Tacc w[KC];
#pragma unroll
        for (int i = 0; i < KC; ++i) w[i] = raw_elem<Tacc, Tw, NW>(wr, i);
#pragma unroll
        for (int i = 0; i < KC; ++i) {
            hs[i] += r * w[i];
#pragma unroll
            for (int j = 0; j <= i; ++j) g[tri(i, j)] += w[i] * w[j];
        }
    };
    // BF16 rows: component i of the pair packed as (w0_i, w1_i) so that one
    // v_dot2c_f32_bf16 adds w0_i w0_j + w1_i w1_j to the Gram (the products of
    // BF16 values are exact in FP32); the right-hand side stays in FP32 FMAs.
    auto fma_pair_bf16 = [&](const uint32_t (&w0)[NW], const uint32_t (&w1)[NW], Tacc r0, Tacc r1) {
        typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
        uint32_t pk[2 * NW];
#pragma unroll
        for (int m = 0; m < NW; ++m) {
            pk[2 * m] = __builtin_amdgcn_perm(w1[m], w0[m], 0x05040100u);
            pk[2 * m + 1] = __builtin_amdgcn_perm(w1[m], w0[m], 0x07060302u);
        }
#pragma unroll
        for (int i = 0; i < KC; ++i) {
            hs[i] += r0 * raw_elem<Tacc, Tw, NW>(w0, i);
            hs[i] += r1 * raw_elem<Tacc, Tw, NW>(w1, i);
            const bf16x2_t pi = __builtin_bit_cast(bf16x2_t, pk[i]);
#pragma unroll
            for (int j = 0; j <= i; ++j)
                g[tri(i, j)] = __builtin_amdgcn_fdot2_f32_bf16(pi, __builtin_bit_cast(bf16x2_t, pk[j]),
                                                               g[tri(i, j)], false);
        }
    };
    const int64_t step = 2 * (int64_t)G;
    int64_t e = p0 + gl;
    if constexpr (sizeof(Tw) < 8) {
        // Four entries per lane per iteration (e, e + G, e + 2G, e + 3G).  Every
        // load is unconditional (addresses clamped to the entity's last entry;
        // entries past the end are masked where the rows are consumed), and
        // the next batch's indices and values are loaded into the registers
        // this batch has finished with: no loaded register is copied or
        // selected before use, so the loads stay in flight across iterations
        // instead of forcing a wait on each one.
        constexpr int B = 4;
        // 32-bit entry offsets from the entity's first entry, and 32-bit byte
        // offsets of the gathered rows from the side's (uniform) base, so the
        // loads take the scalar-base plus vector-offset form
        const int32_t deg = (int32_t)(p1 - p0);
        const int32_t lastk = deg - 1;
        const int32_t *idxb = a.idx + p0;
        const Tv *valb = val + p0;
        const char *ob = reinterpret_cast<const char *>(other);
        constexpr uint32_t RB = KSW * sizeof(Tw);
        int32_t k = gl;
        int dq[B];
        Tacc rq[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int32_t ku = min(k + u * G, lastk);
            dq[u] = deg > 0 ? idxb[ku] : 0;
            rq[u] = deg > 0 ? (Tacc)valb[ku] : (Tacc)0;
        }
        for (; k < deg; k += B * G) {
            Tacc rc[B];
            bool ok[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                ok[u] = k + u * G < deg;
                rc[u] = ok[u] ? rq[u] : (Tacc)0;
            }
            // issue order: this batch's rows, then the next batch's indices and
            // values; one wait (for the rows only) before the arithmetic
            uint32_t w[B][NW];
#pragma unroll
            for (int u = 0; u < B; ++u) load_raw<NW>(ob + (uint32_t)dq[u] * RB, w[u]);
            const int32_t kn = k + B * G;
#pragma unroll
            for (int u = 0; u < B; ++u) dq[u] = idxb[min(kn + u * G, lastk)];
#pragma unroll
            for (int u = 0; u < B; ++u) rq[u] = (Tacc)valb[min(kn + u * G, lastk)];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < B; ++u)
#pragma unroll
                for (int v = 0; v < NW; ++v) asm volatile("" : "+v"(w[u][v]));
#pragma unroll
            for (int u = 0; u < B; ++u)
#pragma unroll
                for (int v = 0; v < NW; ++v) w[u][v] = ok[u] ? w[u][v] : 0u;
            if constexpr (sizeof(Tw) == 2) {
                fma_pair_bf16(w[0], w[1], rc[0], rc[1]);
                fma_pair_bf16(w[2], w[3], rc[2], rc[3]);
            } else {
#pragma unroll
                for (int u = 0; u < B; ++u) fma_entry(w[u], rc[u]);
            }
        }
        e = p0 + k;
    } else {
        // FP64 rows: one pair in flight (the pipeline would cost occupancy)
        for (; e + G < p1; e += step) {
            uint32_t w0r[NW], w1r[NW];
            const int d0 = a.idx[e], d1 = a.idx[e + G];
            const Tacc r0 = (Tacc)val[e], r1 = (Tacc)val[e + G];
            load_raw<NW>(other + (int64_t)d0 * KSW, w0r);
            load_raw<NW>(other + (int64_t)d1 * KSW, w1r);
            fma_entry(w0r, r0);
            fma_entry(w1r, r1);
        }
    }
    if (e < p1) {
        uint32_t w1r[NW];
        load_raw<NW>(other + (int64_t)a.idx[e] * KSW, w1r);
        fma_entry(w1r, (Tacc)val[e]);
    }
    // butterfly inside the wave: every lane of the group ends with bitwise
    // identical sums
    const int Gw = G < 64 ? G : 64;
    group_sum(g, Gw);
    group_sum(hs, Gw);
    if (wide) {
        // groups spanning several waves: wave sums through LDS, added in wave order
        __shared__ Tacc wsum[4][NT + KC];
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int q = 0; q < NT; ++q) wsum[wave][q] = g[q];
#pragma unroll
            for (int i = 0; i < KC; ++i) wsum[wave][NT + i] = hs[i];
        }
        __syncthreads();
        const int w0 = (grp * G) >> 6, nw = G >> 6;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            Tacc v = wsum[w0][q];
            for (int u = 1; u < nw; ++u) v += wsum[w0 + u][q];
            g[q] = v;
        }
#pragma unroll
        for (int i = 0; i < KC; ++i) {
            Tacc v = wsum[w0][NT + i];
            for (int u = 1; u < nw; ++u) v += wsum[w0 + u][NT + i];
            hs[i] = v;
        }
        if (!active && !pack) return;
    }
    if (pack) {
        // one lane per entity from here on: lane t of the block factors the
        // t-th entity of the tile, so that a tile of wide groups runs the
        // factorization on one wavefront instead of on every lane of every group
        constexpr int NS = NT + KC;
        __shared__ Tacc psum[kPackable ? 64 * NS : 1];
        if (active && gl == 0) {
#pragma unroll
            for (int q = 0; q < NT; ++q) psum[grp * NS + q] = g[q];
#pragma unroll
            for (int i = 0; i < KC; ++i) psum[grp * NS + NT + i] = hs[i];
        }
        __syncthreads();
        const int t = threadIdx.x;
        if (t >= tl.count) return;
#pragma unroll
        for (int q = 0; q < NT; ++q) g[q] = psum[t * NS + q];
#pragma unroll
        for (int i = 0; i < KC; ++i) hs[i] = psum[t * NS + NT + i];
        n = a.ord[tl.start + t];
        gl = 0;
    }
    const int Ge = pack ? 1 : G;            // lanes per entity in the factorization

    // A = P + tau G, h = P m + tau hs (identity padding beyond K); the prior is
    // a packed row [P lower (row-major), P m, m]: the side's own row when
    // propagated, the shared Normal-Wishart prior otherwise
    const Tacc tau = (Tacc)sd.tau[(int64_t)sd.tau_stride * n];
    const double *pr = sd.prior + (sd.per_row ? (int64_t)n * a.prow : 0);
    Tacc hraw[SSE ? KC : 1];                // sum r w of the column, for its SSE
    if constexpr (SSE) {
#pragma unroll
        for (int i = 0; i < KC; ++i) hraw[i] = hs[i];
    }
    {
        const double *eta = pr + K * (K + 1) / 2;
#pragma unroll
        for (int i = 0; i < KC; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j)
                g[tri(i, j)] = (i < K) ? (Tacc)pr[tri(i, j)] + tau * g[tri(i, j)] : (Tacc)(i == j);
            hs[i] = (i < K) ? (Tacc)eta[i] + tau * hs[i] : (Tacc)0;
        }
    }

    // Cholesky (column by column) with the pivot test
    const Tacc theta = (Tacc)a.theta;
    bool ok = true;
    Tacc inv[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        const Tacc diag = g[tri(j, j)];
        Tacc dj = diag;
#pragma unroll
        for (int p = 0; p < j; ++p) dj -= g[tri(j, p)] * g[tri(j, p)];
        ok = ok && (kFP32 ? (dj > theta * diag) : (dj > (Tacc)0));
        Tacc l, il;
        pivot_of(dj > (Tacc)0 ? dj : (Tacc)1, l, il);
        g[tri(j, j)] = l;
        inv[j] = il;
#pragma unroll
        for (int i = j + 1; i < KC; ++i) {
            Tacc s = g[tri(i, j)];
#pragma unroll
            for (int p = 0; p < j; ++p) s -= g[tri(i, p)] * g[tri(j, p)];
            g[tri(i, j)] = s * il;
        }
    }
    if (!ok) {
        if (gl == 0) {
            if (a.fb_list) {
                const int slot = atomicAdd(a.fb_count, 1);
                a.fb_list[slot] = make_int2(tl.side, n);
                atomicAdd(a.fb_total, 1);
            } else {
                atomicAdd(a.nonpd, 1);
            }
        }
        return;
    }

    // y = L^-1 h;  y += z;  x = L^-T y
    Tacc y[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) {
        Tacc s = hs[i];
#pragma unroll
        for (int p = 0; p < i; ++p) s -= g[tri(i, p)] * y[p];
        y[i] = s * inv[i];
    }
    // noise: block q of four normals has counter word 3 = q.  A group with at
    // least as many lanes as blocks (inside one wavefront) draws each block once
    // and shares it; otherwise every lane draws every block.
    const int NQ = (K + 3) / 4;
    if (Ge >= NQ && Ge <= 64) {
        Tacc zq[4];
        normals4((uint32_t)n, t_sw, sd.c2, (uint32_t)(gl < NQ ? gl : 0), a.k0, a.k1, zq);
        const int base = (threadIdx.x & 63) & ~(Ge - 1);
#pragma unroll
        for (int q = 0; q < (KC + 3) / 4; ++q) {
            if (q < NQ) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const Tacc zc = __shfl(zq[c], base + q);
                    if (4 * q + c < KC && 4 * q + c < K) y[4 * q + c < KC ? 4 * q + c : 0] += zc;
                }
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < (KC + 3) / 4; ++q) {
            if (4 * q < K) {
                Tacc z[4];
                normals4((uint32_t)n, t_sw, sd.c2, (uint32_t)q, a.k0, a.k1, z);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (4 * q + c < KC && 4 * q + c < K) y[4 * q + c < KC ? 4 * q + c : 0] += z[c];
            }
        }
    }
    Tacc x[KC];
#pragma unroll
    for (int i = KC - 1; i >= 0; --i) {
        Tacc s = y[i];
#pragma unroll
        for (int p = i + 1; p < KC; ++p) s -= g[tri(p, i)] * x[p];
        x[i] = s * inv[i];
    }

    if (gl == 0) {
        Ts *self = reinterpret_cast<Ts *>(a.self);
        store_row<KC>(self + (sd.self_off + n) * KSS, x, K);
        if (sample) store_row<KC>(reinterpret_cast<Tp *>(sample) + (sd.sample_off + n) * KSP, x, K);
    }
    if constexpr (SSE) {
        // Residual SSE of this column with the new w as stored, from the sums
        // this pass already holds: sum_e (r_e - w.x_e)^2 = sum r^2 - 2 w.h_raw
        // + w^T G_raw w, and tau w^T G_raw w = |L^T w|^2 - w^T P w since
        // A = P + tau G_raw = L L^T.  Products and sums in FP64.
        if (gl == 0) {
            Tacc wd[KC];
#pragma unroll
            for (int i = 0; i < KC; ++i) wd[i] = i < K ? (Tacc)elem_to_d(elem_from<Ts>((double)x[i])) : (Tacc)0;
            double hw = 0.0, lw2 = 0.0, pw = 0.0;
#pragma unroll
            for (int i = 0; i < KC; ++i) {
                hw += (double)hraw[i] * (double)wd[i];
                double u = 0.0;
#pragma unroll
                for (int p = i; p < KC; ++p) u += (double)g[tri(p, i)] * (double)wd[p];
                lw2 += u * u;
            }
#pragma unroll
            for (int r = 0; r < KC; ++r) {
                if (r < K) {
                    double q = 0.0;
#pragma unroll
                    for (int c = 0; c < r; ++c) q += pr[tri(r, c)] * (double)wd[c];
                    pw += (double)wd[r] * (2.0 * q + pr[tri(r, r)] * (double)wd[r]);
                }
            }
            double *slot = a.sse_col + 4 * (sd.self_off + n);
            slot[0] = a.colsq[sd.self_off + n] - 2.0 * hw + (lw2 - pw) / (double)tau;
            slot[1] = 0.0;
            slot[2] = 0.0;
            slot[3] = 0.0;
        }
    }
}


// --------------------------------------------------------------------------
// LDS linear algebra for one wavefront (all 64 lanes call these)
// --------------------------------------------------------------------------
// In-place Cholesky of the leading K x K block of M (row stride ld, lower
// triangle).  With theta > 0 a pivot that is not above theta * diag0[k] fails;
// with theta = 0 a pivot that is not positive fails.  *flag is LDS scratch.
template <typename T>
__device__ bool chol_lds(T *M, int K, int ld, T theta, const T *diag0, int lane, int *flag) {
    if (lane == 0) *flag = 0;
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        if (lane == 0) {
            const T d = M[k * ld + k];
            const bool bad = (theta > (T)0) ? !(d > theta * diag0[k]) : !(d > (T)0);
            if (bad) *flag = 1;
            M[k * ld + k] = sqrt(d > (T)0 ? d : (T)1);
        }
        __syncthreads();
        const T lkk = M[k * ld + k];
        for (int i = k + 1 + lane; i < K; i += 64) M[i * ld + k] /= lkk;
        __syncthreads();
        for (int i = k + 1 + lane; i < K; i += 64) {
            const T lik = M[i * ld + k];
            for (int j = k + 1; j <= i; ++j) M[i * ld + j] -= lik * M[j * ld + k];
        }
        __syncthreads();
    }
    return *flag == 0;
}

// y <- L^-1 y, L lower in M.
template <typename T>
__device__ void fwd_lds(const T *M, int K, int ld, T *y, int lane) {
    for (int k = 0; k < K; ++k) {
        if (lane == 0) y[k] /= M[k * ld + k];
        __syncthreads();
        const T yk = y[k];
        for (int i = k + 1 + lane; i < K; i += 64) y[i] -= M[i * ld + k] * yk;
        __syncthreads();
    }
}

// x <- L^-T x, L lower in M.
template <typename T>
__device__ void bwd_lds(const T *M, int K, int ld, T *x, int lane) {
    for (int k = K - 1; k >= 0; --k) {
        if (lane == 0) x[k] /= M[k * ld + k];
        __syncthreads();
        const T xk = x[k];
        for (int i = lane; i < k; i += 64) x[i] -= M[k * ld + i] * xk;
        __syncthreads();
    }
}

// Broadcast of lane `src`'s value to the whole wavefront (src uniform).
__device__ __forceinline__ float wave_bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double wave_bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Left-looking Cholesky A = L L^T with one matrix row per lane (KP <= 64
// lanes): step k forms s_i = a_ik - sum_{p<k} l_ip l_kp in every lane i from
// its own finished row entries and row k of L, read from LDS by broadcast
// 16-byte loads, takes the pivot from lane k (v_readlane) and writes l_ik to
// sL (row stride ldl, a multiple of 16 bytes).  Lanes run every step (entries
// above their diagonal come out as unused values), so the steps need no lane
// masks.  In: sA (lower, row stride ld, KP x KP with identity padding; sL may
// overlay sA: every row of A is read before the first write), diag0 = diag(A).
// Out: r = the lane's row of L, sinv[i] = 1 / l_ii.  Returns false in every
// lane when a pivot is not above theta times its diagonal entry (theta = 0:
// not positive).  lane and z0 (0, a multiple of 16) come opaque from the
// caller: values derived from them must not be hoisted out of its loops.
template <int KP, typename T>
__device__ __forceinline__ bool chol_rows(const T *sA, int ld, T *sL, int ldl, const T *diag0, T *sinv,
                                          T theta, int lane, int z0, T (&r)[KP]) {
    const bool own = lane < KP;
    const int row = own ? lane : KP - 1;    // lanes without a row shadow the last one
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const T v = sA[row * ld + j];
        r[j] = j <= lane ? v : (T)0;
        asm volatile("" : "+v"(r[j]));      // select now, not at first use
    }
    const T d0 = diag0[row];
    __syncthreads();                        // all of A read before L overlays it
    int mybad = 0;
    T myinv = (T)1;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        // two interleaved partial sums halve the dependent chain
        T s0 = r[k], s1 = (T)0;
        const T *lk = sL + z0 + k * ldl;
#pragma unroll
        for (int p = 0; p < k; ++p) {
            if (p & 1) s1 -= r[p] * lk[p];
            else s0 -= r[p] * lk[p];
            // at most 16 broadcast values in flight (register pressure)
            if ((p & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        }
        const T sk = s0 + s1;
        const T dk = wave_bcast(sk, k);
        // pivot test in the pivot's own lane, against its own diagonal entry;
        // padding steps see the identity: pivot 1 > theta, always passes
        mybad = lane == k ? (int)!(sk > theta * d0) : mybad;
        T lkk, inv;
        pivot_of(dk > (T)0 ? dk : (T)1, lkk, inv);
        myinv = lane == k ? inv : myinv;
        r[k] = lane == k ? lkk : sk * inv;
        if (own) sL[lane * ldl + k] = r[k];
        __builtin_amdgcn_wave_barrier();
        // the entry is final: keep the compiler from recomputing it later,
        // and start the next step only after this one
        asm volatile("" : "+v"(r[k]), "+v"(myinv), "+v"(mybad));
        __builtin_amdgcn_sched_barrier(0);
    }
    if (own) sinv[lane] = myinv;
    return __ballot(mybad) == 0;
}

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

// chol_rows for KP = 64 in FP32 with the second panel's update on MFMA: steps
// 0..31 as in chol_rows; then S = L21 L21^T (L21 = rows 32..63, columns 0..31
// of L) by sixteen v_mfma_f32_32x32x2_f32, subtracted from the rows of lanes
// 32..63; then steps 32..63 need only the columns 32..k-1 in their dot products.
// The product's 32 x 32 result passes through the still unwritten block
// (rows and columns 32..63) of sL.  Same contract as chol_rows.
__device__ __forceinline__ bool chol_rows64_mfma(const float *sA, int ld, float *sL, int ldl, const float *diag0,
                                                 float *sinv, float theta, int lane, int z0, float (&r)[64]) {
    constexpr int KP = 64;
    const int row = lane;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const float v = sA[row * ld + j];
        r[j] = j <= lane ? v : 0.0f;
        asm volatile("" : "+v"(r[j]));
    }
    const float d0 = diag0[row];
    __syncthreads();                        // all of A read before L overlays it
    int mybad = 0;
    float myinv = 1.0f;
    auto step = [&](const int k, const int p0) __attribute__((always_inline)) {
        float s0 = r[k], s1 = 0.0f;
        const float *lk = sL + z0 + k * ldl;
#pragma unroll
        for (int p = p0; p < k; ++p) {
            if (p & 1) s1 -= r[p] * lk[p];
            else s0 -= r[p] * lk[p];
            if ((p & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        }
        const float sk = s0 + s1;
        const float dk = wave_bcast(sk, k);
        mybad = lane == k ? (int)!(sk > theta * d0) : mybad;
        float lkk, inv;
        pivot_of(dk > 0.0f ? dk : 1.0f, lkk, inv);
        myinv = lane == k ? inv : myinv;
        r[k] = lane == k ? lkk : sk * inv;
        sL[lane * ldl + k] = r[k];
        __builtin_amdgcn_wave_barrier();
        asm volatile("" : "+v"(r[k]), "+v"(myinv), "+v"(mybad));
        __builtin_amdgcn_sched_barrier(0);
    };
#pragma unroll
    for (int k = 0; k < 32; ++k) step(k, 0);
    // S = L21 L21^T: operand of lane l at pair s is L[32 + l % 32][2s + l / 32]
    // (the same register serves as A and as B)
    f32x16_t acc = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const float up = __int_as_float(__builtin_amdgcn_ds_bpermute(4 * ((lane + 32) & 63), __float_as_int(r[2 * s])));
        const float op = lane < 32 ? up : r[2 * s + 1];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(op, op, acc, 0, 0, 0);
    }
    {
        const int col = lane & 31;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int rw = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
            sL[(32 + rw) * ldl + 32 + col] = acc[v];
        }
    }
    __syncthreads();
    if (lane >= 32) {
#pragma unroll
        for (int j = 32; j < KP; ++j) r[j] -= sL[lane * ldl + j];
    }
#pragma unroll
    for (int j = 32; j < KP; ++j) asm volatile("" : "+v"(r[j]));
    __syncthreads();                        // the product is read before steps 32.. overwrite it
#pragma unroll
    for (int k = 32; k < KP; ++k) step(k, 32);
    sinv[lane] = myinv;
    return __ballot(mybad) == 0;
}

// Factor A = L L^T and solve x = L^-T (L^-1 h + z) in registers (chol_rows,
// then a forward solve with row ownership and a backward solve that reads
// columns of L from LDS).  In: sA (lower, row stride ld, KP x KP with identity
// padding), sh = h, sz = z (zero beyond K), diag0 = diag(A).  Out: sh = x, L
// in sL.  Returns false when a pivot fails the test of chol_rows.  All 64
// lanes call it.
template <int KP, typename T>
__device__ __forceinline__ bool factor_solve_regs(const T *sA, int ld, T *sL, int ldl, T *sh,
                                                  const T *sz, const T *diag0, T *sinv, T theta,
                                                  int K, int lane) {
    // an opaque lane index: the masks and LDS addresses derived from it would
    // otherwise be hoisted out of the caller's item loop and all stay live
    asm volatile("" : "+v"(lane));
    // broadcast reads index from an opaque zero (a multiple of 16 elements, so
    // alignment is still known) so that their constant part folds into the
    // instruction's offset instead of a hoisted address register
    int z0 = 0;
    asm volatile("" : "+v"(z0));
    z0 &= ~15;
    const bool own = lane < KP;
    const int row = own ? lane : KP - 1;
    T r[KP];
    bool ok;
    if constexpr (KP == 64 && sizeof(T) == 4)
        ok = chol_rows64_mfma(sA, ld, sL, ldl, diag0, sinv, theta, lane, z0, r);
    else
        ok = chol_rows<KP, T>(sA, ld, sL, ldl, diag0, sinv, theta, lane, z0, r);
    __syncthreads();
    // each phase compares against a fresh opaque copy of the lane index, so
    // that no lane mask is shared (and kept live) across phases
    asm volatile("" : "+v"(lane));
    // forward: y = L^-1 h, then v = y + z
    T acc = sh[row];
    T y = (T)0;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        const T yq = wave_bcast(acc, q) * sinv[z0 + q];
        y = lane == q ? yq : y;
        acc = (lane > q) ? acc - r[q] * yq : acc;
    }
    const T v = (lane < K) ? y + sz[row] : (T)0;
    asm volatile("" : "+v"(lane));
    // L^T by columns: lane i takes column i of L
    T c[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        const T v2 = sL[q * ldl + row];
        c[q] = q >= lane ? v2 : (T)0;
        asm volatile("" : "+v"(c[q]));
    }
    asm volatile("" : "+v"(lane));
    // backward: x = L^-T v
    acc = v;
    T x = (T)0;
#pragma unroll
    for (int q = KP - 1; q >= 0; --q) {
        const T xq = wave_bcast(acc, q) * sinv[z0 + q];
        x = lane == q ? xq : x;
        acc = (lane < q) ? acc - c[q] * xq : acc;
    }
    __syncthreads();
    if (own) sh[lane] = x;
    __syncthreads();
    return ok;
}


template <typename T> __device__ __forceinline__ T to_acc(float v) { return (T)v; }
template <typename T> __device__ __forceinline__ T to_acc(double v) { return (T)v; }
template <typename T> __device__ __forceinline__ T to_acc(uint16_t v) { return (T)bf16_to_f32(v); }

// --------------------------------------------------------------------------
// k_update_wave: one wavefront per entity, any K <= KP.
// --------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));

// LDS staging of mfma_gram: the rows of one chunk of 32 entries (16-byte
// aligned rows of KP + 8 elements) and the chunk's 32 values.
template <int KP> __host__ __device__ constexpr int gram_stage_bytes() { return 2 * 32 * (KP + 8) + 4 * 32; }

// MFMA Gram and right-hand side of the observed entries [b0, b1) of one
// entity (BF16 factors of stride ks): on return, accumulator v of lane l holds
// G[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] of the blocks G00 (c00), G10
// (c10) and G11 (c11) (KP = 64), and hlo / hhi the lane's partial h[l % 32] /
// h[32 + l % 32] (add lanes l and l ^ 32).
// Chunks of 32 entries go through LDS: the rows are loaded in 16-byte pieces
// (KP / 8 lanes per row, so a few wide loads per lane instead of one 2-byte
// load per element), entries past the end are staged as zero rows, and each
// lane then reads its MFMA operand (component l % 32 of 8 entries) from LDS.
// The next chunk's indices are loaded before this chunk's arithmetic; loads
// are unconditional (addresses clamped to the last entry).
template <int KP>
__device__ __forceinline__ void mfma_gram(const uint16_t *other, int ks, const int32_t *idx,
                                          const float *val, int64_t b0, int64_t b1, int lane,
                                          uint16_t *stage, f32x16_t &c00, f32x16_t &c10,
                                          f32x16_t &c11, float &hlo, float &hhi) {
    constexpr int LDR = KP + 8;             // staged row stride (elements)
    constexpr int LPR = KP / 8;             // lanes per row, one 16-byte piece each
    constexpr int RPI = 64 / LPR;           // rows per load instruction
    constexpr int NLD = 32 / RPI;           // load instructions per chunk
    float *sval = reinterpret_cast<float *>(stage + 32 * LDR);
    const int col = lane & 31;
    const int kg = (lane >> 5) * 8;
    const int rsub = lane / LPR, piece = lane - rsub * LPR;
    const int64_t last = b1 > b0 ? b1 - 1 : b0;
    int dq[NLD];
#pragma unroll
    for (int t = 0; t < NLD; ++t) dq[t] = b1 > b0 ? idx[min(b0 + rsub + RPI * t, last)] : 0;
    for (int64_t c0 = b0; c0 < b1; c0 += 32) {
        uint4 rw[NLD];
#pragma unroll
        for (int t = 0; t < NLD; ++t)
            rw[t] = *reinterpret_cast<const uint4 *>(other + (int64_t)dq[t] * ks + 8 * piece);
        const float vv = val[min(c0 + col, last)];
        const int64_t cn = c0 + 32;
#pragma unroll
        for (int t = 0; t < NLD; ++t) dq[t] = idx[min(cn + rsub + RPI * t, last)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NLD; ++t) {
            const int r = rsub + RPI * t;
            const uint4 v = c0 + r < b1 ? rw[t] : make_uint4(0u, 0u, 0u, 0u);
            *reinterpret_cast<uint4 *>(stage + r * LDR + 8 * piece) = v;
        }
        if (lane < 32) sval[lane] = c0 + lane < b1 ? vv : 0.0f;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            u16x8_t lo, hi;
            float rr[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int r = 16 * u + kg + j;
                lo[j] = stage[r * LDR + col];
                if constexpr (KP == 64) hi[j] = stage[r * LDR + 32 + col];
                rr[j] = sval[r];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                hlo += rr[j] * bf16_to_f32(lo[j]);
                if constexpr (KP == 64) hhi += rr[j] * bf16_to_f32(hi[j]);
            }
            const bf16x8_t blo = __builtin_bit_cast(bf16x8_t, lo);
            c00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(blo, blo, c00, 0, 0, 0);
            if constexpr (KP == 64) {
                const bf16x8_t bhi = __builtin_bit_cast(bf16x8_t, hi);
                c10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bhi, blo, c10, 0, 0, 0);
                c11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bhi, bhi, c11, 0, 0, 0);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    hlo = bfly_step<32>(hlo);
    hhi = bfly_step<32>(hhi);
}

// Store the accumulators of mfma_gram: lower blocks of G at dst[row * ld + col],
// h at rhs[0..KP).
template <int KP, typename T>
__device__ __forceinline__ void store_gram(T *dst, int ld, T *rhs, int lane, const f32x16_t &c00,
                                           const f32x16_t &c10, const f32x16_t &c11, float hlo,
                                           float hhi) {
    const int col = lane & 31;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        dst[row * ld + col] = (T)c00[v];
        if constexpr (KP == 64) {
            dst[(32 + row) * ld + col] = (T)c10[v];
            dst[(32 + row) * ld + 32 + col] = (T)c11[v];
        }
    }
    if (lane < 32) {
        rhs[col] = (T)hlo;
        if constexpr (KP == 64) rhs[32 + col] = (T)hhi;
    }
}

// Partial Gram of one heavy-entity segment per wavefront.
template <int KP>
__global__ __launch_bounds__(64) void k_gram_part(const GramPartArgs a) {
    const SegItem sg = a.segs[blockIdx.x];
    const SideDesc &sd = a.sides[sg.side];
    const uint16_t *other = reinterpret_cast<const uint16_t *>(a.other) + sd.other_off * a.ks_other;
    __shared__ __align__(16) uint16_t stage[gram_stage_bytes<KP>() / 2];
    f32x16_t c00 = {}, c10 = {}, c11 = {};
    float hlo = 0.0f, hhi = 0.0f;
    mfma_gram<KP>(other, a.ks_other, a.idx, reinterpret_cast<const float *>(a.val), sg.begin, sg.end,
                  threadIdx.x, stage, c00, c10, c11, hlo, hhi);
    float *dst = a.gpart + (int64_t)sg.slot * (KP * KP + KP);
    store_gram<KP, float>(dst, KP, dst + KP * KP, threadIdx.x, c00, c10, c11, hlo, hhi);
}

// MF: accumulate the Gram with v_mfma_f32_32x32x16_bf16 (BF16 state, KP = 32
// or 64).  Lane l loads component l mod 32 (and 32 + l mod 32) of the factor
// rows of 8 of every 16 observed entries: the same register is the A operand
// (rows of W^T) and the B operand (columns of W), and the 32x32 FP32
// accumulators hold G = W^T W (blocks G00, G10, G11 when KP = 64).
template <int KP, int P, bool MF>
__global__ __launch_bounds__(64) void k_update_wave(const UpdArgs a) {
    using Tacc = typename PrecT<P>::acc;
    using Tw = typename PrecT<P>::w;
    using Tv = typename PrecT<P>::v;
    using Ts = typename PrecT<P>::s;
    using Tp = typename PrecT<P>::p;
    constexpr int TL = KP / 8;
    constexpr int CH = 32;
    constexpr int LD = KP + 1;                       // A: odd stride, conflict-free rows
    constexpr int LDL = KP + 16 / (int)sizeof(Tacc); // L: 16-byte rows for broadcast loads
    __shared__ __align__(16) Tacc sA[KP * LDL];
    // the VALU Gram stages its chunks in sA when they fit (the Gram is held in
    // registers until the chunks are done): less LDS, more waves per CU
    constexpr bool kSwInA = CH * KP <= KP * LDL;
    __shared__ Tacc swbuf[MF || kSwInA ? 1 : CH * KP];
    Tacc *const sw = kSwInA ? sA : swbuf;
    __shared__ Tacc sr[MF ? 1 : CH];
    __shared__ Tacc sh[KP];
    __shared__ Tacc sz[KP];
    __shared__ Tacc sd0[KP];
    __shared__ Tacc sinv[KP];
    __shared__ Tacc shraw[KP];                    // sum r w of the entity (column SSE)

    const int K = a.K;
    const int nitems = a.nitems_dev ? *a.nitems_dev : a.nitems;
    uint32_t t_sw = a.t;
    void *sample = a.sample;
    if (a.ss) {
        t_sw = a.ss->t;
        sample = a.ss->slot >= 0 ? reinterpret_cast<char *>(a.sample) + a.ss->slot * a.ss->slot_bytes : nullptr;
    }
    const Tw *otherb = reinterpret_cast<const Tw *>(a.other);
    const Tv *val = reinterpret_cast<const Tv *>(a.val);

    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        // an opaque lane index per item: lane-derived addresses and masks are
        // recomputed for each item instead of being hoisted out of the loop
        // and held in registers across all of it
        int lane = threadIdx.x;
        asm volatile("" : "+v"(lane));
        const int ti = lane >> 3, tj = lane & 7;
        const int2 item = a.items[it];
        const SideDesc &sd = a.sides[item.x];
        const int n = item.y;
        const int64_t p0 = a.ptr[sd.ptr_off + n];
        const int64_t p1 = a.ptr[sd.ptr_off + n + 1];
        const Tw *other = otherb + sd.other_off * a.ks_other;

        if constexpr (MF) {
            const int2 sp = a.splits ? a.splits[it] : make_int2(0, 0);
            __syncthreads();
            if (sp.y > 0) {
                // heavy entity: sum the segments' partial Grams in segment order
                constexpr int PS = KP * KP + KP;
                const float *base = a.gpart + (int64_t)sp.x * PS;
                for (int q = lane; q < KP * KP + KP; q += 64) {
                    const int ra = q / KP, cb = q - ra * KP;
                    if (q < KP * KP && (cb > ra || (KP == 64 && ra < 32 && cb >= 32))) continue;
                    float v = 0.0f;
                    for (int g2 = 0; g2 < sp.y; ++g2) v += base[(int64_t)g2 * PS + q];
                    if (q < KP * KP) sA[ra * LD + cb] = v;
                    else sh[q - KP * KP] = v;
                }
            } else {
                f32x16_t c00 = {}, c10 = {}, c11 = {};
                float hlo = 0.0f, hhi = 0.0f;
                // the Gram's LDS is free until store_gram: it stages the chunks
                static_assert(gram_stage_bytes<KP>() <= (int)sizeof(Tacc) * KP * LDL, "stage fits sA");
                mfma_gram<KP>(reinterpret_cast<const uint16_t *>(other), a.ks_other, a.idx,
                              reinterpret_cast<const float *>(val), p0, p1, lane,
                              reinterpret_cast<uint16_t *>(sA), c00, c10, c11, hlo, hhi);
                __builtin_amdgcn_wave_barrier();
                store_gram<KP, Tacc>(sA, LD, sh, lane, c00, c10, c11, hlo, hhi);
            }
        } else {
            Tacc acc[TL][TL];
            Tacc hacc[TL];
    #pragma unroll
            for (int i = 0; i < TL; ++i) {
                hacc[i] = 0;
    #pragma unroll
                for (int j = 0; j < TL; ++j) acc[i][j] = 0;
            }
            for (int64_t c0 = p0; c0 < p1; c0 += CH) {
                const int nc = (int)((p1 - c0) < CH ? (p1 - c0) : CH);
                __syncthreads();
                for (int q = lane; q < CH * KP; q += 64) {
                    const int nz = q / KP, k = q - nz * KP;
                    Tacc v = 0;
                    if (nz < nc && k < K) v = to_acc<Tacc>(other[(int64_t)a.idx[c0 + nz] * a.ks_other + k]);
                    sw[q] = v;
                }
                if (lane < CH) sr[lane] = lane < nc ? (Tacc)val[c0 + lane] : (Tacc)0;
                __syncthreads();
                for (int nz = 0; nz < nc; ++nz) {
                    Tacc wi[TL], wj[TL];
    #pragma unroll
                    for (int i = 0; i < TL; ++i) {
                        wi[i] = sw[nz * KP + ti * TL + i];
                        wj[i] = sw[nz * KP + tj * TL + i];
                    }
    #pragma unroll
                    for (int i = 0; i < TL; ++i)
    #pragma unroll
                        for (int j = 0; j < TL; ++j) acc[i][j] += wi[i] * wj[j];
                    if (tj == 0) {
                        const Tacc r = sr[nz];
    #pragma unroll
                        for (int i = 0; i < TL; ++i) hacc[i] += r * wi[i];
                    }
                }
            }
            __syncthreads();
            // the raw Gram and right-hand side, for the prior pass below
    #pragma unroll
            for (int i = 0; i < TL; ++i)
    #pragma unroll
                for (int j = 0; j < TL; ++j) sA[(ti * TL + i) * LD + tj * TL + j] = acc[i][j];
            if (tj == 0) {
    #pragma unroll
                for (int i = 0; i < TL; ++i) sh[ti * TL + i] = hacc[i];
            }
        }
        __syncthreads();
        const Tacc tau = (Tacc)sd.tau[(int64_t)sd.tau_stride * n];
        const double *pr = sd.prior + (sd.per_row ? (int64_t)n * a.prow : 0);
        const double *pv = pr + K * (K + 1) / 2;
        // packed lower prior, lanes over consecutive entries (coalesced), all
        // loads issued before the first use.  Row of entry q: the floor of
        // (sqrt(8q + 1) - 1) / 2, which is an integer at the start of a row
        // and at least 2 / (2 row + 3) > 0.015 below the next integer
        // elsewhere (row < 64), so an approximate square root plus 1e-3
        // floors to the right row
        const int npk = K * (K + 1) / 2;
        constexpr int NQ = (KP * (KP + 1) / 2 + 63) / 64;
        constexpr int CQ = 8;                            // loads in flight per chunk
#pragma unroll
        for (int u0 = 0; u0 < NQ; u0 += CQ) {
            double pq[CQ];
#pragma unroll
            for (int u = 0; u < CQ; ++u) {
                const int q = lane + 64 * (u0 + u);
                pq[u] = (u0 + u < NQ && q < npk) ? pr[q] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CQ; ++u) {
                const int q = lane + 64 * (u0 + u);
                if (u0 + u < NQ && q < npk) {
                    const int ra = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f + 1e-3f);
                    const int cb = q - ra * (ra + 1) / 2;
                    sA[ra * LD + cb] = (Tacc)pq[u] + tau * sA[ra * LD + cb];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // identity padding rows K..KP-1
        for (int q = lane; q < (KP - K) * KP; q += 64) {
            const int ra = K + q / KP, cb = q % KP;
            if (cb <= ra) sA[ra * LD + cb] = (Tacc)(ra == cb);
        }
        for (int q = lane; q < KP; q += 64) {
            shraw[q] = sh[q];
            sh[q] = q < K ? (Tacc)pv[q] + tau * sh[q] : (Tacc)0;
        }
        if (lane * 4 < K) {
            Tacc z[4];
            normals4((uint32_t)n, t_sw, sd.c2, (uint32_t)lane, a.k0, a.k1, z);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (4 * lane + c < K) sz[4 * lane + c] = z[c];
        }
        if (lane >= K && lane < KP) sz[lane] = (Tacc)0;
        __syncthreads();
        if (lane < KP) sd0[lane] = sA[lane * LD + lane];
        __syncthreads();
        const bool ok = factor_solve_regs<KP, Tacc>(sA, LD, sA, LDL, sh, sz, sd0, sinv, (Tacc)a.theta, K, lane);
        if (!ok) {
            if (lane == 0) {
                if (a.fb_list) {
                    const int slot = atomicAdd(a.fb_count, 1);
                    a.fb_list[slot] = make_int2(item.x, n);
                    atomicAdd(a.fb_total, 1);
                } else {
                    atomicAdd(a.nonpd, 1);
                }
            }
            continue;
        }
        const Tacc xv = lane < K ? sh[lane] : (Tacc)0;
        Ts *self = reinterpret_cast<Ts *>(a.self);
        if (lane < a.ks_self) self[(sd.self_off + n) * a.ks_self + lane] = elem_from<Ts>((double)xv);
        if (sample && lane < a.ks_sample)
            reinterpret_cast<Tp *>(sample)[(sd.sample_off + n) * a.ks_sample + lane] = (Tp)xv;
        if (a.sse_col) {
            // Residual SSE of this column with the new w as stored, from the sums
            // of this pass: sum r^2 - 2 w.h_raw + (|L^T w|^2 - w^T P w) / tau
            // (A = P + tau G_raw = L L^T), in FP64.
            __syncthreads();
            if (lane < KP) sz[lane] = lane < K ? (Tacc)elem_to_d(elem_from<Ts>((double)xv)) : (Tacc)0;
            __syncthreads();
            const double tauv = (double)tau;                 // the tau that scaled A
            double acc = 0.0;
            if (lane < KP) {
                // (L^T w)_lane = sum_{p >= lane} L_p,lane w_p (L in sA, row stride LDL)
                double u = 0.0;
                for (int p = lane; p < KP; ++p) u += (double)sA[p * LDL + lane] * (double)sz[p];
                acc = u * u - 2.0 * tauv * (double)shraw[lane] * (double)sz[lane];
            }
            // w^T P w over the packed prior (coalesced), off-diagonal entries twice
            const double *prs = sd.prior + (sd.per_row ? (int64_t)n * a.prow : 0);
            for (int q = lane; q < K * (K + 1) / 2; q += 64) {
                const int ra = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f + 1e-3f);
                const int cb = q - ra * (ra + 1) / 2;
                acc -= (ra == cb ? 1.0 : 2.0) * prs[q] * (double)sz[ra] * (double)sz[cb];
            }
            acc = group_sum1(acc, 64);
            if (lane < 4)
                a.sse_col[4 * (sd.self_off + n) + lane] = lane == 0 ? a.colsq[sd.self_off + n] + acc / tauv : 0.0;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// k_update_duo: two entities per wavefront (16 < K <= 32, FP32 arithmetic).
// Lanes 32h .. 32h + 31 hold entity h: lane r owns row r of its factor and of
// its solves, so the factorisation steps, which leave half of a wavefront
// idle at one entity per wavefront, serve two.  The Gram: MF = false, lane r
// forms row r of its entity's Gram on the VALU, for entities with at most
// kDuoNnz entries (their rows are staged in LDS at once); MF = true (BF16
// state), the whole wavefront forms the two Grams one after the other with
// mfma_gram (or sums a heavy entity's partial Grams), any number of entries.
// --------------------------------------------------------------------------
constexpr int kDuoNnz = 16;

// Value of lane 32h + q for the lanes of half h (q uniform; hb = 128 h, the
// byte address of the half's first lane): one cross-lane permute.
__device__ __forceinline__ float half_bcast(float v, int q, int hb) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(hb + 4 * q, __float_as_int(v)));
}

template <int P, bool MF>
__global__ __launch_bounds__(64) void k_update_duo(const UpdArgs a) {
    using Tacc = typename PrecT<P>::acc;
    using Tw = typename PrecT<P>::w;
    using Tv = typename PrecT<P>::v;
    using Ts = typename PrecT<P>::s;
    using Tp = typename PrecT<P>::p;
    static_assert(sizeof(Tacc) == 4, "FP32 arithmetic");
    constexpr int KP = 32;
    constexpr int LDL = KP + 4;                      // 16-byte rows for broadcast loads
    constexpr int CH = kDuoNnz;
    static_assert(CH * KP <= KP * LDL, "staged rows fit the Gram's LDS");
    static_assert(!MF || P == kPBF, "the MFMA Gram reads BF16 factors");
    static_assert(gram_stage_bytes<KP>() <= (int)sizeof(Tacc) * KP * LDL, "MFMA staging fits");
    __shared__ __align__(16) Tacc sA[2 * KP * LDL];  // per entity: staged rows, then A, then L
    __shared__ Tacc sr[2 * CH];
    __shared__ Tacc sh[2 * KP];
    __shared__ Tacc shraw[2 * KP];
    __shared__ Tacc sz[2 * KP];
    __shared__ Tacc sinv[2 * KP];

    const int K = a.K;
    const int nitems = a.nitems_dev ? *a.nitems_dev : a.nitems;
    uint32_t t_sw = a.t;
    void *sample = a.sample;
    if (a.ss) {
        t_sw = a.ss->t;
        sample = a.ss->slot >= 0 ? reinterpret_cast<char *>(a.sample) + a.ss->slot * a.ss->slot_bytes : nullptr;
    }
    const Tw *otherb = reinterpret_cast<const Tw *>(a.other);
    const Tv *val = reinterpret_cast<const Tv *>(a.val);

    for (int pit = blockIdx.x; 2 * pit < nitems; pit += gridDim.x) {
        int lane = threadIdx.x;
        asm volatile("" : "+v"(lane));
        const int h = lane >> 5, r = lane & 31;
        const int it = 2 * pit + h;
        const bool valid = it < nitems;             // uniform per half
        const int2 item = a.items[valid ? it : 2 * pit];
        const SideDesc &sd = a.sides[item.x];
        const int n = item.y;
        const int64_t p0 = a.ptr[sd.ptr_off + n];
        const int deg = (int)(a.ptr[sd.ptr_off + n + 1] - p0);
        const bool fits = MF || deg <= CH;           // else: the FP64 redo takes it
        const int nc = fits ? deg : 0;
        const Tw *other = otherb + sd.other_off * a.ks_other;
        Tacc *A = sA + h * (KP * LDL);
        Tacc *rv = sr + h * CH;
        Tacc *hh = sh + h * KP, *hr = shraw + h * KP, *zz = sz + h * KP, *iv = sinv + h * KP;

        __syncthreads();                             // the previous pair is done with the LDS
        Tacc hs = (Tacc)0;
        if constexpr (MF) {
            // the two Grams, one after the other, by the whole wavefront (the
            // chunks are staged in the second entity's A, which its own Gram
            // overwrites only after its last chunk is read)
            // both entities' rows, entry ranges and segment splits first, so
            // that the second's loads overlap the first's Gram
            int2 sps[2];
            int64_t q0s[2], q1s[2];
            const Tw *oth[2];
#pragma unroll
            for (int hq = 0; hq < 2; ++hq) {
                const int itq = 2 * pit + hq < nitems ? 2 * pit + hq : 2 * pit;
                const int2 iq = a.items[itq];
                const SideDesc &sq = a.sides[iq.x];
                sps[hq] = a.splits ? a.splits[itq] : make_int2(0, 0);
                q0s[hq] = a.ptr[sq.ptr_off + iq.y];
                q1s[hq] = a.ptr[sq.ptr_off + iq.y + 1];
                oth[hq] = otherb + sq.other_off * a.ks_other;
            }
            for (int hq = 0; hq < 2; ++hq) {
                Tacc *Aq = sA + hq * (KP * LDL);
                Tacc *hq_ = sh + hq * KP;
                const int2 sp = sps[hq];
                if (sp.y > 0) {
                    // heavy entity: sum its segments' partial Grams in segment order
                    constexpr int PS = KP * KP + KP;
                    const float *base = a.gpart + (int64_t)sp.x * PS;
                    for (int q = lane; q < PS; q += 64) {
                        const int ra = q / KP, cb = q - ra * KP;
                        if (q < KP * KP && cb > ra) continue;
                        float v = 0.0f;
                        for (int g2 = 0; g2 < sp.y; ++g2) v += base[(int64_t)g2 * PS + q];
                        if (q < KP * KP) Aq[ra * LDL + cb] = v;
                        else hq_[q - KP * KP] = v;
                    }
                } else {
                    f32x16_t c00 = {}, c10 = {}, c11 = {};
                    float hlo = 0.0f, hhi = 0.0f;
                    mfma_gram<KP>(reinterpret_cast<const uint16_t *>(oth[hq]),
                                  a.ks_other, a.idx, reinterpret_cast<const float *>(val), q0s[hq], q1s[hq], lane,
                                  reinterpret_cast<uint16_t *>(sA + KP * LDL), c00, c10, c11, hlo, hhi);
                    __builtin_amdgcn_wave_barrier();
                    store_gram<KP, Tacc>(Aq, LDL, hq_, lane, c00, c10, c11, hlo, hhi);
                }
                __syncthreads();
            }
            hs = hh[r];
        } else {
        // the entity's rows (zero beyond K) and values, staged in its A
        for (int q = r; q < nc * KP; q += 32) {
            const int e = q / KP, k = q - e * KP;
            A[q] = k < K ? to_acc<Tacc>(other[(int64_t)a.idx[p0 + e] * a.ks_other + k]) : (Tacc)0;
        }
        if (r < CH) rv[r] = r < nc ? (Tacc)val[p0 + r] : (Tacc)0;
        __syncthreads();
        // row r of the Gram and entry r of the right-hand side
        Tacc g[KP];
#pragma unroll
        for (int c = 0; c < KP; ++c) g[c] = (Tacc)0;
        for (int e = 0; e < nc; ++e) {
            const Tacc *we = A + e * KP;
            const Tacc wr = we[r];
#pragma unroll
            for (int c = 0; c < KP; ++c) g[c] += wr * we[c];
            hs += rv[e] * wr;
        }
        __syncthreads();                             // staged rows read
#pragma unroll
        for (int c = 0; c < KP; ++c) A[r * LDL + c] = g[c];
        hh[r] = hs;
        __syncthreads();
        }
        // A = P + tau G, h = P m + tau hs: the packed prior, coalesced over the
        // half's lanes (row of entry q as in the wave kernel)
        const Tacc tau = (Tacc)sd.tau[(int64_t)sd.tau_stride * n];
        const double *pr = sd.prior + (sd.per_row ? (int64_t)n * a.prow : 0);
        const int npk = K * (K + 1) / 2;
        constexpr int NQ = (KP * (KP + 1) / 2 + 31) / 32;
        constexpr int CQ = 9;
#pragma unroll
        for (int u0 = 0; u0 < NQ; u0 += CQ) {
            double pq[CQ];
#pragma unroll
            for (int u = 0; u < CQ; ++u) {
                const int q = r + 32 * (u0 + u);
                pq[u] = (u0 + u < NQ && q < npk) ? pr[q] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CQ; ++u) {
                const int q = r + 32 * (u0 + u);
                if (u0 + u < NQ && q < npk) {
                    const int ra = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f + 1e-3f);
                    const int cb = q - ra * (ra + 1) / 2;
                    A[ra * LDL + cb] = (Tacc)pq[u] + tau * A[ra * LDL + cb];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (r >= K) {
            // identity padding row
#pragma unroll
            for (int c = 0; c < KP; ++c)
                if (c <= r) A[r * LDL + c] = (Tacc)(c == r);
        }
        hr[r] = hs;
        hh[r] = r < K ? (Tacc)pr[npk + r] + tau * hs : (Tacc)0;
        if (r * 4 < K) {
            Tacc z[4];
            normals4((uint32_t)n, t_sw, sd.c2, (uint32_t)r, a.k0, a.k1, z);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (4 * r + c < K) zz[4 * r + c] = z[c];
        }
        if (r >= K) zz[r] = (Tacc)0;
        __syncthreads();

        // left-looking Cholesky, row r in registers, rows of L broadcast from LDS
        // (L overlays A: every row is read before the first write).  Each phase
        // derives its lane masks from a fresh opaque lane index, so that none is
        // kept live (in scalar registers) across phases.
        asm volatile("" : "+v"(lane));
        Tacc rr[KP];
        bool ok;
        {
        const int r = lane & 31, h = lane >> 5;
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const Tacc v = A[r * LDL + j];
            rr[j] = j <= r ? v : (Tacc)0;
            asm volatile("" : "+v"(rr[j]));
        }
        const Tacc d0 = A[r * LDL + r];
        __syncthreads();
        int mybad = 0;
        Tacc myinv = (Tacc)1;
        const Tacc theta = (Tacc)a.theta;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            Tacc s0 = rr[k], s1 = (Tacc)0;
            const Tacc *lk = A + k * LDL;
#pragma unroll
            for (int p = 0; p < k; ++p) {
                if (p & 1) s1 -= rr[p] * lk[p];
                else s0 -= rr[p] * lk[p];
                if ((p & 15) == 15) __builtin_amdgcn_sched_barrier(0);
            }
            const Tacc sk = s0 + s1;
            const Tacc dk = half_bcast(sk, k, 128 * h);
            mybad = r == k ? (int)!(sk > theta * d0) : mybad;
            Tacc lkk, inv;
            pivot_of(dk > (Tacc)0 ? dk : (Tacc)1, lkk, inv);
            myinv = r == k ? inv : myinv;
            rr[k] = r == k ? lkk : sk * inv;
            A[r * LDL + k] = rr[k];
            __builtin_amdgcn_wave_barrier();
            asm volatile("" : "+v"(rr[k]), "+v"(myinv), "+v"(mybad));
            __builtin_amdgcn_sched_barrier(0);
        }
        iv[r] = myinv;
        const uint64_t bad = __ballot(mybad);
        ok = fits && ((bad >> (32 * h)) & 0xFFFFFFFFull) == 0;
        __syncthreads();
        asm volatile("" : "+v"(lane));
        }
        const int r2 = lane & 31, h2 = lane >> 5;
        // y = L^-1 h; v = y + z; x = L^-T v (columns of L read from LDS)
        Tacc acc = hh[r2], y = (Tacc)0;
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const Tacc yq = half_bcast(acc, q, 128 * h2) * iv[q];
            y = r2 == q ? yq : y;
            acc = r2 > q ? acc - rr[q] * yq : acc;
        }
        const Tacc v = r2 < K ? y + zz[r2] : (Tacc)0;
        asm volatile("" : "+v"(lane));
        const int r3 = lane & 31, h3 = lane >> 5;
        Tacc cc[KP];
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const Tacc v2 = A[q * LDL + r3];
            cc[q] = q >= r3 ? v2 : (Tacc)0;
            asm volatile("" : "+v"(cc[q]));
        }
        acc = v;
        Tacc x = (Tacc)0;
#pragma unroll
        for (int q = KP - 1; q >= 0; --q) {
            const Tacc xq = half_bcast(acc, q, 128 * h3) * iv[q];
            x = r3 == q ? xq : x;
            acc = r3 < q ? acc - cc[q] * xq : acc;
        }
        if (valid && !ok) {
            if (r == 0) {
                if (a.fb_list) {
                    const int slot = atomicAdd(a.fb_count, 1);
                    a.fb_list[slot] = make_int2(item.x, n);
                    atomicAdd(a.fb_total, 1);
                } else {
                    atomicAdd(a.nonpd, 1);
                }
            }
        }
        const bool wr = valid && ok;
        const Tacc xv = r < K ? x : (Tacc)0;
        Ts *self = reinterpret_cast<Ts *>(a.self);
        if (wr && r < a.ks_self) self[(sd.self_off + n) * a.ks_self + r] = elem_from<Ts>((double)xv);
        if (wr && sample && r < a.ks_sample)
            reinterpret_cast<Tp *>(sample)[(sd.sample_off + n) * a.ks_sample + r] = (Tp)xv;
        if (a.sse_col) {
            // the column's residual SSE in closed form (as in the wave kernel), FP64
            __syncthreads();
            zz[r] = r < K ? (Tacc)elem_to_d(elem_from<Ts>((double)xv)) : (Tacc)0;
            __syncthreads();
            const double tauv = (double)tau;
            double u = 0.0;
            for (int p = r; p < KP; ++p) u += (double)A[p * LDL + r] * (double)zz[p];
            double sacc = u * u - 2.0 * tauv * (double)hr[r] * (double)zz[r];
            for (int q = r; q < npk; q += 32) {
                const int ra = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f + 1e-3f);
                const int cb = q - ra * (ra + 1) / 2;
                sacc -= (ra == cb ? 1.0 : 2.0) * pr[q] * (double)zz[ra] * (double)zz[cb];
            }
            sacc = group_sum1(sacc, 32);
            if (wr && r < 4)
                a.sse_col[4 * (sd.self_off + n) + r] = r == 0 ? a.colsq[sd.self_off + n] + sacc / tauv : 0.0;
        }
    }
}

// --------------------------------------------------------------------------
// The low-rank update of an entity with 1 .. kLowRankNnz entries under a
// propagated per-row prior whose factor U = L_P^-T (Lambda = L_P L_P^T) was
// computed at stage begin.  With v_e = L_P^-1 w_e,
//     A = Lambda + tau sum_e w_e w_e^T = L_P (I + tau sum_e v_e v_e^T) L_P^T,
// and the Cholesky factor of A is L_P M_1 ... M_nc with M_e the factor of the
// rank-one modification I + tau u_e u_e^T, u_e = (M_1 ... M_(e-1))^-1 v_e (the
// product form of Gill, Golub, Murray and Saunders, 1974).  With
// t_j = 1 + tau sum_(i<=j) u_i^2 (t_-1 = 1), M has diagonal sqrt(t_j / t_(j-1))
// and entries tau u_i u_j / sqrt(t_j t_(j-1)) below it, and its triangular
// solves reduce to one prefix (M^-1) or suffix (M^-T) sum each:
//     (M^-1 b)_j = (b_j - tau u_j P_j / t_(j-1)) / d_j,    P_j = sum_(i<j) u_i b_i,
//     (M^-T b)_j = (b_j - tau beta_j t_j S_j) / d_j,        S_j = sum_(i>j) u_i b_i / (d_i t_(i-1)),
// with beta_j = u_j / sqrt(t_j t_(j-1)).  The draw x = L^-T (L^-1 h + z) is then
// U (M_1^-T ... M_nc^-T (M_nc^-1 ... M_1^-1 U^T h + z)): the same factor
// and the same noise as the factorising kernels, at O(nc K) segment scans and
// nc + 2 triangular products instead of a K^3 / 3 factorisation.  64 / KP
// entities per wavefront; a half with fewer entries than the other applies
// identity factors (u = 0, which leave every value unchanged), so that every
// lane runs the same scans.  The column pass computes the residual SSE
// directly from the few entries.  An entity with no entries needs no update:
// its conditional precision is the prior's, A = Lambda, and A^-1 h = mu, so
// its draw is x = mu + U z.  An entity whose prior precision was not positive
// definite (flag at K(K+1)/2 of the factor row is 0) goes to the FP64 redo
// queue, as a failed factorisation would.
// --------------------------------------------------------------------------
constexpr int kLowRankNnz = 8;
constexpr int kLowRankSmall = 2;                 // a second instance for 1 .. 2 entries

// Cross-lane moves of the segment scans (GFX9 DPP; lanes without a source,
// and rows left out by the row mask, read 0).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp0(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float lane_f(float x, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
// Inclusive prefix sums within W-lane segments (W = 32 or 64): four row_shr
// steps inside each 16-lane row, then row_bcast:15 (rows 1, 3 take the last
// lane of rows 0, 2) and, for W = 64, row_bcast:31 (rows 2, 3 take lane 31).
template <int W>
__device__ __forceinline__ float seg_prefix(float x) {
    x += dpp0<0x111>(x);
    x += dpp0<0x112>(x);
    x += dpp0<0x114>(x);
    x += dpp0<0x118>(x);
    x += dpp0<0x142, 0xA>(x);
    if (W == 64) x += dpp0<0x143, 0xC>(x);
    return x;
}
// Inclusive suffix sums within W-lane segments: row_shl steps inside each row,
// then each row adds the totals of the later rows of its segment (their first
// lanes, read with v_readlane).
template <int W>
__device__ __forceinline__ float seg_suffix(float x, int lane) {
    x += dpp0<0x101>(x);
    x += dpp0<0x102>(x);
    x += dpp0<0x104>(x);
    x += dpp0<0x108>(x);
    const float s1 = lane_f(x, 16), s2 = lane_f(x, 32), s3 = lane_f(x, 48);
    const int row = lane >> 4;
    if (W == 32) return x + (row == 0 ? s1 : (row == 2 ? s3 : 0.0f));
    return x + (row == 0 ? s1 + s2 + s3 : (row == 1 ? s2 + s3 : (row == 2 ? s3 : 0.0f)));
}
// The value of lane - 1 (wave_shr:1) and of lane + 1 (wave_shl:1).
__device__ __forceinline__ float from_prev(float x) { return dpp0<0x138>(x); }
__device__ __forceinline__ float from_next(float x) { return dpp0<0x130>(x); }

// --------------------------------------------------------------------------
// k_update_group: the copies of one propagated row (or column) n in the
// sibling blocks of a stage -- the blocks whose prior for n is the same
// moment-matched row of the same source block (X rows of blocks (i, j), j > 0,
// from (i, 0); W columns of (i, j), i > 0, from (0, j)) -- that have at most
// kLowRankNnz entries in their block.  They share the prior's stored factor
// U = L^-T and its mean, so one wavefront expands U once into a dense LDS
// matrix and draws every copy from it, 64 / KP copies at a time: copies
// without entries as x = mu + U z, the others by the product-form rank-one
// update above.  The host orders a group's copies by entry count (none, one
// or two, three to eight), so the copies run side by side take the same
// number of scans, and the two short kinds run a two-vector form.  Lane l
// loads copy l's side, entry range and noise precision at the group's start;
// the lanes that update a copy take them by cross-lane reads.  Workgroups
// stride over the groups.  A copy's arithmetic does not depend on which copy
// runs beside it (a shorter partner applies identity factors), so per-block
// launches, whose groups hold one copy, give the same draws.
// --------------------------------------------------------------------------
// Products with the dense LDS copy of U (row r at r (KP + 4), so that the
// lanes' 16-byte row reads fall in distinct banks; zeros left of the
// diagonal and past K) and vectors that every lane of a half-wave reads by
// broadcast, four entries per read, summed in index order.  row_dot: lane r
// forms (U b)_r from its row; col_dots: lane c forms (U^T b_e)_c for NV
// vectors from its column, one read of U per entry for all of them.
template <int KP>
__device__ __forceinline__ float row_dot(const float *urow, const float *s) {
    const float4 *u4 = reinterpret_cast<const float4 *>(urow);
    const float4 *s4 = reinterpret_cast<const float4 *>(s);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < KP / 4; ++j) {
        const float4 u = u4[j], b = s4[j];
        acc += u.x * b.x;
        acc += u.y * b.y;
        acc += u.z * b.z;
        acc += u.w * b.w;
    }
    return acc;
}
template <int KP, int NV>
__device__ __forceinline__ void col_dots(const float *ucol, const float *const (&s)[NV], float (&acc)[NV]) {
    constexpr int UP = KP + 4;
#pragma unroll
    for (int j = 0; j < KP / 4; ++j) {
        const float u0 = ucol[(4 * j) * UP], u1 = ucol[(4 * j + 1) * UP];
        const float u2 = ucol[(4 * j + 2) * UP], u3 = ucol[(4 * j + 3) * UP];
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            const float4 b = reinterpret_cast<const float4 *>(s[e])[j];
            acc[e] += u0 * b.x;
            acc[e] += u1 * b.y;
            acc[e] += u2 * b.z;
            acc[e] += u3 * b.w;
        }
    }
}

template <int P, int KP, int NC>
__device__ __forceinline__ void group_lowrank_copy(
    const UpdArgs &a, const int sx, const int64_t p0, const int deg, const float tau, const bool valid,
    const int n, const float *ucol,
    const float *urow, const double *pr, float (&sw)[kLowRankNnz][KP], float (&sy)[kLowRankNnz],
    float (&sb)[KP], const float *sz, void *sample, const bool ok, const int lane) {
    using Tw = typename PrecT<P>::w;
    using Tv = typename PrecT<P>::v;
    using Ts = typename PrecT<P>::s;
    using Tp = typename PrecT<P>::p;
    const int r = lane % KP;
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    const SideDesc &sd = a.sides[sx];
    const int nc = valid && deg <= NC ? deg : 0;
    const Tw *other = reinterpret_cast<const Tw *>(a.other) + sd.other_off * a.ks_other;
    const Tv *val = reinterpret_cast<const Tv *>(a.val);
    // the entries' rows and values: loads from clamped (valid) positions, the
    // ones beyond the copy's entries masked, so that only one branch (on a
    // copy having entries at all) remains
    float wv[NC], yv = 0.0f;
#pragma unroll
    for (int e = 0; e < NC; ++e) wv[e] = 0.0f;
    if (nc > 0) {
        const int rr = min(r, K - 1);
#pragma unroll
        for (int e = 0; e < NC; ++e)
            wv[e] = to_acc<float>(other[(int64_t)a.idx[p0 + min(e, nc - 1)] * a.ks_other + rr]);
        yv = (float)val[p0 + min(r, nc - 1)];
    }
#pragma unroll
    for (int e = 0; e < NC; ++e) wv[e] = (e < nc && r < K) ? wv[e] : 0.0f;
    __syncthreads();                                 // the previous copies' LDS is read
#pragma unroll
    for (int e = 0; e < NC; ++e) sw[e][r] = wv[e];
    if (r < NC) sy[r] = r < nc ? yv : 0.0f;
    __syncthreads();
    // h = Lambda mu + tau sum_e y_e w_e
    float hs = 0.0f;
#pragma unroll
    for (int e = 0; e < NC; ++e) hs += sy[e] * wv[e];
    sb[r] = r < K ? (float)pr[kk2 + r] + tau * hs : 0.0f;
    int ncw = nc;
    if (64 / KP == 2) ncw = max(nc, __shfl_xor(nc, 32));
    __syncthreads();
    // y = U^T h and v_e = U^T w_e: lane c reads column c of U (zeros below
    // the diagonal) from LDS, the vectors by broadcast; a v_e past both
    // halves' entry counts is never used
    float y, v[NC];
    if (NC == kLowRankSmall || ncw > kLowRankNnz / 2) {
        const float *vs[NC + 1];
        float acc[NC + 1];
        vs[0] = sb;
        acc[0] = 0.0f;
#pragma unroll
        for (int e = 0; e < NC; ++e) {
            vs[e + 1] = sw[e];
            acc[e + 1] = 0.0f;
        }
        col_dots<KP, NC + 1>(ucol, vs, acc);
        y = acc[0];
#pragma unroll
        for (int e = 0; e < NC; ++e) v[e] = acc[e + 1];
    } else {
        constexpr int NH = NC > 1 ? NC / 2 : 1;
        const float *vs[NH + 1];
        float acc[NH + 1];
        vs[0] = sb;
        acc[0] = 0.0f;
#pragma unroll
        for (int e = 0; e < NH; ++e) {
            vs[e + 1] = sw[e];
            acc[e + 1] = 0.0f;
        }
        col_dots<KP, NH + 1>(ucol, vs, acc);
        y = acc[0];
#pragma unroll
        for (int e = 0; e < NC; ++e) v[e] = e < NH ? acc[e + 1] : 0.0f;
    }
    float fu[NC], ft[NC], fitm[NC], fid[NC];
#pragma unroll
    for (int e = 0; e < NC; ++e) {
        fu[e] = 0.0f;
        ft[e] = fitm[e] = fid[e] = 1.0f;
        if (e >= ncw) continue;
        const float u = v[e];
        const float t = 1.0f + tau * seg_prefix<KP>(u * u);
        const float tp = from_prev(t);
        const float itm = r == 0 ? 1.0f : __builtin_amdgcn_rcpf(tp);
        const float id = __builtin_amdgcn_rsqf(t * itm);
        fu[e] = u;
        ft[e] = t;
        fitm[e] = itm;
        fid[e] = id;
        {
            const float pp = from_prev(seg_prefix<KP>(u * y));
            const float pe = r == 0 ? 0.0f : pp;
            y = (y - tau * u * pe * itm) * id;
        }
#pragma unroll
        for (int f = e + 1; f < NC; ++f) {
            if (f >= ncw) continue;
            const float pp = from_prev(seg_prefix<KP>(u * v[f]));
            const float pe = r == 0 ? 0.0f : pp;
            v[f] = (v[f] - tau * u * pe * itm) * id;
        }
    }
    y += r < K ? sz[r] : 0.0f;
#pragma unroll
    for (int e = NC - 1; e >= 0; --e) {
        if (e >= ncw) continue;
        const float u = fu[e], t = ft[e], itm = fitm[e], id = fid[e];
        const float sn = from_next(seg_suffix<KP>(u * y * id * itm, lane));
        const float se = r == KP - 1 ? 0.0f : sn;
        y = (y - tau * u * id * itm * t * se) * id;
    }
    __syncthreads();                                 // h is read
    sb[r] = r < K ? y : 0.0f;
    __syncthreads();
    // x = U y: lane r holds row r of U (zeros left of the diagonal)
    const float acc = row_dot<KP>(urow, sb);
    const float xv = r < K ? acc : 0.0f;
    const bool wr = valid && ok;
    Ts *self = reinterpret_cast<Ts *>(a.self);
    if (wr && r < a.ks_self) self[(sd.self_off + n) * a.ks_self + r] = elem_from<Ts>((double)xv);
    if (wr && sample && r < a.ks_sample)
        reinterpret_cast<Tp *>(sample)[(sd.sample_off + n) * a.ks_sample + r] = (Tp)xv;
    if (a.sse_col) {
        // residual SSE over the entries, FP64, from the state-rounded draw
        __syncthreads();
        sb[r] = r < K ? (float)elem_to_d(elem_from<Ts>((double)xv)) : 0.0f;
        __syncthreads();
        double res = 0.0;
        if (r < nc) {
            double dot = 0.0;
            for (int k = 0; k < K; ++k) dot += (double)sb[k] * (double)sw[r][k];
            res = (double)sy[r] - dot;
            res *= res;
        }
#pragma unroll
        for (int o = 1; o < NC; o <<= 1) res += __shfl_down(res, o, KP);
        if (wr && r < 4) a.sse_col[4 * (sd.self_off + n) + r] = r == 0 ? res : 0.0;
    }
}

template <int P, int KP>
__global__ __launch_bounds__(64, KP <= 32 ? 4 : 2) void k_update_group(const UpdArgs a) {
    using Ts = typename PrecT<P>::s;
    using Tp = typename PrecT<P>::p;
    constexpr int G = 64 / KP;
    constexpr int WIN = 8;                           // copies whose noise is drawn together
    constexpr int LPC = KP / 4;                      // lanes per copy in a draw (4 normals each)
    constexpr int CPD = 64 / LPC;                    // copies per draw
    static_assert(WIN % G == 0 && WIN % CPD == 0, "whole copies per window");
    constexpr int UP = KP + 4;                       // padded row stride of the dense copy of U
    constexpr int NQ = (KP * (KP + 1) / 2 + 63) / 64;  // stored entries per lane
    __shared__ __align__(16) float ud[KP * UP];      // ud[r][j] = U[r][j] (zero left of the diagonal)
    __shared__ unsigned short dmap[NQ * 64];         // where stored entry q goes in ud (0xFFFF: none)
    __shared__ __align__(16) float sw[G][kLowRankNnz][KP];  // a copy's entries' rows of the other side
    __shared__ float sy[G][kLowRankNnz];             // their values
    __shared__ __align__(16) float sb[G][KP];        // right-hand side, then the solved vector
    __shared__ __align__(16) float sz[WIN][KP];      // noise of the window's copies
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    uint32_t t_sw = a.t;
    void *sample = a.sample;
    if (a.ss) {
        t_sw = a.ss->t;
        sample = a.ss->slot >= 0 ? reinterpret_cast<char *>(a.sample) + a.ss->slot * a.ss->slot_bytes : nullptr;
    }
    Ts *self = reinterpret_cast<Ts *>(a.self);
    const int lane = threadIdx.x;
    const int h = lane / KP, r = lane % KP;
    for (int q = lane; q < KP * UP; q += 64) ud[q] = 0.0f;
    // the stored factor holds diagonal d (entries U[p][p + d], p < K - d) from
    // offset d K - d (d - 1) / 2: where each of this lane's entries goes in ud
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = lane + 64 * i;
        const float fq = (float)(2 * K + 1);
        int d = (int)((fq - sqrtf(fmaxf(fq * fq - 8.0f * (float)q, 0.0f))) * 0.5f);
        d = max(0, min(d, K - 1));
        if ((d + 1) * K - (d + 1) * d / 2 <= q) ++d;
        if (d * K - d * (d - 1) / 2 > q) --d;
        const int p = q - (d * K - d * (d - 1) / 2);
        dmap[q] = q < kk2 ? (unsigned short)(p * UP + p + d) : (unsigned short)0xFFFF;
    }
    for (int g = blockIdx.x; g < a.ngroups; g += gridDim.x) {
        const int i0 = a.gstart[g];
        const int cnt = a.gstart[g + 1] - i0;        // copies in the group (at most 64)
        const int2 first = a.items[i0];
        const SideDesc &sd0 = a.sides[first.x];
        const int n = first.y;
        const float *pf = sd0.pfac + (int64_t)n * a.pfrow;
        const double *pr = sd0.prior + (int64_t)n * a.prow;
        const bool ok = pf[kk2] > 0.0f;
        // lane l < cnt holds copy l's side and entry count (none, one or two,
        // three to eight, in that order; packed as side + count << 24) and its
        // first entry (entry offsets fit 32 bits: the entry count does), handed
        // to the lanes that update the copy by cross-lane reads instead of a
        // chain of loads each
        int dl = 0, ml = 0, pl = 0;
        float tl = 0.0f;
        if (lane < cnt) {
            const int2 it = a.items[i0 + lane];
            const SideDesc &sl = a.sides[it.x];
            const int64_t po = sl.ptr_off + n;
            const int64_t q0 = a.ptr[po];
            tl = (float)sl.tau[(int64_t)sl.tau_stride * n];
            dl = (int)(a.ptr[po + 1] - q0);
            pl = (int)q0;
            ml = it.x | (dl << 24);
        }
        const int n0 = __popcll(__ballot(lane < cnt && dl == 0));
        const int n2 = __popcll(__ballot(lane < cnt && dl >= 1 && dl <= kLowRankSmall));
        __syncthreads();                             // the previous group's factor is read
        // the group's factor into the dense copy (its zeros were cleared at the start)
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int q = lane + 64 * i, dq = dmap[q];
            if (dq != 0xFFFF) ud[dq] = pf[q];
        }
        // windows of WIN copies: their noise in one draw per lane, then the
        // window's copies of each kind, G side by side (the kinds stay in order
        // inside a window, and a copy's draw does not depend on its partner)
        for (int w0 = 0; w0 < cnt; w0 += WIN) {
            const int w1 = min(cnt, w0 + WIN);
            __syncthreads();                         // the previous window's noise is read
#pragma unroll
            for (int d0 = 0; d0 < WIN; d0 += CPD) {
                const int cw = d0 + lane / LPC, q = lane % LPC;
                const int sxw = __shfl(ml, min(w0 + cw, cnt - 1)) & 0xFFFFFF;
                if (w0 + cw < w1) {
                    // entries K .. KP - 1 are zeros (the products read them)
                    float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (4 * q < K) normals4((uint32_t)n, t_sw, a.sides[sxw].c2, (uint32_t)q, a.k0, a.k1, z);
#pragma unroll
                    for (int e2 = 0; e2 < 4; ++e2) sz[cw][4 * q + e2] = 4 * q + e2 < K ? z[e2] : 0.0f;
                }
            }
            __syncthreads();
            // copies without entries: x = mu + U z
            const int e0 = min(n0, w1);
            for (int c = w0; c < e0; c += G) {
                const bool valid = c + h < e0;
                const int ci = valid ? c + h : c;
                const SideDesc &sd = a.sides[__shfl(ml, ci) & 0xFFFFFF];
                const float acc = row_dot<KP>(ud + r * UP, sz[ci - w0]);
                const double *mu = pr + kk2 + K;
                const float xv = r < K ? (float)(mu[r] + (double)acc) : 0.0f;
                const bool wr = valid && ok;
                if (wr && r < a.ks_self) self[(sd.self_off + n) * a.ks_self + r] = elem_from<Ts>((double)xv);
                if (wr && sample && r < a.ks_sample)
                    reinterpret_cast<Tp *>(sample)[(sd.sample_off + n) * a.ks_sample + r] = (Tp)xv;
                if (wr && a.sse_col && r < 4)
                    a.sse_col[4 * (sd.self_off + n) + r] = r == 0 ? a.colsq[sd.self_off + n] : 0.0;
            }
            // one or two entries, then three to eight
            const int s0 = max(n0, w0), s1 = min(n0 + n2, w1);
            for (int c = s0; c < s1; c += G) {
                const bool valid = c + h < s1;
                const int ci = valid ? c + h : c;
                const int mc = __shfl(ml, ci);
                group_lowrank_copy<P, KP, kLowRankSmall>(a, mc & 0xFFFFFF, (int64_t)__shfl(pl, ci), mc >> 24,
                                                         __shfl(tl, ci), valid, n,
                                                         ud + r, ud + r * UP, pr, sw[h], sy[h], sb[h],
                                                         sz[ci - w0], sample, ok, lane);
            }
            const int b0 = max(n0 + n2, w0);
            for (int c = b0; c < w1; c += G) {
                const bool valid = c + h < w1;
                const int ci = valid ? c + h : c;
                const int mc = __shfl(ml, ci);
                group_lowrank_copy<P, KP, kLowRankNnz>(a, mc & 0xFFFFFF, (int64_t)__shfl(pl, ci), mc >> 24,
                                                       __shfl(tl, ci), valid, n,
                                                       ud + r, ud + r * UP, pr, sw[h], sy[h], sb[h],
                                                       sz[ci - w0], sample, ok, lane);
            }
        }
        if (!ok && lane < cnt) {
            const int2 it = a.items[i0 + lane];
            if (a.fb_list) {
                const int slot = atomicAdd(a.fb_count, 1);
                a.fb_list[slot] = make_int2(it.x, n);
                atomicAdd(a.fb_total, 1);
            } else {
                atomicAdd(a.nonpd, 1);
            }
        }
    }
}

// --------------------------------------------------------------------------
// k_sse: residual SSE of every column of a column tile (the same per-column
// slots the fused column pass writes), for a tau step on its own.
// --------------------------------------------------------------------------
template <int KC, int P>
__global__ __launch_bounds__(256) void k_sse(const SseArgs a) {
    using Ts = typename PrecT<P>::s;
    using Tv = typename PrecT<P>::v;
    constexpr int KS = ks_of<Ts>(KC);
    const Tile tl = a.tiles[blockIdx.x];
    const int G = tl.G;
    const int grp = threadIdx.x / G;
    const bool wide = G > 64;
    const int Gw = G < 64 ? G : 64;
    const int gl = threadIdx.x & (G - 1);
    if (grp >= tl.count) return;
    const SideDesc &sd = a.sides[tl.side];
    const int n = a.ord[tl.start + grp];
    const int64_t p0 = a.ptr[sd.ptr_off + n], p1 = a.ptr[sd.ptr_off + n + 1];
    const Ts *Xs = reinterpret_cast<const Ts *>(a.X) + sd.other_off * KS;
    const Tv *val = reinterpret_cast<const Tv *>(a.val);
    using Tacc = typename PrecT<P>::acc;
    Tacc wd[KS];
    load_row<Tacc, KS>(reinterpret_cast<const Ts *>(a.W) + (sd.self_off + n) * KS, wd);
    double acc = 0.0;
    for (int64_t e = p0 + gl; e < p1; e += G) {
        Tacc xr[KS];
        load_row<Tacc, KS>(Xs + (int64_t)a.idx[e] * KS, xr);
        Tacc dot = 0;
#pragma unroll
        for (int i = 0; i < KS; ++i) dot += wd[i] * xr[i];
        const double res = (double)((Tacc)val[e] - dot);
        acc += res * res;
    }
    acc = group_sum1(acc, Gw);
    double *slot = a.sse_col + 4 * (sd.self_off + n);
    if (!wide) {
        if (gl == 0) {
            slot[0] = acc;
            slot[1] = 0.0;
            slot[2] = 0.0;
            slot[3] = 0.0;
        }
    } else if ((threadIdx.x & 63) == 0) {
        const int wv = (threadIdx.x >> 6) - ((grp * G) >> 6);
        slot[wv] = acc;
        if (wv == 0)
            for (int u = G >> 6; u < 4; ++u) slot[u] = 0.0;
    }
}

// --------------------------------------------------------------------------
// Normal-Wishart sufficient statistics: k_stats_mfma (below, with the
// reductions) writes one partial per job; k_reduce sums the jobs of a side in
// job order.  Fixed order throughout: deterministic.
// --------------------------------------------------------------------------

// --------------------------------------------------------------------------
// k_reduce: dst[p] = sum_{q < count} src[q * width + p], one workgroup per job.
// Thread t takes element p = t mod E and the q-slice t div E (E = min(width,
// 256)); each slice sums its q's in increasing order, slices are then added
// in slice order.  Deterministic for a given (count, width).
// --------------------------------------------------------------------------
// Fixed-order reductions, one job per block: dst[p] = sum over q < count of
// src[q * width + p].  Q threads per output (Q a power of two) each sum the
// rows q = s, s + Q, ... with 8 loads in flight; the Q partials are combined
// by a pairwise tree in LDS.
// Normal-Wishart sufficient statistics (sum x, sum x x^T) of one job's rows
// on FP64 MFMA.  The block's WB wavefronts split the rows; a wavefront takes
// them four at a time, lane l supplying component 16 b + l % 16 of row l / 16
// as both operands of v_mfma_f64_16x16x4_f64, so that tile (I, J) accumulates
// sum x_[16 I + i] x_[16 J + j] (lane l, register v: i = 4 v + l / 16,
// j = l % 16); sum x accumulates beside it on the VALU.  The wavefronts' sums
// are added in wavefront order through LDS: one partial per job.  Every
// product and sum is exact FP64 arithmetic in a fixed order.
typedef double f64x4_t __attribute__((ext_vector_type(4)));
template <typename Ts, int KB, int WB>
__global__ __launch_bounds__(64 * WB) void k_stats_mfma(const StatsArgs a) {
    constexpr int NT = KB * (KB + 1) / 2;
    extern __shared__ double wsum[];                 // WB x npair
    const StatsJob jb = a.jobs[blockIdx.x];
    const SideDesc &sd = a.sides[jb.side];
    const Ts *X = reinterpret_cast<const Ts *>(jb.side < a.nrow_sides ? a.X : a.W) + sd.self_off * a.ks;
    const int K = a.K;
    const int npair = K + K * (K + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int comp = lane & 15, rsub = lane >> 4;
    f64x4_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    double sx[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b) sx[b] = 0.0;
    // this wavefront's rows: a contiguous range, a multiple of 4 long
    const int per = ((jb.count + 4 * WB - 1) / (4 * WB)) * 4;
    const int lo = wave * per, hi = min(jb.count, lo + per);
    for (int r0 = lo; r0 < hi; r0 += 16) {
        double v[4][KB];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + 4 * u + rsub;
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                const int k = 16 * b + comp;
                v[u][b] = (r < hi && k < K) ? elem_to_d(X[(int64_t)(jb.first + r) * a.ks + k]) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int t = 0;
#pragma unroll
            for (int I = 0; I < KB; ++I) {
                sx[I] += v[u][I];
#pragma unroll
                for (int J = 0; J <= I; ++J, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][I], v[u][J], acc[t], 0, 0, 0);
            }
        }
    }
    // sum x over the four row groups of the wavefront
#pragma unroll
    for (int b = 0; b < KB; ++b) sx[b] = bfly_step<32>(bfly_step<16>(sx[b]));
    double *ws = wsum + wave * npair;
    if (rsub == 0) {
#pragma unroll
        for (int b = 0; b < KB; ++b)
            if (16 * b + comp < K) ws[16 * b + comp] = sx[b];
    }
    {
        int t = 0;
#pragma unroll
        for (int I = 0; I < KB; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J, ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * v + rsub, j = comp;
                    const int ra = 16 * I + i, cb = 16 * J + j;
                    if (ra < K && cb < K && (I > J || i >= j)) ws[K + ra * (ra + 1) / 2 + cb] = acc[t][v];
                }
    }
    __syncthreads();
    double *part = a.part + (int64_t)jb.part * npair;
    for (int p = threadIdx.x; p < npair; p += 64 * WB) {
        double s = 0.0;
        for (int w = 0; w < WB; ++w) s += wsum[w * npair + p];
        part[p] = s;
    }
}

// Noise of one Normal-Wishart draw, written to dst: [Bartlett diagonal
// sqrt(chi2(nu* - i)), i < K | K(K-1)/2 standard normals below the diagonal,
// row-major | K standard normals for the mean].  The diagonal is drawn by
// threads [0, K), the normals in blocks of four by threads from `first` on,
// `stride` apart (first = 0 and stride = 64 in a single wavefront).
__device__ void nw_noise(const HyperJob &jb, int K, double nu0, uint32_t t_sw, uint32_t k0, uint32_t k1,
                         double *dst, int tid, int first, int stride) {
    const uint32_t c2 = counter_word(jb.block, jb.kind == 0 ? kHyperX : kHyperW);
    const double nu_s = nu0 + (double)jb.n;
    if (tid < K) dst[tid] = sqrt(2.0 * gamma_draw(k0, k1, (uint32_t)(tid + 1), t_sw, c2, 0.5 * (nu_s - tid)));
    const int noff = K * (K - 1) / 2;
    const int go = (noff + 3) / 4, gm = (K + 3) / 4;
    for (int u = tid - first; u >= 0 && u < go + gm; u += stride) {
        double z[4];
        const bool off = u < go;
        const int g = off ? u : u - go;
        normals4(off ? 0u : (uint32_t)(K + 1), t_sw, c2, (uint32_t)g, k0, k1, z);
        const int lim = off ? noff : K;
        double *d = dst + K + (off ? 0 : noff);
        for (int c = 0; c < 4; ++c)
            if (4 * g + c < lim) d[4 * g + c] = z[c];
    }
}

constexpr int kReduceThreads = 1024;
constexpr int kReduceSlice = 256;           // outputs per block at most (blockIdx.y: slice)
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const ReduceJob *jobs, const int32_t njobs,
                                                           const NoiseArgs na) {
    __shared__ double red[kReduceThreads];
    if ((int)blockIdx.x >= njobs) {
        // the Normal-Wishart noise of hyper job blockIdx.x - njobs (first slice
        // only): the diagonal in the first wavefront, the normals from the second
        const int j = blockIdx.x - njobs;
        if (blockIdx.y != 0) return;
        const HyperJob hj = na.jobs[j];
        if (hj.kind > 1) return;
        const uint32_t t_sw = na.ss ? na.ss->t : na.t;
        nw_noise(hj, na.K, na.nu0, t_sw, na.k0, na.k1, na.noise + (int64_t)j * (na.K * (na.K + 3) / 2),
                 threadIdx.x, 64, kReduceThreads - 64);
        return;
    }
    const ReduceJob jb = jobs[blockIdx.x];
    const int t = threadIdx.x;
    const int lo = blockIdx.y * kReduceSlice;
    if (lo >= jb.width) return;             // uniform per block
    const int hi = min(jb.width, lo + kReduceSlice);
    const int E = hi - lo;
    int Q = 1;
    while (2 * Q * E <= kReduceThreads) Q *= 2;
    const int s = t / E, pe = t - s * E;
    for (int base = lo; base < hi; base += E) {
        const int p = base + pe;
        double acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.0;
        if (s < Q && p < hi) {
            int q = s;
            for (; q + 7 * Q < jb.count; q += 8 * Q) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = jb.src[(int64_t)(q + u * Q) * jb.width + p];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[u] += v[u];
            }
            for (int u = 0; q < jb.count; q += Q, ++u) acc[u & 7] += jb.src[(int64_t)q * jb.width + p];
        }
        __syncthreads();
        if (s < Q) red[s * E + pe] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        for (int h = Q / 2; h > 0; h /= 2) {
            __syncthreads();
            if (s < h) red[s * E + pe] += red[(s + h) * E + pe];
        }
        __syncthreads();
        if (s == 0 && p < hi) jb.dst[p] = red[pe];
    }
}

// --------------------------------------------------------------------------
// k_hyper: Normal-Wishart draw of one side of one block, or a tau draw (FP64).
//   x_bar = sum x / N,  N S_bar = sum x x^T - N x_bar x_bar^T (the footnote's
//   alternative to the centred form), beta* = beta0 + N, nu* = nu0 + N,
//   mu* = (beta0 mu0 + N x_bar) / beta*,
//   W*^-1 = W0^-1 + N S_bar + (beta0 N / beta*) (mu0 - x_bar)(mu0 - x_bar)^T;
//   Bartlett: R R^T = W*^-1, T = R^-T, A lower (A_kk^2 ~ chi2(nu* - k + 1),
//   A_kl ~ N(0,1)), Lambda = (T A)(T A)^T; mu = mu* + beta*^-1/2 C^-T z with
//   C C^T = Lambda.  tau ~ Gamma(a0 + M/2, rate b0 + SSE/2).
// --------------------------------------------------------------------------
// Normal-Wishart draw of one side of one block (one wavefront).
template <int KP>
__device__ __forceinline__ void nw_draw(const HyperArgs &a, const HyperJob &jb, uint32_t t_sw, int lane) {
    constexpr int LD = KP + 2;                     // doubles; 16-byte rows, few bank conflicts
    __shared__ __align__(16) double S0[KP * LD];   // W*^-1, then Lambda
    __shared__ __align__(16) double S1[KP * LD];   // R, then C (rows of the factors)
    __shared__ __align__(16) double S2[KP * LD];   // Bartlett A, then B = R^-T A
    __shared__ double sx[KP], mus[KP], dg[KP], sinv[KP], zz[KP];
    const int K = a.K;
    asm volatile("" : "+v"(lane));
    int z0 = 0;
    asm volatile("" : "+v"(z0));
    z0 &= ~15;
    const bool own = lane < KP;
    const int row = own ? lane : KP - 1;
    const int npair = K + K * (K + 1) / 2;
    // the draw's noise: made by the reduction launch before this one, or here
    const double *nz = a.noise + (int64_t)blockIdx.x * (K * (K + 3) / 2);
    if (!a.noise_ready) {
        nw_noise(jb, K, a.nu0, t_sw, a.k0, a.k1, const_cast<double *>(nz), lane, 0, 64);
        __syncthreads();
    }
    // 1. the side's sums (reduced in fixed order by the statistics kernel):
    //    sum x, then sum x x^T packed lower
    const double *part = a.part + (int64_t)jb.part_begin * npair;
    if (lane < K) sx[lane] = part[lane];
    __syncthreads();
    const double N = (double)jb.n;
    const double beta_s = a.beta0 + N;
    if (lane < K) mus[lane] = (a.beta0 * a.mu0[lane] + sx[lane]) / beta_s;
    // 2. W*^-1 = W0^-1 + (sum x x^T - N xbar xbar^T) + beta0 N / beta* (mu0 - xbar)(mu0 - xbar)^T,
    //    identity padding beyond K (the KP x KP grid, no index unranking)
    const double coef = a.beta0 * N / beta_s;
    for (int q = lane; q < KP * KP; q += 64) {
        const int r = q / KP, c = q - (q / KP) * KP;
        double v = (double)(r == c);
        if (r < K && c < K) {
            const double sxx = part[K + (r >= c ? tri(r, c) : tri(c, r))];
            const double xr = sx[r] / N, xc = sx[c] / N;
            const double ns = sxx - N * xr * xc;
            v = a.W0inv[r * K + c] + ns + coef * (a.mu0[r] - xr) * (a.mu0[c] - xc);
        }
        S0[r * LD + c] = v;
    }
    __syncthreads();
    if (own) dg[lane] = S0[lane * LD + lane];
    __syncthreads();
    // 3. R R^T = W*^-1 (rows of R in registers and in S1)
    double rr[KP];
    bool ok = chol_rows<KP, double>(S0, LD, S1, LD, dg, sinv, 0.0, lane, z0, rr);
    // 4. Bartlett factor A (lower) in S2: A_kk^2 ~ chi2(nu* - k) for k < K,
    //    A_kl ~ N(0, 1) below the diagonal (row-major order of the strict lower
    //    triangle: entry (r, c) is number tri(r - 1, c)), identity padding
    const int noff = K * (K - 1) / 2;
    for (int q = lane; q < KP * KP; q += 64) {
        const int r = q / KP, c = q - (q / KP) * KP;
        double v = 0.0;
        if (r == c) v = r < K ? nz[r] : 1.0;
        else if (c < r && r < K) v = nz[K + tri(r - 1, c)];
        S2[r * LD + c] = v;
    }
    __syncthreads();
    asm volatile("" : "+v"(lane));
    // 5. B = R^-T A: lane c solves R^T b = (column c of A) from the bottom,
    //    b_i = (a_ic - sum_{p>i} R_pi b_p) / R_ii, R_pi read by broadcast
    {
        double bb[KP];
#pragma unroll
        for (int i = KP - 1; i >= 0; --i) {
            double s0 = S2[i * LD + row], s1 = 0.0;
#pragma unroll
            for (int p = i + 1; p < KP; ++p) {
                if (p & 1) s1 -= S1[z0 + p * LD + i] * bb[p];
                else s0 -= S1[z0 + p * LD + i] * bb[p];
            }
            bb[i] = (s0 + s1) * sinv[z0 + i];
            asm volatile("" : "+v"(bb[i]));
        }
        __syncthreads();                        // every column of A read
        if (own) {
#pragma unroll
            for (int i = 0; i < KP; ++i) S2[i * LD + lane] = bb[i];
        }
    }
    __syncthreads();
    asm volatile("" : "+v"(lane));
    // 6. Lambda = B B^T: lane r takes row r of B and forms row r of Lambda
    //    against every row of B read by broadcast
    double *outL = jb.out;
    {
        double br[KP];
#pragma unroll
        for (int c = 0; c < KP; ++c) br[c] = S2[row * LD + c];
        __syncthreads();
        for (int s = 0; s < KP; ++s) {
            const double *bs = S2 + z0 + s * LD;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
            for (int c = 0; c < KP; c += 4) {
                a0 += br[c] * bs[c];
                if (c + 1 < KP) a1 += br[c + 1] * bs[c + 1];
                if (c + 2 < KP) a2 += br[c + 2] * bs[c + 2];
                if (c + 3 < KP) a3 += br[c + 3] * bs[c + 3];
            }
            const double v = (a0 + a2) + (a1 + a3);
            if (own) S0[lane * LD + s] = v;
            if (lane < K && s < K) outL[lane * K + s] = v;
        }
    }
    __syncthreads();
    if (own) dg[lane] = S0[lane * LD + lane];
    __syncthreads();
    // 7. C C^T = Lambda (rows of C in S1); 8. mu = mu* + C^-T z / sqrt(beta*)
    ok = chol_rows<KP, double>(S0, LD, S1, LD, dg, sinv, 0.0, lane, z0, rr) && ok;
    if (own) zz[lane] = lane < K ? nz[K + noff + lane] : 0.0;
    __syncthreads();
    asm volatile("" : "+v"(lane));
    {
        // backward solve with columns of C: lane i holds C_qi for q >= i
        double cc[KP];
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const double v2 = S1[q * LD + row];
            cc[q] = q >= lane ? v2 : 0.0;
            asm volatile("" : "+v"(cc[q]));
        }
        double acc = zz[row], x = 0.0;
#pragma unroll
        for (int q = KP - 1; q >= 0; --q) {
            const double xq = wave_bcast(acc, q) * sinv[z0 + q];
            x = lane == q ? xq : x;
            acc = (lane < q) ? acc - cc[q] * xq : acc;
        }
        if (lane < K) {
            const double m = mus[lane] + x / sqrt(beta_s);
            sx[lane] = m;
            outL[K * K + lane] = m;
        }
    }
    __syncthreads();
    double *packed = outL + K * K + 2 * K;      // [Lambda packed lower, Lambda mu, mu]
    if (lane < K) {
        double s = 0.0;
        for (int c = 0; c < K; ++c) s += S0[lane * LD + c] * sx[c];
        outL[K * K + K + lane] = s;
        packed[K * (K + 1) / 2 + lane] = s;
        packed[K * (K + 1) / 2 + K + lane] = sx[lane];
    }
    for (int q = lane; q < KP * KP; q += 64) {
        const int r = q / KP, c = q - (q / KP) * KP;
        if (c <= r && r < K) packed[tri(r, c)] = S0[r * LD + c];
    }
    if (!ok && lane == 0) atomicAdd(a.nonpd, 1);
}

template <int KP>
__global__ __launch_bounds__(64) void k_hyper(const HyperArgs a) {
    const HyperJob jb = a.jobs[blockIdx.x];
    const int lane = threadIdx.x;
    const uint32_t t_sw = a.ss ? a.ss->t : a.t;
    if (jb.kind == 2) {
        if (lane == 0) {
            const double s = a.sse_part[jb.part_begin];
            const double shape = a.a0 + 0.5 * (double)jb.n;
            const double rate = a.b0 + 0.5 * s;
            *jb.out = gamma_draw(a.k0, a.k1, 0u, t_sw, counter_word(jb.block, kTau), shape) / rate;
        }
    } else {
        nw_draw<KP>(a, jb, t_sw, lane);
    }
    if (a.advance) {
        // the last block to finish (every block has read the sweep index)
        // advances the sweep state and clears the counter for the next launch
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            if (atomicAdd(a.done, 1) == (int)gridDim.x - 1) {
                __threadfence();
                sweep_advance(a.advance, a.fb_counts);
                *a.done = 0;
            }
        }
    }
}

// --------------------------------------------------------------------------
// k_init: initial factors (K^-1/4 z from the INIT counters, or the propagated
// means) for every entity of the listed sides.
// --------------------------------------------------------------------------
template <typename Ts>
__global__ __launch_bounds__(256) void k_init(const InitArgs a) {
    const int K = a.K;
    const double scale = pow((double)K, -0.25);
    for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < a.nitems; it += gridDim.x * blockDim.x) {
        const int2 item = a.items[it];
        const SideDesc &sd = a.sides[item.x];
        const int n = item.y;
        Ts *dst = reinterpret_cast<Ts *>(a.self) + (sd.self_off + n) * a.ks_self;
        for (int k = K; k < a.ks_self; ++k) dst[k] = elem_from<Ts>(0.0);
        if (sd.per_row) {
            const double *mu = sd.prior + (int64_t)n * a.prow + K * (K + 1) / 2 + K;
            for (int k = 0; k < K; ++k) dst[k] = elem_from<Ts>(mu[k]);
        } else {
            for (int g = 0; 4 * g < K; ++g) {
                double z[4];
                normals4((uint32_t)n, 0xFFFFFFFFu, sd.c2_init, (uint32_t)g, a.k0, a.k1, z);
                for (int c = 0; c < 4 && 4 * g + c < K; ++c) dst[4 * g + c] = elem_from<Ts>(scale * z[c]);
            }
        }
    }
}

// --------------------------------------------------------------------------
// k_mm: moment matching of one entity from the S kept samples (FP64):
// mean, covariance with 1/(S-1) (two passes), ridge when S <= K or not SPD,
// Lambda_hat = L^-T L^-1, eta = Lambda_hat mu_hat.  Output row:
// [Lambda_hat packed lower, eta, mu_hat].
// --------------------------------------------------------------------------
template <typename Ts, int KP>
__global__ __launch_bounds__(64) void k_mm(const MmArgs a) {
    constexpr int LD = KP + 1;                     // LDS sized to K: more entities per CU
    constexpr int MC = 16;                         // samples per LDS chunk
    constexpr int NPL = (KP * (KP + 1) / 2 + 63) / 64;   // covariance pairs per lane
    __shared__ double sig[KP * LD];
    __shared__ double lin[KP * LD];
    __shared__ double xs[MC * KP];
    __shared__ double mu[KP];
    __shared__ int flag;
    const int lane = threadIdx.x;
    const int K = a.K, S = a.S;
    const int kk2 = K * (K + 1) / 2;
    for (int it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const int2 item = a.items[it];
        const SideDesc &sd = a.sides[item.x];
        const int n = item.y;
        const Ts *smp = reinterpret_cast<const Ts *>(a.sample) + (sd.sample_off + n) * a.ks;
        double *out = a.out[item.x] + (int64_t)n * a.prow;
        if (lane < K) {
            double s = 0.0;
            for (int q = 0; q < S; ++q) s += (double)smp[(int64_t)q * a.slot_elems + lane];
            mu[lane] = s / (double)S;
        }
        __syncthreads();
        if (S < 2) {
            for (int q = lane; q < kk2 + K; q += 64) out[q] = 0.0;
            if (lane < K) out[kk2 + K + lane] = mu[lane];
            __syncthreads();
            continue;
        }
        // covariance: lane owns packed pairs lane, lane + 64, ...; the centred
        // samples pass through LDS in chunks of MC, each sum still in sample order
        double cacc[NPL];
#pragma unroll
        for (int u = 0; u < NPL; ++u) cacc[u] = 0.0;
        for (int t0 = 0; t0 < S; t0 += MC) {
            const int nt = min(MC, S - t0);
            for (int q = lane; q < nt * K; q += 64) {
                const int t = q / K, k = q - t * K;
                xs[t * KP + k] = (double)smp[(int64_t)(t0 + t) * a.slot_elems + k] - mu[k];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < NPL; ++u) {
                const int q = lane + 64 * u;
                if (q < kk2) {
                    const int r = (int)((__builtin_sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5 + 1e-9);
                    const int c = q - r * (r + 1) / 2;
                    double sacc = cacc[u];
                    for (int t = 0; t < nt; ++t) sacc += xs[t * KP + r] * xs[t * KP + c];
                    cacc[u] = sacc;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < NPL; ++u) {
            const int q = lane + 64 * u;
            if (q < kk2) {
                const int r = (int)((__builtin_sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5 + 1e-9);
                const int c = q - r * (r + 1) / 2;
                const double v = cacc[u] / (double)(S - 1);
                sig[r * LD + c] = v;
                sig[c * LD + r] = v;
            }
        }
        __syncthreads();
        bool need = S <= K;
        if (!need) {
            for (int q = lane; q < K * K; q += 64) lin[q / K * LD + q % K] = sig[q / K * LD + q % K];
            __syncthreads();
            need = !chol_lds<double>(lin, K, LD, 0.0, nullptr, lane, &flag);
        }
        if (need) {
            double tr = 0.0;
            for (int k = 0; k < K; ++k) tr += sig[k * LD + k];
            const double delta = 1e-6 * tr / (double)K + 1e-300;
            __syncthreads();
            if (lane < K) sig[lane * LD + lane] += delta;
            __syncthreads();
            for (int q = lane; q < K * K; q += 64) lin[q / K * LD + q % K] = sig[q / K * LD + q % K];
            __syncthreads();
            chol_lds<double>(lin, K, LD, 0.0, nullptr, lane, &flag);
            if (lane == 0) atomicAdd(a.ridged, 1);
        }
        // sig <- L^-1 (column c by lane c)
        for (int c = lane; c < K; c += 64) {
            for (int i = 0; i < K; ++i) {
                if (i < c) {
                    sig[i * LD + c] = 0.0;
                } else {
                    double s = (i == c) ? 1.0 : 0.0;
                    for (int p = c; p < i; ++p) s -= lin[i * LD + p] * sig[p * LD + c];
                    sig[i * LD + c] = s / lin[i * LD + i];
                }
            }
        }
        __syncthreads();
        for (int q = lane; q < K * K; q += 64) {
            const int r = q / K, c = q - r * K;
            if (c <= r) {
                double s = 0.0;
                for (int p = r; p < K; ++p) s += sig[p * LD + r] * sig[p * LD + c];
                lin[r * LD + c] = s;
                lin[c * LD + r] = s;
            }
        }
        __syncthreads();
        for (int q = lane; q < K * K; q += 64) {
            const int r = q / K, c = q - (q / K) * K;
            if (c <= r) out[tri(r, c)] = lin[r * LD + c];
        }
        if (lane < K) {
            double s = 0.0;
            for (int c = 0; c < K; ++c) s += lin[lane * LD + c] * mu[c];
            out[kk2 + lane] = s;
            out[kk2 + K + lane] = mu[lane];
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// k_mm_rows: moment matching for K <= KP <= 32, one covariance row per lane
// and 64 / KP entities per wavefront (lanes KP h .. KP h + KP - 1 hold entity
// h; padding rows and columns beyond K hold the identity).  The mean and the
// two-pass covariance sum the kept samples in sample order; a chunk of
// centred samples passes through LDS and every lane reads it back by
// broadcast.  Lambda_hat = Sigma_hat^-1 comes from the symmetric sweep
// operator (Goodnight, 1979) applied to pivots 0 .. K-1: after each sweep the
// working matrix is still symmetric, so pivot row k is the column k that the
// lanes hold, and the full sweep leaves -Sigma_hat^-1.  The pivots are the
// successive Schur complements of Sigma_hat (the squares of its Cholesky
// pivots), so a pivot that is not positive is the factorisation failing: the
// entity is computed again with the ridge.  The output row is staged in LDS
// and stored contiguously.
// --------------------------------------------------------------------------
template <typename Ts, int KP>
__global__ __launch_bounds__(64) void k_mm_rows(const MmArgs a) {
    constexpr int G = 64 / KP;
    constexpr int MC = KP == 32 ? 20 : 12;          // samples per LDS chunk
    static_assert(MC * KP >= KP * (KP + 1) / 2 + 2 * KP, "the output row is staged in the chunk buffer");
    __shared__ __align__(16) double xs[G][MC * KP];
    __shared__ __align__(16) double bc[G][KP];
    const int lane = threadIdx.x;
    const int h = lane / KP, r = lane % KP;
    const int K = a.K, S = a.S;
    const int kk2 = K * (K + 1) / 2;
    for (int pit = blockIdx.x; G * pit < a.nitems; pit += gridDim.x) {
        const int it = G * pit + h;
        const bool valid = it < a.nitems;           // uniform per entity
        const int iq = valid ? it : G * pit;
        const int2 item = a.items[iq];
        const SideDesc &sd = a.sides[item.x];
        const int n = item.y;
        const Ts *smp = reinterpret_cast<const Ts *>(a.sample) + (sd.sample_off + n) * a.ks;
        // the samples taken (every one, or one cluster's)
        int w = -1;
        const uint8_t *lab = nullptr;
        if (a.labels) {
            w = a.which[(int64_t)iq * kMaxComp + a.comp];
            lab = a.labels[item.x] + (int64_t)n * a.maxS;
        }
        const bool has = w != -2;
        int m = S;
        if (w >= 0) {
            m = 0;
            for (int q = 0; q < S; ++q) m += lab[q] == w;
        }
        double mu = 0.0;
        if (r < K && has) {
            double s = 0.0;
            for (int q = 0; q < S; ++q)
                if (w < 0 || lab[q] == w) s += (double)smp[(int64_t)q * a.slot_elems + r];
            mu = s / (double)m;
        }
        double row[KP];
#pragma unroll
        for (int c = 0; c < KP; ++c) row[c] = 0.0;
        bool ridge = m <= K;
        double ld = 0.0;                            // log det Lambda_hat = -sum log pivots
        for (int pass = 0; pass < 2 && S >= 2; ++pass) {
#pragma unroll
            for (int c = 0; c < KP; ++c) row[c] = 0.0;
            for (int t0 = 0; t0 < S; t0 += MC) {
                const int nt = min(MC, S - t0);
                __syncthreads();                    // the previous chunk is read
                for (int t = 0; t < nt; ++t) {
                    const bool tk = r < K && has && (w < 0 || lab[t0 + t] == w);
                    xs[h][t * KP + r] = tk ? (double)smp[(int64_t)(t0 + t) * a.slot_elems + r] - mu : 0.0;
                }
                __syncthreads();
                for (int t = 0; t < nt; ++t) {
                    const double xr = xs[h][t * KP + r];
#pragma unroll
                    for (int c = 0; c < KP; ++c) row[c] += xr * xs[h][t * KP + c];
                }
            }
            const double inv_s1 = 1.0 / (double)(m >= 2 ? m - 1 : 1);
#pragma unroll
            for (int c = 0; c < KP; ++c) row[c] = r < K ? row[c] * inv_s1 : (c == r ? 1.0 : 0.0);
            if (ridge) {
                double dg = 0.0;
#pragma unroll
                for (int c = 0; c < KP; ++c) dg = c == r ? row[c] : dg;
                double tr = 0.0;
                for (int k = 0; k < K; ++k) tr += __shfl(dg, h * KP + k, 64);   // in index order
                const double delta = 1e-6 * tr / (double)K + 1e-300;
#pragma unroll
                for (int c = 0; c < KP; ++c) row[c] += (c == r && r < K) ? delta : 0.0;
            }
            // sweep pivots 0 .. K-1
            int bad = 0;
            ld = 0.0;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                if (k < K) {
                    __syncthreads();                // the previous pivot column is read
                    bc[h][r] = row[k];
                    __syncthreads();
                    const double p = bc[h][k];
                    bad |= !(p > 0.0);
                    ld -= log(p > 0.0 ? p : 1.0);
                    const double ip = 1.0 / (p > 0.0 ? p : 1.0);
                    const double f = row[k] * ip;
                    const bool own = r == k;
#pragma unroll
                    for (int j = 0; j < KP; ++j) {
                        if (j == k) continue;
                        const double bj = bc[h][j];
                        row[j] = own ? bj * ip : row[j] - f * bj;
                    }
                    row[k] = own ? -ip : f;
                }
            }
            const bool again = !ridge && bad && has && m >= 2;   // the factorisation failed: take the ridge
            if (__ballot(valid && again) == 0) break;
            ridge = ridge || again;
            if (pass == 1) break;
        }
        const bool fit = has && m >= 2 && S >= 2;
        if (valid && fit && ridge && r == 0 && a.comp == 0) atomicAdd(a.ridged, 1);
        // Lambda_hat mu_hat, then the packed row through LDS
        __syncthreads();
        bc[h][r] = mu;
        __syncthreads();
        double eta = 0.0;
#pragma unroll
        for (int c = 0; c < KP; ++c) eta -= row[c] * bc[h][c];
        __syncthreads();                            // the chunk buffer is free
        if (r < K) {
            const int base = r * (r + 1) / 2;
#pragma unroll
            for (int c = 0; c < KP; ++c)
                if (c <= r) xs[h][base + c] = fit ? -row[c] : 0.0;
            xs[h][kk2 + r] = fit ? eta : 0.0;
            xs[h][kk2 + K + r] = mu;
        }
        __syncthreads();
        if (valid && has) {
            double *out = a.out[item.x] + (int64_t)n * a.prow;
            for (int q = r; q < a.prow; q += KP) out[q] = xs[h][q];
            if (a.aux && r == 0) a.aux[item.x][(int64_t)n * 2 + 1] = ld;
        }
    }
}

// --------------------------------------------------------------------------
// Per-column noise precisions (the tau_d variant of Sec. 2.1).  The row
// conditional with entry weights tau_d, A = P + sum tau_d w_d w_d^T and
// h = P m + sum tau_d r_nd w_d, is the unweighted one of w~_d = sqrt(tau_d) w_d
// and r~_nd = sqrt(tau_d) r_nd; k_tau_scale forms both (rounded once to the
// state and value precision) for the row pass, from the current W and tau.
// k_tau_cols draws tau_d ~ Gamma(a0 + M_d / 2, b0 + SSE_d / 2) per column, on
// counter (d, t, (block << 8) | TAU, attempt), with SSE_d the column's
// residual SSE of this sweep's column pass.
// --------------------------------------------------------------------------
template <typename Ts, typename Tv>
__global__ __launch_bounds__(256) void k_tau_scale(const TauColArgs a) {
    const TauColJob jb = a.jobs[blockIdx.y];
    const Ts *W = reinterpret_cast<const Ts *>(a.W) + jb.w_off * a.ks;
    Ts *Wt = reinterpret_cast<Ts *>(a.Wt) + jb.w_off * a.ks;
    const double *tau = a.tau + jb.w_off;
    const int64_t nw = (int64_t)jb.C * a.ks;
    for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < nw; q += (int64_t)gridDim.x * 256) {
        const int64_t d = q / a.ks;
        Wt[q] = (Ts)(sqrt(tau[d]) * (double)W[q]);
    }
    const Tv *val = reinterpret_cast<const Tv *>(a.val) + jb.e0;
    Tv *vt = reinterpret_cast<Tv *>(a.vt) + jb.e0;
    const int32_t *idx = a.idx + jb.e0;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < jb.M; e += (int64_t)gridDim.x * 256)
        vt[e] = (Tv)(sqrt(tau[idx[e]]) * (double)val[e]);
}

__global__ __launch_bounds__(256) void k_tau_cols(const TauColArgs a) {
    const TauColJob jb = a.jobs[blockIdx.y];
    const uint32_t t = a.ss ? a.ss->t : a.t;
    for (int d = blockIdx.x * 256 + threadIdx.x; d < jb.C; d += gridDim.x * 256) {
        const int64_t m = a.cptr[jb.cptr_off + d + 1] - a.cptr[jb.cptr_off + d];
        const double *sp = a.sse_col + 4 * (jb.w_off + d);
        const double sse = ((sp[0] + sp[1]) + sp[2]) + sp[3];
        const double shape = a.a0 + 0.5 * (double)m;
        const double rate = a.b0 + 0.5 * sse;
        a.tau[jb.w_off + d] = gamma_draw(a.k0, a.k1, (uint32_t)d, t, counter_word(jb.block, kTau), shape) / rate;
    }
}

// --------------------------------------------------------------------------
// k_lmeans: clustering of each entity's kept samples for the dominant-mode and
// mixture approximations (Sec. 4.1; Sec. 5.1, which clusters with
// lambda-means), one lane per entity, by the hard-clustering DP-means
// iteration (Kulis and Jordan, 2012): one initial cluster at the mean of the
// samples; then rounds of (1) assignment in sample order -- the nearest centre
// (squared distance, lowest index on ties), or a new cluster on the sample
// itself when that centre is farther than lambda and fewer than kLmCmax
// clusters exist -- and (2) centres moved to their members' means (sums in
// sample order), clusters without members dropped with the others keeping
// their order; until the assignment repeats, at most kLmMaxit rounds.
// lambda^2 = c^2 sum_t |x_(t+1) - x_t|^2 / (2 (S - 1)), c = lam_scale.  Every
// sum runs in index order without fused multiply-adds, so the labels are the
// exact FP64 result of these steps.  Then the components: the ncomp largest
// clusters with at least two members (decreasing size, lower index on ties),
// or every sample as one component when none has two; weights proportional
// to their sizes.  Centres, labels and counts live in the lane's private
// memory; the samples are read from the sample store as needed.
// --------------------------------------------------------------------------
template <typename Ts, int KP>
__global__ __launch_bounds__(64) void k_lmeans(const LmeansArgs a) {
#pragma clang fp contract(off)
    const int it = blockIdx.x * 64 + threadIdx.x;
    if (it >= a.nitems) return;
    const int K = a.K, S = a.S;
    const int2 item = a.items[it];
    const SideDesc &sd = a.sides[item.x];
    const int n = item.y;
    const Ts *smp = reinterpret_cast<const Ts *>(a.sample) + (sd.sample_off + n) * a.ks;
    auto x = [&](int q, int k) { return (double)smp[(int64_t)q * a.slot_elems + k]; };
    double cent[kLmCmax][KP];
    int cnt[kLmCmax];
    uint8_t lab[kLmMaxS], prev[kLmMaxS];
    auto dist2 = [&](int q, int c) {
        double t = 0.0;
        for (int k = 0; k < K; ++k) {
            const double d = x(q, k) - cent[c][k];
            t = t + d * d;
        }
        return t;
    };
    double steps = 0.0;
    for (int q = 0; q + 1 < S; ++q) {
        double t = 0.0;
        for (int k = 0; k < K; ++k) {
            const double d = x(q + 1, k) - x(q, k);
            t = t + d * d;
        }
        steps = steps + t;
    }
    const double lam2 = S > 1 ? a.lam_scale * a.lam_scale * steps / (2.0 * (double)(S - 1)) : 0.0;
    int C = 1;
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int q = 0; q < S; ++q) t = t + x(q, k);
        cent[0][k] = t / (double)S;
    }
    for (int q = 0; q < S; ++q) prev[q] = 0xFF;
    for (int round = 0; round < kLmMaxit; ++round) {
        for (int q = 0; q < S; ++q) {
            int best = 0;
            double dbest = dist2(q, 0);
            for (int c = 1; c < C; ++c) {
                const double d = dist2(q, c);
                if (d < dbest) {
                    dbest = d;
                    best = c;
                }
            }
            if (dbest > lam2 && C < kLmCmax) {
                for (int k = 0; k < K; ++k) cent[C][k] = x(q, k);
                best = C++;
            }
            lab[q] = (uint8_t)best;
        }
        for (int c = 0; c < C; ++c) {
            cnt[c] = 0;
            for (int k = 0; k < K; ++k) cent[c][k] = 0.0;
        }
        for (int q = 0; q < S; ++q) {
            const int c = lab[q];
            for (int k = 0; k < K; ++k) cent[c][k] = cent[c][k] + x(q, k);
            cnt[c] += 1;
        }
        int Cn = 0;
        for (int c = 0; c < C; ++c) {
            if (cnt[c] == 0) continue;
            for (int k = 0; k < K; ++k) cent[Cn][k] = cent[c][k] / (double)cnt[c];
            cnt[Cn] = cnt[c];
            for (int q = 0; q < S; ++q)
                if (lab[q] == c) lab[q] = (uint8_t)Cn;
            ++Cn;
        }
        C = Cn;
        bool same = true;
        for (int q = 0; q < S; ++q) {
            same = same && lab[q] == prev[q];
            prev[q] = lab[q];
        }
        if (same) break;
    }
    uint8_t *lo = a.labels[item.x] + (int64_t)n * a.maxS;
    for (int q = 0; q < S; ++q) lo[q] = lab[q];
    // components
    int chosen[kMaxComp];
    int taken = 0, nch = 0;
    for (int c = 0; c < a.ncomp; ++c) {
        int best = -1;
        for (int j = 0; j < C; ++j)
            if (!((taken >> j) & 1) && cnt[j] >= 2 && (best < 0 || cnt[j] > cnt[best])) best = j;
        if (best < 0) break;
        taken |= 1 << best;
        chosen[nch++] = best;
    }
    int total = 0;
    for (int c = 0; c < nch; ++c) total += cnt[chosen[c]];
    double *ax = a.aux[item.x] + (int64_t)n * 2;
    for (int c = 0; c < kMaxComp; ++c) {
        int8_t wv = -2;
        double pi = 0.0;
        if (nch == 0 && c == 0) {
            wv = -1;
            pi = 1.0;
        } else if (c < nch) {
            wv = (int8_t)chosen[c];
            pi = (double)cnt[chosen[c]] / (double)total;
        }
        a.which[(int64_t)it * kMaxComp + c] = wv;
        if (c < a.ncomp) ax[c * a.aux_plane] = pi;
    }
}

// --------------------------------------------------------------------------
// k_gmm_pool: the pooled moments of each entity's mixture (eq.
// marginal_mixture): mu = sum_c pi_c mu_c and Sigma = sum_c pi_c (Sigma_c +
// (mu_c - mu)(mu_c - mu)^T) with Sigma_c = Lambda_c^-1, written as the
// entity's moment-matched row [Lambda packed, Lambda mu, mu] with
// Lambda = Sigma^-1.  64 / KP entities per wavefront, lane r of a group
// holding row r; inverses by the symmetric sweep (sweep_inv).
// --------------------------------------------------------------------------
template <int KP>
__device__ __forceinline__ void sweep_inv(double (&m)[KP], const int K, const int r, double *bc) {
    // m (row r of a symmetric positive definite matrix, identity padding) <- row r of its inverse
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        if (k < K) {
            __syncthreads();
            bc[r] = m[k];
            __syncthreads();
            const double p = bc[k];
            const double ip = 1.0 / (p > 0.0 ? p : 1.0);
            const double f = m[k] * ip;
            const bool own = r == k;
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                if (j == k) continue;
                const double bj = bc[j];
                m[j] = own ? bj * ip : m[j] - f * bj;
            }
            m[k] = own ? -ip : f;
        }
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) m[c] = (r < K && c < K) ? -m[c] : (c == r ? 1.0 : 0.0);
}

template <int KP>
__global__ __launch_bounds__(64) void k_gmm_pool(const GmmPoolArgs a) {
    constexpr int G = 64 / KP;
    constexpr int NP = KP * (KP + 1) / 2 + 2 * KP;
    __shared__ __align__(16) double rowb[G][NP];
    __shared__ double bc[G][KP];
    const int lane = threadIdx.x;
    const int h = lane / KP, r = lane % KP;
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    for (int pit = blockIdx.x; G * pit < a.nitems; pit += gridDim.x) {
        const int it = G * pit + h;
        const bool valid = it < a.nitems;
        const int iq = valid ? it : G * pit;
        const int2 item = a.items[iq];
        const int n = item.y;
        const double *ax = a.aux[item.x] + (int64_t)n * 2;
        // pooled mean, components in order
        double mu = 0.0;
        for (int c = 0; c < a.ncomp; ++c) {
            if (a.which[(int64_t)iq * kMaxComp + c] == -2) continue;
            const double *cr = a.comp[item.x] + c * a.plane + (int64_t)n * a.prow;
            mu += ax[c * a.aux_plane] * (r < K ? cr[kk2 + K + r] : 0.0);
        }
        double sig[KP];
#pragma unroll
        for (int j = 0; j < KP; ++j) sig[j] = 0.0;
        for (int c = 0; c < a.ncomp; ++c) {
            const bool pres = a.which[(int64_t)iq * kMaxComp + c] != -2;
            if (__ballot(pres) == 0) continue;       // uniform over the wavefront
            const double *cr = a.comp[item.x] + c * a.plane + (int64_t)n * a.prow;
            const double pi = pres ? ax[c * a.aux_plane] : 0.0;
            __syncthreads();
            if (pres)
                for (int q = r; q < kk2 + 2 * K; q += KP) rowb[h][q] = cr[q];
            __syncthreads();
            double m[KP];
#pragma unroll
            for (int j = 0; j < KP; ++j)
                m[j] = (pres && r < K && j < K) ? rowb[h][r >= j ? tri(r, j) : tri(j, r)] : (j == r ? 1.0 : 0.0);
            const double dr = (pres && r < K) ? rowb[h][kk2 + K + r] - mu : 0.0;
            sweep_inv<KP>(m, K, r, bc[h]);
            __syncthreads();
            bc[h][r] = dr;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < KP; ++j)
                if (r < K && j < K) sig[j] += pi * (m[j] + dr * bc[h][j]);
        }
#pragma unroll
        for (int j = 0; j < KP; ++j) sig[j] = (r < K && j < K) ? sig[j] : (j == r ? 1.0 : 0.0);
        sweep_inv<KP>(sig, K, r, bc[h]);
        __syncthreads();
        bc[h][r] = mu;
        __syncthreads();
        double eta = 0.0;
#pragma unroll
        for (int j = 0; j < KP; ++j)
            if (j < K) eta += sig[j] * bc[h][j];
        __syncthreads();
        if (r < K) {
#pragma unroll
            for (int j = 0; j < KP; ++j)
                if (j <= r) rowb[h][tri(r, j)] = sig[j];
            rowb[h][kk2 + r] = eta;
            rowb[h][kk2 + K + r] = mu;
        }
        __syncthreads();
        if (valid) {
            double *out = a.out[item.x] + (int64_t)n * a.prow;
            for (int q = r; q < kk2 + 2 * K; q += KP) out[q] = rowb[h][q];
        }
    }
}

// --------------------------------------------------------------------------
// k_gmm_pick: the mixture prior of a row for this sweep (Sec. 5.1): the
// component c of largest log pi_c + log det(Lambda_c) / 2 - (x - mu_c)^T
// Lambda_c (x - mu_c) / 2 at the row's current value x (the Gaussian
// densities' common constant cancels; lowest index on ties; force0: the
// largest component), copied into the side's own prior rows.  64 / KP rows
// per wavefront, lane r of a group computing entry r of Lambda_c (x - mu_c).
// --------------------------------------------------------------------------
template <typename Ts, int KP>
__global__ __launch_bounds__(64) void k_gmm_pick(const GmmPickArgs a) {
    constexpr int G = 64 / KP;
    __shared__ double bc[G][KP];
    const int lane = threadIdx.x;
    const int h = lane / KP, r = lane % KP;
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    for (int pit = blockIdx.x; G * pit < a.nitems; pit += gridDim.x) {
        const int it = G * pit + h;
        const bool valid = it < a.nitems;
        const int2 item = a.items[valid ? it : G * pit];
        const GmmSide &gs = a.gsides[item.x];
        const int n = item.y;
        const Ts *st = reinterpret_cast<const Ts *>(gs.state) + (int64_t)n * a.ks_state;
        const double xr = r < K ? elem_to_d(st[r]) : 0.0;
        int best = 0;
        if (!a.force0) {
            double bval = -INFINITY;
            for (int c = 0; c < a.ncomp; ++c) {
                const double pi = gs.aux[c * a.aux_plane + (int64_t)n * 2];
                const double ldt = gs.aux[c * a.aux_plane + (int64_t)n * 2 + 1];
                const double *cr = gs.src + c * a.plane + (int64_t)n * a.prow;
                const double dr = r < K ? xr - cr[kk2 + K + r] : 0.0;
                __syncthreads();
                bc[h][r] = dr;
                __syncthreads();
                double t = 0.0;
                for (int j = 0; j < K; ++j) t += (r < K ? cr[r >= j ? tri(r, j) : tri(j, r)] : 0.0) * bc[h][j];
                const double qf = group_sum1(dr * t, KP);
                const double v = log(pi > 0.0 ? pi : 1.0) + 0.5 * ldt - 0.5 * qf;
                if (pi > 0.0 && v > bval) {
                    bval = v;
                    best = c;
                }
            }
        }
        if (valid) {
            const double *cr = gs.src + best * a.plane + (int64_t)n * a.prow;
            double *dst = gs.dst + (int64_t)n * a.prow;
            for (int q = r; q < a.prow; q += KP) dst[q] = cr[q];
        }
    }
}

// --------------------------------------------------------------------------
// k_pfac_rows: the factor k_update_group applies, from one moment-matched row
// [Lambda packed, Lambda mu, mu] (FP64): L = chol(Lambda), U = L^-T, written
// as FP32 rows j = 0 .. K-1 of U[r][r + j] (r < K - j, row j at offset
// j K - j (j - 1) / 2), then a flag (1: Lambda positive definite).  Items are
// (side, entity); sides whose rows seed no later stage have no output.
// 64 / KP entities per wavefront, lane r of a group holding row r.  With
// Lambda = L L^T, the factor
// U = L^-T is the upper-triangular factor of Sigma = Lambda^-1 = U U^T, which
// is unique with a positive diagonal; so Sigma comes from the symmetric sweep
// of Lambda over pivots 0 .. K-1 (it leaves -Sigma), and U from Sigma by the
// Cholesky elimination taken from the last pivot to the first:
// U[k][k] = sqrt(S[k][k]), U[r][k] = S[r][k] / U[k][k] (r < k), then
// S[r][j] -= U[r][k] U[j][k] for r, j < k.  The flag is 1 when every pivot of
// both eliminations is positive (Lambda positive definite).  The packed input
// row and the output row pass through LDS so that both are moved contiguously.
// --------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(64) void k_pfac_rows(const PfacArgs a) {
    constexpr int G = 64 / KP;
    constexpr int NP = KP * (KP + 1) / 2;
    __shared__ __align__(16) double pk[G][NP];
    __shared__ __align__(16) float po[G][NP + 1];
    __shared__ double bc[G][KP];
    const int lane = threadIdx.x;
    const int h = lane / KP, r = lane % KP;
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    for (int pit = blockIdx.x; G * pit < a.nitems; pit += gridDim.x) {
        const int it = G * pit + h;
        const bool valid = it < a.nitems;
        const int2 item = a.items[valid ? it : G * pit];
        float *pfo = a.pfout[item.x];
        const bool act = valid && pfo != nullptr;          // uniform per group
        if (__ballot(act) == 0) continue;                   // uniform per wavefront
        __syncthreads();                                    // the previous rows are read
        if (act) {
            const double *row = a.out[item.x] + (int64_t)item.y * a.prow;
            for (int q = r; q < kk2; q += KP) pk[h][q] = row[q];
        }
        __syncthreads();
        double m[KP];
#pragma unroll
        for (int c = 0; c < KP; ++c)
            m[c] = (act && r < K && c < K) ? pk[h][r >= c ? tri(r, c) : tri(c, r)] : (c == r ? 1.0 : 0.0);
        int bad = 0;
        // sweep: m <- -Lambda^-1
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            if (k < K) {
                __syncthreads();
                bc[h][r] = m[k];
                __syncthreads();
                const double p = bc[h][k];
                bad |= !(p > 0.0);
                const double ip = 1.0 / (p > 0.0 ? p : 1.0);
                const double f = m[k] * ip;
                const bool own = r == k;
#pragma unroll
                for (int j = 0; j < KP; ++j) {
                    if (j == k) continue;
                    const double bj = bc[h][j];
                    m[j] = own ? bj * ip : m[j] - f * bj;
                }
                m[k] = own ? -ip : f;
            }
        }
        // Sigma = -m; its upper factor from the last pivot to the first
#pragma unroll
        for (int c = 0; c < KP; ++c) m[c] = -m[c];
#pragma unroll
        for (int k = KP - 1; k >= 0; --k) {
            if (k < K) {
                __syncthreads();
                bc[h][r] = m[k];
                __syncthreads();
                const double d = bc[h][k];
                bad |= !(d > 0.0);
                const double u = d > 0.0 ? sqrt(d) : 1.0;
                const double iu = 1.0 / u;
                const double f = m[k] * iu;                 // U[r][k] for r <= k
#pragma unroll
                for (int j = 0; j < k; ++j) m[j] -= f * (bc[h][j] * iu);
                m[k] = r <= k ? f : 0.0;
            }
        }
        // U[r][r + j] at j K - j (j - 1) / 2 + r, then the flag
#pragma unroll
        for (int c = 0; c < KP; ++c) {
            const int j = c - r;
            if (act && r < K && c < K && j >= 0) po[h][j * K - j * (j - 1) / 2 + r] = (float)m[c];
        }
        if (act && r == 0) po[h][kk2] = bad ? 0.0f : 1.0f;
        __syncthreads();
        if (act)
            for (int q = r; q <= kk2; q += KP) pfo[(int64_t)item.y * a.pfrow + q] = po[h][q];
    }
}


// --------------------------------------------------------------------------
// k_agg: Algorithm 2 for one row of a row (or column) block (FP64), one
// wavefront per row.
// --------------------------------------------------------------------------
// Smallest eigenvalue of the symmetric K x K matrix in S (full, row stride ld,
// destroyed) by cyclic Jacobi rotations (Golub & Van Loan, Sec. 8.5) in the
// parallel ordering of Brent & Luk: a sweep is n - 1 rounds of n/2 rotations
// on disjoint index pairs (n = K rounded up to even; an odd K gets one dummy
// index with zero coupling, which no rotation touches).  Rotations on disjoint
// pairs commute and do not change each other's 2 x 2 blocks, so a round equals
// applying its rotations one after another.  All 64 lanes call it; S needs
// n rows and columns; sc holds n/2 (c, s) pairs, sp n/2 index pairs.
template <int KP>
__device__ double wave_min_eig(double *S, int K, int ld, int lane, double *sc, int *sp) {
    const int n = K + (K & 1);
    if (K & 1) {
        for (int q = lane; q < n; q += 64) {
            S[K * ld + q] = 0.0;
            S[q * ld + K] = 0.0;
        }
    }
    __syncthreads();
    const int half = n / 2;
    // lane's first (pair, index) item of the half * n updates of a phase, and
    // the step to its next one (64 items on)
    const int m0 = lane / n, k0 = lane - m0 * n, dm = 64 / n, dk = 64 - dm * n;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int q = lane; q < K * K; q += 64) {
            const int r = q / K, c = q - r * K;
            const double v = S[r * ld + c] * S[r * ld + c];
            tot += v;
            if (r != c) off += v;
        }
        off = group_sum1(off, 64);
        tot = group_sum1(tot, 64);
        // converged: the off-diagonal Frobenius norm at most 1e-12 of the whole,
        // so the diagonal holds every eigenvalue to 1e-12 ||S||_F (Weyl) and in
        // practice to its square; rounding alone keeps the off-diagonal mass
        // near (K - 1) eps^2 of the whole, which a tighter bound would not reach
        if (off <= 1e-24 * tot) break;
        for (int rd = 0; rd < n - 1; ++rd) {
            if (lane < half) {
                int p, q;
                if (lane == 0) {
                    p = rd;
                    q = n - 1;
                } else {
                    p = (rd + lane) % (n - 1);
                    q = (rd - lane + n - 1) % (n - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double apq = S[p * ld + q];
                double c = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    const double th = (S[q * ld + q] - S[p * ld + p]) / (2.0 * apq);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sn = t * c;
                }
                sc[2 * lane] = c;
                sc[2 * lane + 1] = sn;
                sp[2 * lane] = p;
                sp[2 * lane + 1] = q;
            }
            __syncthreads();
            // columns p, q of every row
            for (int m = m0, k = k0; m < half;) {
                const int p = sp[2 * m], q = sp[2 * m + 1];
                const double c = sc[2 * m], sn = sc[2 * m + 1];
                const double akp = S[k * ld + p], akq = S[k * ld + q];
                S[k * ld + p] = c * akp - sn * akq;
                S[k * ld + q] = sn * akp + c * akq;
                m += dm;
                k += dk;
                if (k >= n) {
                    k -= n;
                    ++m;
                }
            }
            __syncthreads();
            // rows p, q of every column
            for (int m = m0, k = k0; m < half;) {
                const int p = sp[2 * m], q = sp[2 * m + 1];
                const double c = sc[2 * m], sn = sc[2 * m + 1];
                const double apk = S[p * ld + k], aqk = S[q * ld + k];
                S[p * ld + k] = c * apk - sn * aqk;
                S[q * ld + k] = sn * apk + c * aqk;
                m += dm;
                k += dk;
                if (k >= n) {
                    k -= n;
                    ++m;
                }
            }
            __syncthreads();
        }
    }
    double m = S[0];
    for (int k = 1; k < K; ++k) m = fmin(m, S[k * ld + k]);
    __syncthreads();
    return m;
}

// Entry (r, c) of a packed lower-triangular row-major symmetric matrix.
__device__ __forceinline__ double packed_sym(const double *P, int r, int c) {
    return r >= c ? P[tri(r, c)] : P[tri(c, r)];
}

// Algorithm 2 for one row: Lambda* = (2 - J) Lambda_b + sum_j Lambda~_j and
// Lambda* mu* = (2 - J) Lambda_b mu_b + sum_j Lambda~_j mu_j, where
// Lambda~_j = Lambda_j when Lambda_j - Lambda_b is positive definite and
// (Lambda_j - Lambda_b) + (|lambda_min| + eps) I + Lambda_b otherwise,
// eps = 1e-6 tr(Lambda_b) / K.  The rows (packed [Lambda, Lambda mu, mu]) are
// read from global memory; the positive-definiteness test is a register
// Cholesky with a zero pivot threshold.
template <int KP>
__global__ __launch_bounds__(64) void k_agg(const AggArgs a) {
    constexpr int LD = KP + 2;                     // doubles; 16-byte rows
    __shared__ __align__(16) double sLb[KP * LD];  // Lambda_b (full)
    __shared__ __align__(16) double sA[KP * LD];   // D_j, its factor, Jacobi scratch
    __shared__ __align__(16) double sS[KP * LD];   // Lambda* (lower, identity padding)
    __shared__ double mub[KP], rhs[KP], dg[KP], sinv[KP], zero[KP], sc[KP];
    __shared__ int sp[KP];
    int lane = threadIdx.x;
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    const bool own = lane < KP;
    for (int it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        asm volatile("" : "+v"(lane));
        int z0 = 0;
        asm volatile("" : "+v"(z0));
        z0 &= ~15;
        const int2 item = a.items[it];
        const AggJob &jb = a.jobs[item.x];
        const int n = item.y;
        const double *brow = jb.base + (int64_t)n * a.prow;
        double *out = a.out + (jb.out_off + n) * K;
        if (jb.nsib == 0) {
            if (lane < K) out[lane] = brow[kk2 + K + lane];
            continue;
        }
        for (int q = lane; q < KP * KP; q += 64) {
            const int r = q / KP, c = q - r * KP;
            sLb[r * LD + c] = (r < K && c < K) ? packed_sym(brow, r, c) : 0.0;
        }
        if (own) {
            mub[lane] = lane < K ? brow[kk2 + K + lane] : 0.0;
            zero[lane] = 0.0;
        }
        __syncthreads();
        double tr = 0.0;
        for (int k = 0; k < K; ++k) tr += sLb[k * LD + k];
        const double eps = 1e-6 * tr / (double)K;
        const double cb = 2.0 - (double)(jb.nsib + 1);
        for (int q = lane; q < KP * KP; q += 64) {
            const int r = q / KP, c = q - r * KP;
            sS[r * LD + c] = (r < K && c < K) ? cb * sLb[r * LD + c] : (double)(r == c);
        }
        if (own) {
            double s2 = 0.0;
            for (int c = 0; c < K; ++c) s2 += sLb[lane * LD + c] * mub[c];
            rhs[lane] = lane < K ? cb * s2 : 0.0;
        }
        __syncthreads();
        for (int s = 0; s < jb.nsib; ++s) {
            const double *srow = jb.sib[s] + (int64_t)n * a.prow;
            // D_j = Lambda_j - Lambda_b (lower, identity padding)
            for (int q = lane; q < KP * KP; q += 64) {
                const int r = q / KP, c = q - r * KP;
                sA[r * LD + c] = (r < K && c < K) ? packed_sym(srow, r, c) - sLb[r * LD + c] : (double)(r == c);
            }
            __syncthreads();
            if (own) dg[lane] = sA[lane * LD + lane];
            __syncthreads();
            double rr[KP];
            const bool pd = chol_rows<KP, double>(sA, LD, sA, LD, dg, sinv, 0.0, lane, z0, rr);
            __syncthreads();
            double shift = 0.0;
            if (!pd) {
                for (int q = lane; q < KP * KP; q += 64) {
                    const int r = q / KP, c = q - r * KP;
                    sA[r * LD + c] = (r < K && c < K) ? packed_sym(srow, r, c) - sLb[r * LD + c] : 0.0;
                }
                __syncthreads();
                const double lmin = wave_min_eig<KP>(sA, K, LD, lane, sc, sp);
                shift = fabs(lmin) + eps;
                if (lane == 0) atomicAdd(a.corrections, 1);
            }
            // Lambda~_j into Lambda*, Lambda~_j mu_j into the right-hand side
            for (int q = lane; q < K * K; q += 64) {
                const int r = q / K, c = q - r * K;
                double v = packed_sym(srow, r, c);
                if (!pd) v = ((v - sLb[r * LD + c]) + (r == c ? shift : 0.0)) + sLb[r * LD + c];
                sS[r * LD + c] += v;
            }
            if (lane < K) {
                double s2 = 0.0;
                for (int c = 0; c < K; ++c) {
                    double v = packed_sym(srow, lane, c);
                    if (!pd) v = ((v - sLb[lane * LD + c]) + (lane == c ? shift : 0.0)) + sLb[lane * LD + c];
                    s2 += v * srow[kk2 + K + c];
                }
                rhs[lane] += s2;
            }
            __syncthreads();
        }
        // mu* = Lambda*^-1 (Lambda* mu*)
        if (own) dg[lane] = sS[lane * LD + lane];
        __syncthreads();
        factor_solve_regs<KP, double>(sS, LD, sS, LD, rhs, zero, dg, sinv, 0.0, K, lane);
        if (lane < K) out[lane] = rhs[lane];
        __syncthreads();
    }
}

// Positive-definiteness test of the symmetric K x K matrix whose row r the
// group's lane r holds in d[] (destroyed; identity padding beyond K): the
// symmetric elimination A <- A22 - a21 a21^T / a11, whose pivots are the
// squares of the Cholesky pivots.  Column k of the trailing matrix is its row
// k, so each step broadcasts the lanes' entries k through the group's LDS row
// bc.  Returns false when a pivot is not positive, as the factorisation would.
template <int KP>
__device__ __forceinline__ bool grp_pd_test(double (&d)[KP], const int K, const int r, double *bc) {
    int bad = 0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        if (k < K) {
            __syncthreads();                        // the previous column is read
            bc[r] = d[k];
            __syncthreads();
            const double p = bc[k];
            bad |= !(p > 0.0);
            const double f = d[k] / (p > 0.0 ? p : 1.0);
#pragma unroll
            for (int j = k + 1; j < KP; ++j) d[j] -= f * bc[j];
        }
    }
    return bad == 0;
}

// Smallest eigenvalue of the symmetric K x K matrix whose row r the group's
// lane r holds in a[] (destroyed).  Householder reduction to a tridiagonal T
// (Golub and Van Loan, Sec. 8.3.1) with the rows in registers: step k
// reflects column k below the diagonal onto its first entry and applies the
// reflector from both sides as the rank-two update A - v w^T - w v^T.  Then
// bisection on Sturm counts of T (the number of negative pivots of T - s I;
// Golub and Van Loan, Sec. 8.4.1), KP shifts at a time, one per lane: each
// round keeps the subinterval where the count first reaches one, until it is
// within two units of roundoff of ||T||.  gl0 is the group's first lane; vb,
// wb, td, te hold KP doubles of the group's LDS.
template <int KP>
__device__ double grp_min_eig(double (&a)[KP], const int K, const int r, const int gl0, double *vb, double *wb,
                              double *td, double *te) {
    const unsigned long long gmask = KP == 64 ? ~0ull : (((1ull << KP) - 1) << gl0);
#pragma unroll
    for (int k = 0; k < KP - 2; ++k) {
        if (k < K - 2) {
            const double x = r > k ? a[k] : 0.0;    // column k below the diagonal
            const double x1 = __shfl(x, gl0 + k + 1, 64);
            const double s2 = group_sum1(r > k + 1 ? x * x : 0.0, KP);
            double alpha = x1, beta = 0.0, v = 0.0;
            if (s2 > 0.0) {                          // otherwise column k is reduced already
                const double mu = sqrt(x1 * x1 + s2);
                alpha = x1 <= 0.0 ? mu : -mu;
                const double v1 = x1 - alpha;
                beta = 2.0 / (v1 * v1 + s2);
                v = r == k + 1 ? v1 : x;
            }
            if (r == 0) te[k] = alpha;
            __syncthreads();                         // the previous step's vb, wb are read
            vb[r] = v;
            __syncthreads();
            double p = 0.0;
#pragma unroll
            for (int j = 0; j < KP; ++j) p += a[j] * vb[j];
            p *= beta;
            const double pv = group_sum1(p * v, KP);
            const double w = r > k ? p - 0.5 * beta * pv * v : 0.0;
            wb[r] = w;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < KP; ++j) a[j] -= v * wb[j] + w * vb[j];
        }
    }
    // diagonal and last off-diagonal entry of T
    double dr = 0.0, el = 0.0;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        dr = j == r ? a[j] : dr;
        el = j == K - 2 ? a[j] : el;
    }
    if (r < K) td[r] = dr;
    if (K >= 2 && r == K - 1) te[K - 2] = el;
    __syncthreads();
    // Gershgorin bounds: every eigenvalue lies above lo, and the smallest one
    // lies below the smallest diagonal entry
    double lo = 1e300, hi = 1e300, tn = 0.0, e2max = 0.0;
    if (r < K) {
        const double em = r > 0 ? fabs(te[r - 1]) : 0.0, ep = r < K - 1 ? fabs(te[r]) : 0.0;
        lo = td[r] - em - ep;
        hi = td[r];
        tn = fabs(td[r]) + em + ep;
        e2max = ep * ep;
    }
#pragma unroll
    for (int o = 1; o < KP; o <<= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmin(hi, __shfl_xor(hi, o, 64));
        tn = fmax(tn, __shfl_xor(tn, o, 64));
        e2max = fmax(e2max, __shfl_xor(e2max, o, 64));
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
    const double tol = 4.440892098500626e-16 * tn;
    // every group runs the same number of rounds; a finished group keeps its interval
    for (int round = 0; round < 64; ++round) {
        const bool open = hi - lo > tol;
        if (__ballot(open) == 0) break;
        const double width = hi - lo;
        const double sg = lo + (double)(r + 1) * width / (double)(KP + 1);
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < K; ++i) {
            double t = td[i] - sg;
            if (i > 0) {
                // e^2 / q through the reciprocal with one Newton step: the count
                // only needs the sign of each pivot
                const double rc0 = __builtin_amdgcn_rcp(q);
                const double rc = fma(rc0, fma(-q, rc0, 1.0), rc0);
                t -= te[i - 1] * te[i - 1] * rc;
            }
            q = fabs(t) < pivmin ? -pivmin : t;
            cnt += q < 0.0;
        }
        const unsigned long long hit = __ballot(cnt > 0) & gmask;
        const int first = hit ? (int)(__builtin_ctzll(hit) - gl0) : KP;
        if (open) {
            const double nhi = first < KP ? lo + (double)(first + 1) * width / (double)(KP + 1) : hi;
            const double nlo = first > 0 ? lo + (double)first * width / (double)(KP + 1) : lo;
            lo = nlo;
            hi = nhi;
        }
    }
    return 0.5 * (lo + hi);
}

// k_agg_rows: Algorithm 2 for one row per wavefront (K <= KP <= 32), the
// siblings 64 / KP at a time, one per group of KP lanes (lane r of a group
// holds row r).  A group stages D_j = Lambda_j - Lambda_b in its LDS block,
// tests it (grp_pd_test) and, when the test fails, takes lambda_min(D_j) from
// grp_min_eig; Lambda~_j and Lambda~_j mu_j then replace D_j there, and every
// lane adds the groups' blocks into its row of Lambda* in sibling order, as
// the sequential algorithm does.  mu* = Lambda*^-1 (Lambda* mu*) by
// factor_solve_regs.
template <int KP>
__global__ __launch_bounds__(64, 2) void k_agg_rows(const AggArgs a) {
    constexpr int G = 64 / KP;
    constexpr int LD = KP + 2;                      // doubles; 16-byte rows
    __shared__ __align__(16) double sT[G][KP * LD];
    __shared__ double vb[G][KP], wb[G][KP], td[G][KP], te[G][KP], rv[G][KP];
    __shared__ double rhs[KP], dg[KP], sinv[KP], zero[KP];
    int lane = threadIdx.x;
    const int g = lane / KP, r = lane % KP, gl0 = g * KP;
    const int K = a.K;
    const int kk2 = K * (K + 1) / 2;
    for (int it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const int2 item = a.items[it];
        const AggJob &jb = a.jobs[item.x];
        const int n = item.y;
        const double *brow = jb.base + (int64_t)n * a.prow;
        double *out = a.out + (jb.out_off + n) * K;
        if (jb.nsib == 0) {
            if (lane < K) out[lane] = brow[kk2 + K + lane];
            continue;
        }
        double tr = 0.0;
        for (int k = 0; k < K; ++k) tr += brow[tri(k, k)];
        const double eps = 1e-6 * tr / (double)K;
        const double cb = 2.0 - (double)(jb.nsib + 1);
        // row r of Lambda* = (2 - J) Lambda_b + ..., and of its right-hand side
        double acc[KP];
        double hr = 0.0;
        {
            double s2 = 0.0;
#pragma unroll
            for (int c = 0; c < KP; ++c) {
                const double lb = (r < K && c < K) ? packed_sym(brow, r, c) : 0.0;
                acc[c] = (r < K && c < K) ? cb * lb : (c == r ? 1.0 : 0.0);
                if (c < K) s2 += lb * brow[kk2 + K + c];
            }
            hr = r < K ? cb * s2 : 0.0;
        }
        for (int s0 = 0; s0 < jb.nsib; s0 += G) {
            const int s = s0 + g;
            const bool act = s < jb.nsib;
            const double *srow = jb.sib[act ? s : s0] + (int64_t)n * a.prow;
            __syncthreads();                        // the previous siblings' blocks are read
            for (int q = r; q < K * K; q += KP) {
                const int rr = q / K, cc = q - rr * K;
                sT[g][rr * LD + cc] = packed_sym(srow, rr, cc) - packed_sym(brow, rr, cc);
            }
            __syncthreads();
            double d[KP];
#pragma unroll
            for (int c = 0; c < KP; ++c) d[c] = (r < K && c < K) ? sT[g][r * LD + c] : (c == r ? 1.0 : 0.0);
            const bool pd = grp_pd_test<KP>(d, K, r, vb[g]);
            double shift = 0.0;
            if (__ballot(act && !pd) != 0) {
#pragma unroll
                for (int c = 0; c < KP; ++c) d[c] = (r < K && c < K) ? sT[g][r * LD + c] : (c == r ? 1.0 : 0.0);
                const double lmin = grp_min_eig<KP>(d, K, r, gl0, vb[g], wb[g], td[g], te[g]);
                shift = fabs(lmin) + eps;
            }
            if (act && !pd && r == 0) atomicAdd(a.corrections, 1);
            // Lambda~_j (row r) over D_j, and Lambda~_j mu_j
            double s2 = 0.0;
            for (int c = 0; c < K; ++c) {
                double v = packed_sym(srow, r < K ? r : 0, c);
                if (!pd) v = (sT[g][r * LD + c] + (r == c ? shift : 0.0)) + packed_sym(brow, r < K ? r : 0, c);
                s2 += v * srow[kk2 + K + c];
                if (r < K) sT[g][r * LD + c] = v;
            }
            rv[g][r] = s2;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (s0 + q < jb.nsib) {
#pragma unroll
                    for (int c = 0; c < KP; ++c)
                        if (r < K && c < K) acc[c] += sT[q][r * LD + c];
                    if (r < K) hr += rv[q][r];
                }
            }
        }
        // mu* = Lambda*^-1 (Lambda* mu*)
        __syncthreads();
        if (g == 0) {
#pragma unroll
            for (int c = 0; c < KP; ++c) sT[0][r * LD + c] = acc[c];
            rhs[r] = hr;
            zero[r] = 0.0;
            double dd = 0.0;
#pragma unroll
            for (int c = 0; c < KP; ++c) dd = c == r ? acc[c] : dd;
            dg[r] = dd;
        }
        __syncthreads();
        factor_solve_regs<KP, double>(sT[0], LD, sT[0], LD, rhs, zero, dg, sinv, 0.0, K, lane);
        if (lane < K) out[lane] = rhs[lane];
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// k_predict: y_hat = y_bar + mu*_x^T mu*_w (FP64), one thread per pair.
// --------------------------------------------------------------------------
__device__ __forceinline__ float predict_one(const double *x, const double *w, int K, double ybar) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += x[k] * w[k];
    return (float)(ybar + s);
}

__global__ __launch_bounds__(256) void k_predict(const PredictArgs a) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.n;
         q += (int64_t)gridDim.x * blockDim.x)
        a.out[q] = predict_one(a.mux + a.xslot[q] * a.K, a.muw + a.wslot[q] * a.K, a.K, a.ybar);
}

// The same from original ids, mapped to positions on the device.
__global__ __launch_bounds__(256) void k_predict_ids(const PredictIdsArgs a) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.n;
         q += (int64_t)gridDim.x * blockDim.x)
        a.out[q] = predict_one(a.mux + a.row_pos[a.row[q]] * a.K, a.muw + a.col_pos[a.col[q]] * a.K, a.K,
                               a.ybar);
}

// Staging of the allocation-free prediction entry point: one array per device,
// held until the process ends.  Host code never passes this name to a kernel
// (on the host it is only a stand-in for the symbol): it takes the device
// address from scratch_address().
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// End of a sweep: next sweep index and its sample slot (kept when
// t >= burnin, (t - burnin) % thin == 0 and the store is not full).
__global__ void k_advance(SweepState *ss, int32_t *fb_counts) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sweep_advance(ss, fb_counts);
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
int32_t capacity_for(int32_t K) {
    const int32_t caps[] = {2, 4, 6, 8, 10, 12, 16, 32, 64};
    for (int32_t c : caps)
        if (K <= c) return c;
    return -1;
}

int32_t stride_for(int32_t kc, int32_t elem_bytes) {
    const int32_t v = 16 / elem_bytes;
    return kc >= 32 ? kc : ((kc + v - 1) / v) * v;
}

static inline int grid_for(int64_t work, int per, int cap) {
    int64_t g = (work + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <int KC, bool SSE>
static hipError_t upd_reg_kc_sse(int32_t prec, const UpdArgs &a, int32_t ntiles, hipStream_t s) {
    switch (prec) {
    case kP64:
        // FP64 above K = 12 exceeds the register file; the wavefront kernel serves it
        if constexpr (KC > 12) return hipErrorInvalidValue;
        else hipLaunchKernelGGL((k_update_reg<KC, kP64, SSE>), dim3(ntiles), dim3(256), 0, s, a);
        break;
    case kP32: hipLaunchKernelGGL((k_update_reg<KC, kP32, SSE>), dim3(ntiles), dim3(256), 0, s, a); break;
    case kPBF: hipLaunchKernelGGL((k_update_reg<KC, kPBF, SSE>), dim3(ntiles), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KC>
static hipError_t upd_reg_kc(int32_t prec, const UpdArgs &a, int32_t ntiles, hipStream_t s) {
    return a.sse_col ? upd_reg_kc_sse<KC, true>(prec, a, ntiles, s)
                     : upd_reg_kc_sse<KC, false>(prec, a, ntiles, s);
}

hipError_t launch_update_reg(int32_t kc, int32_t prec, const UpdArgs &a, int32_t ntiles, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    switch (kc) {
    case 2: return upd_reg_kc<2>(prec, a, ntiles, s);
    case 4: return upd_reg_kc<4>(prec, a, ntiles, s);
    case 6: return upd_reg_kc<6>(prec, a, ntiles, s);
    case 8: return upd_reg_kc<8>(prec, a, ntiles, s);
    case 10: return upd_reg_kc<10>(prec, a, ntiles, s);
    case 12: return upd_reg_kc<12>(prec, a, ntiles, s);
    case 16: return upd_reg_kc<16>(prec, a, ntiles, s);
    default: return hipErrorInvalidValue;
    }
}

template <int KP>
static hipError_t upd_wave_kp(int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s, bool vgram) {
    constexpr bool kMF = KP >= 32;   // BF16 state: Gram on MFMA
    switch (prec) {
    case kP64: hipLaunchKernelGGL((k_update_wave<KP, kP64, false>), dim3(grid), dim3(64), 0, s, a); break;
    case kP32: hipLaunchKernelGGL((k_update_wave<KP, kP32, false>), dim3(grid), dim3(64), 0, s, a); break;
    case kPBF:
        if (kMF && !vgram)
            hipLaunchKernelGGL((k_update_wave<KP, kPBF, kMF>), dim3(grid), dim3(64), 0, s, a);
        else
            hipLaunchKernelGGL((k_update_wave<KP, kPBF, false>), dim3(grid), dim3(64), 0, s, a);
        break;
    case kPFB32: hipLaunchKernelGGL((k_update_wave<KP, kPFB32, false>), dim3(grid), dim3(64), 0, s, a); break;
    case kPFB16: hipLaunchKernelGGL((k_update_wave<KP, kPFB16, false>), dim3(grid), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update_duo(int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s, bool mf) {
    if (grid <= 0) return hipSuccess;
    switch (prec) {
    case kP32:
        if (mf) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_update_duo<kP32, false>), dim3(grid), dim3(64), 0, s, a);
        break;
    case kPBF:
        if (mf) hipLaunchKernelGGL((k_update_duo<kPBF, true>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_update_duo<kPBF, false>), dim3(grid), dim3(64), 0, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update_group(int32_t kp, int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s) {
    if (grid <= 0 || a.ngroups <= 0) return hipSuccess;
    if (a.K > kp || (kp != 32 && kp != 64)) return hipErrorInvalidValue;
    // each workgroup clears its dense factor copy and maps the stored entries
    // once, then strides over groups: about two rounds of resident
    // workgroups (256 CUs, 16 at a time) spread that set-up over many groups
    grid = std::min(grid, 8192);
    switch (prec) {
    case kP32:
        if (kp == 32) hipLaunchKernelGGL((k_update_group<kP32, 32>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_update_group<kP32, 64>), dim3(grid), dim3(64), 0, s, a);
        break;
    case kPBF:
        if (kp == 32) hipLaunchKernelGGL((k_update_group<kPBF, 32>), dim3(grid), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_update_group<kPBF, 64>), dim3(grid), dim3(64), 0, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int32_t lowrank_max_nnz() { return kLowRankNnz; }
int32_t lowrank_small_nnz() { return kLowRankSmall; }

hipError_t launch_update_wave(int32_t kp, int32_t prec, const UpdArgs &a, int32_t grid, hipStream_t s, bool vgram) {
    if (grid <= 0) return hipSuccess;
    if (kp <= 16) return upd_wave_kp<16>(prec, a, grid, s, vgram);
    if (kp <= 32) return upd_wave_kp<32>(prec, a, grid, s, vgram);
    if (kp <= 64) return upd_wave_kp<64>(prec, a, grid, s, vgram);
    return hipErrorInvalidValue;
}

template <int KC>
static hipError_t sse_kc(int32_t prec, const SseArgs &a, int32_t ntiles, hipStream_t s) {
    if (prec == kP64)
        hipLaunchKernelGGL((k_sse<KC, kP64>), dim3(ntiles), dim3(256), 0, s, a);
    else if (prec == kPBF)
        hipLaunchKernelGGL((k_sse<KC, kPBF>), dim3(ntiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_sse<KC, kP32>), dim3(ntiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sse(int32_t kc, int32_t prec, const SseArgs &a, int32_t ntiles, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    switch (kc) {
    case 2: return sse_kc<2>(prec, a, ntiles, s);
    case 4: return sse_kc<4>(prec, a, ntiles, s);
    case 6: return sse_kc<6>(prec, a, ntiles, s);
    case 8: return sse_kc<8>(prec, a, ntiles, s);
    case 10: return sse_kc<10>(prec, a, ntiles, s);
    case 12: return sse_kc<12>(prec, a, ntiles, s);
    case 16: return sse_kc<16>(prec, a, ntiles, s);
    case 32: return sse_kc<32>(prec, a, ntiles, s);
    case 64: return sse_kc<64>(prec, a, ntiles, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gram_part(int32_t kp, const GramPartArgs &a, hipStream_t s) {
    if (a.nseg <= 0) return hipSuccess;
    if (kp == 32)
        hipLaunchKernelGGL(k_gram_part<32>, dim3(a.nseg), dim3(64), 0, s, a);
    else if (kp == 64)
        hipLaunchKernelGGL(k_gram_part<64>, dim3(a.nseg), dim3(64), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename Ts, int KB, int WB>
static void stats_mfma(const StatsArgs &a, int32_t njobs, hipStream_t s) {
    const size_t lds = sizeof(double) * WB * (a.K + a.K * (a.K + 1) / 2);
    hipLaunchKernelGGL((k_stats_mfma<Ts, KB, WB>), dim3(njobs), dim3(64 * WB), lds, s, a);
}
template <typename Ts>
static hipError_t stats_ts(const StatsArgs &a, int32_t njobs, hipStream_t s) {
    // wavefronts per block: the LDS holding their sums stays within 64 KB
    if (a.K <= 16) stats_mfma<Ts, 1, 16>(a, njobs, s);
    else if (a.K <= 32) stats_mfma<Ts, 2, 8>(a, njobs, s);
    else if (a.K <= 64) stats_mfma<Ts, 4, 2>(a, njobs, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}
hipError_t launch_stats(int32_t prec, const StatsArgs &a, int32_t njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (prec == kP64) return stats_ts<double>(a, njobs, s);
    if (prec == kPBF) return stats_ts<uint16_t>(a, njobs, s);
    return stats_ts<float>(a, njobs, s);
}

hipError_t launch_reduce(const ReduceJob *jobs, int32_t njobs, int32_t max_width, hipStream_t s,
                         const NoiseArgs *noise) {
    const int nn = noise ? noise->njobs : 0;
    if (njobs + nn <= 0) return hipSuccess;
    const int slices = (max_width + kReduceSlice - 1) / kReduceSlice;
    NoiseArgs na{};
    if (noise) na = *noise;
    hipLaunchKernelGGL(k_reduce, dim3(njobs + nn, slices < 1 ? 1 : slices), dim3(kReduceThreads), 0, s, jobs,
                       njobs, na);
    return hipGetLastError();
}

hipError_t launch_hyper(const HyperArgs &a, int32_t njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (a.K <= 8)
        hipLaunchKernelGGL(k_hyper<8>, dim3(njobs), dim3(64), 0, s, a);
    else if (a.K <= 12)
        hipLaunchKernelGGL(k_hyper<12>, dim3(njobs), dim3(64), 0, s, a);
    else if (a.K <= 16)
        hipLaunchKernelGGL(k_hyper<16>, dim3(njobs), dim3(64), 0, s, a);
    else if (a.K <= 32)
        hipLaunchKernelGGL(k_hyper<32>, dim3(njobs), dim3(64), 0, s, a);
    else if (a.K <= 64)
        hipLaunchKernelGGL(k_hyper<64>, dim3(njobs), dim3(64), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_init(int32_t prec, const InitArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    const int g = grid_for(a.nitems, 256, 65536);
    if (prec == kP64)
        hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(256), 0, s, a);
    else if (prec == kPBF)
        hipLaunchKernelGGL(k_init<uint16_t>, dim3(g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pfac(int32_t kp, const PfacArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    const int g = grid_for(a.nitems, 1, 65536);
    if (a.K > kp) return hipErrorInvalidValue;
    if (kp <= 32) hipLaunchKernelGGL((k_pfac_rows<32>), dim3(grid_for((a.nitems + 1) / 2, 1, 65536)), dim3(64), 0,
                                     s, a);
    else if (kp <= 64) hipLaunchKernelGGL((k_pfac_rows<64>), dim3(g), dim3(64), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_tau_scale(int32_t prec, const TauColArgs &a, hipStream_t s) {
    if (a.njobs <= 0) return hipSuccess;
    const dim3 grid(256, a.njobs);
    if (prec == kP64) hipLaunchKernelGGL((k_tau_scale<double, double>), grid, dim3(256), 0, s, a);
    else if (prec == kP32) hipLaunchKernelGGL((k_tau_scale<float, float>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_tau_cols(const TauColArgs &a, hipStream_t s) {
    if (a.njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tau_cols, dim3(16, a.njobs), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lmeans(int32_t prec, const LmeansArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    if (a.K > 32 || a.S > kLmMaxS || a.ncomp < 1 || a.ncomp > kMaxComp) return hipErrorInvalidValue;
    const dim3 grid((a.nitems + 63) / 64);
    const bool d = prec == kP64;
    if (a.K <= 8) {
        if (d) hipLaunchKernelGGL((k_lmeans<double, 8>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_lmeans<float, 8>), grid, dim3(64), 0, s, a);
    } else if (a.K <= 16) {
        if (d) hipLaunchKernelGGL((k_lmeans<double, 16>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_lmeans<float, 16>), grid, dim3(64), 0, s, a);
    } else {
        if (d) hipLaunchKernelGGL((k_lmeans<double, 32>), grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_lmeans<float, 32>), grid, dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_gmm_pool(const GmmPoolArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    if (a.K > 32) return hipErrorInvalidValue;
    if (a.K <= 16) hipLaunchKernelGGL(k_gmm_pool<16>, dim3(grid_for((a.nitems + 3) / 4, 1, 65536)), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_gmm_pool<32>, dim3(grid_for((a.nitems + 1) / 2, 1, 65536)), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gmm_pick(int32_t prec, const GmmPickArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    if (a.K > 32) return hipErrorInvalidValue;
    const dim3 g16(grid_for((a.nitems + 3) / 4, 1, 65536)), g32(grid_for((a.nitems + 1) / 2, 1, 65536));
    if (a.K <= 16) {
        if (prec == kP64) hipLaunchKernelGGL((k_gmm_pick<double, 16>), g16, dim3(64), 0, s, a);
        else if (prec == kP32) hipLaunchKernelGGL((k_gmm_pick<float, 16>), g16, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_gmm_pick<uint16_t, 16>), g16, dim3(64), 0, s, a);
    } else {
        if (prec == kP64) hipLaunchKernelGGL((k_gmm_pick<double, 32>), g32, dim3(64), 0, s, a);
        else if (prec == kP32) hipLaunchKernelGGL((k_gmm_pick<float, 32>), g32, dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_gmm_pick<uint16_t, 32>), g32, dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_mm(int32_t prec, const MmArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    const int g = grid_for(a.nitems, 1, 65536);
    const bool d = prec == kP64;
    if (a.K <= 16) {
        const int g4 = grid_for((a.nitems + 3) / 4, 1, 65536);
        if (d) hipLaunchKernelGGL((k_mm_rows<double, 16>), dim3(g4), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_mm_rows<float, 16>), dim3(g4), dim3(64), 0, s, a);
    } else if (a.K <= 32) {
        const int g2 = grid_for((a.nitems + 1) / 2, 1, 65536);
        if (d) hipLaunchKernelGGL((k_mm_rows<double, 32>), dim3(g2), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_mm_rows<float, 32>), dim3(g2), dim3(64), 0, s, a);
    } else {
        if (d) hipLaunchKernelGGL((k_mm<double, 64>), dim3(g), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_mm<float, 64>), dim3(g), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_agg(const AggArgs &a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    const dim3 grid(grid_for(a.nitems, 1, 65536));
    if (a.K <= 16) hipLaunchKernelGGL(k_agg_rows<16>, grid, dim3(64), 0, s, a);
    else if (a.K <= 32) hipLaunchKernelGGL(k_agg_rows<32>, grid, dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_agg<64>, grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_predict(const PredictArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict, dim3(grid_for(a.n, 256, 65536)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_predict_ids(const PredictIdsArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict_ids, dim3(grid_for(a.n, 256, 65536)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t scratch_address(void **p) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = q;
    }
    *p = addr[dev];
    return hipSuccess;
}

hipError_t launch_advance(SweepState *ss, int32_t *fb_counts, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ss, fb_counts);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace bmf
