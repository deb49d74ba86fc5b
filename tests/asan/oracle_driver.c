/*
 * Exercises every public function of the C oracle on small seeded inputs, for
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure: tests/test_sanitizers.py compiles and runs it).  Exits 0
 * when every call returns; the sanitizers abort on the first fault.
 */
#include "../../oracle/bmf_oracle.c"

#include <stdio.h>

static uint64_t st = 88172645463325252ull;
static double unif(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    const int R = 37, C = 23, K = 5, S = 30;
    /* a sparse block: CSR of about a third of the cells, some rows empty */
    int64_t *ptr = malloc(sizeof(int64_t) * (R + 1));
    int32_t *idx = malloc(sizeof(int32_t) * R * C);
    double *val = malloc(sizeof(double) * R * C);
    int64_t nz = 0;
    ptr[0] = 0;
    for (int r = 0; r < R; ++r) {
        for (int c = 0; c < C; ++c)
            if (r % 7 != 3 && unif() < 0.35) {
                idx[nz] = c;
                val[nz++] = 2.0 * unif() - 1.0;
            }
        ptr[r + 1] = nz;
    }
    double *X = malloc(sizeof(double) * R * K), *W = malloc(sizeof(double) * C * K);
    orc_init_side(R, K, 7, 0x100, X);
    orc_init_side(C, K, 7, 0x101, W);
    double P[25] = {0}, m[5] = {0}, W0inv[25] = {0}, mu0[5] = {0};
    for (int k = 0; k < K; ++k) P[k * K + k] = W0inv[k * K + k] = 1.0;
    if (orc_update_side(R, K, ptr, idx, val, W, 0, P, m, 1.5, 7, 3, 0x102, X, 1) != 0) return 2;
    double Lam[25], mu[5];
    if (orc_nw_draw(R, K, X, mu0, 2.0, K, W0inv, 7, 3, 0x104, Lam, mu) != 0) return 3;
    const double sse = orc_sse(R, K, ptr, idx, val, X, W);
    (void)orc_tau_draw(sse, nz, 1.0, 1.0, 7, 3, 0x106);
    double z[9];
    orc_normals(7, 1, 2, 3, 9, z);
    (void)orc_gamma(7, 1, 2, 3, 0.4);
    (void)orc_gamma(7, 1, 2, 3, 3.0);
    float fv[5] = {1, 2, 3, 4, 5};
    (void)orc_seq_mean(5, fv);
    double L[25];
    (void)orc_cholesky(K, Lam, L);
    /* moment matching, clustering and the cluster fits on a chain that jumps */
    double *smp = malloc(sizeof(double) * S * R * K);
    for (int q = 0; q < S; ++q)
        for (int r = 0; r < R; ++r)
            for (int k = 0; k < K; ++k)
                smp[((int64_t)q * R + r) * K + k] = (q < S / 2 ? 0.0 : 4.0) + 0.3 * (2.0 * unif() - 1.0);
    double *mus = malloc(sizeof(double) * R * K), *Lams = malloc(sizeof(double) * R * K * K);
    (void)orc_mm(R, K, S, smp, mus, Lams);
    int32_t *lab = malloc(sizeof(int32_t) * R * S), *ncl = malloc(sizeof(int32_t) * R);
    int32_t *which = malloc(sizeof(int32_t) * R), *cnt = malloc(sizeof(int32_t) * R);
    double *ld = malloc(sizeof(double) * R);
    for (double sc = 0.5; sc < 5.0; sc *= 2.0) {
        (void)orc_lmeans(R, K, S, smp, sc, 16, 32, lab, ncl);
        for (int r = 0; r < R; ++r)
            which[r] = r % 3 == 0 ? -1 : lab[r * S];
        (void)orc_mm_sel(R, K, S, smp, lab, which, mus, Lams, ld, cnt);
    }
    (void)orc_lmeans(R, K, S, smp, 1e-9, 16, 32, lab, ncl);       /* the cluster cap binds */
    uint32_t ctr[8] = {1, 2, 3, 4, 5, 6, 7, 8}, out[8];
    orc_philox_batch(2, ctr, 99, out);
    printf("oracle driver done (%lld entries)\n", (long long)nz);
    free(ptr); free(idx); free(val); free(X); free(W); free(smp); free(mus); free(Lams);
    free(lab); free(ncl); free(which); free(cnt); free(ld);
    return 0;
}
