"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against a published value, a closed form, a
library routine or a statistical law, so that a dropped term, a wrong sign or a
transposed operand in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import native
from oracle.bpmf import Oracle, aggregate_side
from oracle.native import ptr
from oracle.plan import Plan, counter_c2, part_sizes

import synth

L = native.lib


# --------------------------------------------------------------------- Philox
def test_philox_known_answers(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = native.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_batch_matches_single():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(17, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x1234_5678_9ABC_DEF0
    out = native.philox_batch(ctr, seed)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for q in range(17):
        assert np.array_equal(out[q], native.philox4x32_10(ctr[q], key))


def test_u23_exact_and_open_interval():
    u = L()
    assert u.orc_u23(0) == 0.5 / 2**23
    assert u.orc_u23(0x1FF) == 0.5 / 2**23
    assert u.orc_u23(0xFFFFFFFF) == (2**23 - 0.5) / 2**23
    # exactly representable in FP32
    for x in (0, 255, 256, 0x80000000, 0xFFFFFFFF, 123456789):
        v = u.orc_u23(x)
        assert float(np.float32(v)) == v


# ------------------------------------------------------------------- Normals
def test_normals_ks_and_moments():
    z = np.concatenate([native.normals(7, c0, 3, 99, 64) for c0 in range(1000)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)


def test_normals_box_muller_layout():
    # z[4g], z[4g+1] come from (u0, u1); z[4g+2], z[4g+3] from (u2, u3).
    seed, c0, c1, c2 = 11, 5, 6, 7
    z = native.normals(seed, c0, c1, c2, 8)
    for g in range(2):
        o = native.philox4x32_10([c0, c1, c2, g], [seed, 0])
        u = [L().orc_u23(int(x)) for x in o]
        r1, r2 = np.sqrt(-2 * np.log(u[0])), np.sqrt(-2 * np.log(u[2]))
        assert z[4 * g] ** 2 + z[4 * g + 1] ** 2 == pytest.approx(r1 ** 2, rel=1e-13)
        assert z[4 * g + 2] ** 2 + z[4 * g + 3] ** 2 == pytest.approx(r2 ** 2, rel=1e-13)
        assert np.arctan2(z[4 * g + 1], z[4 * g]) % (2 * np.pi) == pytest.approx(
            2 * np.pi * u[1], rel=1e-12)


# --------------------------------------------------------------------- Gamma
@pytest.mark.parametrize("shape", [0.3, 1.0, 2.5, 17.0, 5000.5])
def test_gamma_ks(shape):
    g = np.array([native.gamma(3, c0, 1, 2, shape) for c0 in range(4000)])
    assert stats.kstest(g, "gamma", args=(shape,)).pvalue > 1e-3
    assert abs(g.mean() - shape) < 5 * np.sqrt(shape / g.size)


def test_chi2_from_gamma():
    nu = 7.0
    x = np.array([2.0 * native.gamma(9, c0, 4, 5, nu / 2) for c0 in range(4000)])
    assert stats.kstest(x, "chi2", args=(nu,)).pvalue > 1e-3


# ------------------------------------------------------------- Linear algebra
def test_cholesky_matches_numpy():
    rng = np.random.default_rng(1)
    for K in (1, 2, 5, 16, 33):
        B = rng.standard_normal((K, K + 3))
        A = B @ B.T + 0.1 * np.eye(K)
        np.testing.assert_allclose(native.cholesky(A), np.linalg.cholesky(A), rtol=1e-12,
                                   atol=1e-12)
    assert native.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]])) is None


# ------------------------------------------------ conditional update (rows)
def _one_row_update(K, w, r, P, m, tau, seed=5, t=3, c2=77, nrep=1):
    """nrep identical rows with the same observed set: draws differ only by z."""
    deg = w.shape[0]
    ptr_ = np.arange(nrep + 1, dtype=np.int64) * deg
    idx = np.tile(np.arange(deg, dtype=np.int32), nrep)
    val = np.tile(np.asarray(r, dtype=np.float64), nrep)
    out = np.zeros((nrep, K))
    f = L().orc_update_side(nrep, K, ptr(ptr_), ptr(idx), ptr(val),
                            ptr(np.ascontiguousarray(w, dtype=np.float64)), 0,
                            ptr(np.ascontiguousarray(P)), ptr(np.ascontiguousarray(m)),
                            tau, seed, t, c2, ptr(out), 1)
    assert f == 0
    return out


def test_update_k1_closed_form():
    rng = np.random.default_rng(2)
    w = rng.standard_normal((6, 1))
    r = rng.standard_normal(6)
    lam_p, m, tau = 1.7, 0.3, 2.2
    x = _one_row_update(1, w, r, np.array([[lam_p]]), np.array([m]), tau)[0, 0]
    Lam = lam_p + tau * np.sum(w[:, 0] ** 2)
    mu = (lam_p * m + tau * np.sum(r * w[:, 0])) / Lam
    z = native.normals(5, 0, 3, 77, 1)[0]
    assert x == pytest.approx(mu + z / np.sqrt(Lam), rel=1e-12, abs=1e-14)


def test_update_k2_closed_form():
    rng = np.random.default_rng(3)
    w = rng.standard_normal((9, 2))
    r = rng.standard_normal(9)
    P = np.array([[2.0, 0.4], [0.4, 1.5]])
    m = np.array([0.2, -0.7])
    tau = 1.3
    x = _one_row_update(2, w, r, P, m, tau)[0]
    # explicit 2x2 algebra
    a = P[0, 0] + tau * np.sum(w[:, 0] ** 2)
    b = P[0, 1] + tau * np.sum(w[:, 0] * w[:, 1])
    d = P[1, 1] + tau * np.sum(w[:, 1] ** 2)
    h0 = P[0, 0] * m[0] + P[0, 1] * m[1] + tau * np.sum(r * w[:, 0])
    h1 = P[1, 0] * m[0] + P[1, 1] * m[1] + tau * np.sum(r * w[:, 1])
    det = a * d - b * b
    mu = np.array([d * h0 - b * h1, a * h1 - b * h0]) / det
    # lower Cholesky factor of [[a, b], [b, d]] and x = mu + L^-T z
    l11 = np.sqrt(a)
    l21 = b / l11
    l22 = np.sqrt(d - l21 ** 2)
    z = native.normals(5, 0, 3, 77, 2)
    v1 = z[1] / l22
    v0 = (z[0] - l21 * v1) / l11
    np.testing.assert_allclose(x, mu + np.array([v0, v1]), rtol=1e-12, atol=1e-14)


def test_update_monte_carlo_moments():
    rng = np.random.default_rng(4)
    K, deg, n = 4, 12, 100_000
    w = rng.standard_normal((deg, K))
    r = rng.standard_normal(deg)
    B = rng.standard_normal((K, K))
    P = B @ B.T + np.eye(K)
    m = rng.standard_normal(K)
    tau = 0.8
    X = _one_row_update(K, w, r, P, m, tau, nrep=n)
    A = P + tau * w.T @ w
    Ainv = np.linalg.inv(A)
    mu = Ainv @ (P @ m + tau * w.T @ r)
    se = np.sqrt(np.diag(Ainv) / n)
    assert np.all(np.abs(X.mean(0) - mu) < 5 * se)
    C = np.cov(X.T)
    assert np.linalg.norm(C - Ainv) / np.linalg.norm(Ainv) < 0.02


def test_update_per_row_prior_equals_shared_when_identical():
    rng = np.random.default_rng(5)
    K, R, C = 3, 20, 7
    ptr_ = np.sort(rng.integers(0, 40, size=R + 1)).astype(np.int64)
    ptr_[0] = 0
    idx = rng.integers(0, C, size=ptr_[-1]).astype(np.int32)
    val = rng.standard_normal(ptr_[-1])
    W = rng.standard_normal((C, K))
    B = rng.standard_normal((K, K))
    P = B @ B.T + np.eye(K)
    m = rng.standard_normal(K)
    o1 = np.zeros((R, K))
    o2 = np.zeros((R, K))
    L().orc_update_side(R, K, ptr(ptr_), ptr(idx), ptr(val), ptr(W), 0, ptr(P), ptr(m), 1.1, 9, 2,
                        5, ptr(o1), 2)
    Pr = np.ascontiguousarray(np.broadcast_to(P, (R, K, K)))
    mr = np.ascontiguousarray(np.broadcast_to(m, (R, K)))
    L().orc_update_side(R, K, ptr(ptr_), ptr(idx), ptr(val), ptr(W), 1, ptr(Pr), ptr(mr), 1.1, 9,
                        2, 5, ptr(o2), 3)
    assert np.array_equal(o1, o2)


# ---------------------------------------------------------- Normal-Wishart
def test_nw_draw_moments_against_uncentred_footnote_formula():
    """E[Lambda] = nu* W*, Var[Lambda_ij] = nu* (W*_ij^2 + W*_ii W*_jj), E[mu] = mu*,
    with W*^-1 written in the footnote's third (uncentred) form."""
    rng = np.random.default_rng(6)
    K, Nb = 3, 40
    X = rng.standard_normal((Nb, K)) * 0.7 + 0.4
    mu0 = np.array([0.1, -0.2, 0.3])
    beta0, nu0 = 2.0, 5.0
    W0 = np.array([[1.0, 0.2, 0.0], [0.2, 2.0, 0.1], [0.0, 0.1, 0.5]])
    W0inv = np.linalg.inv(W0)
    ndraw = 20000
    Lams = np.zeros((ndraw, K, K))
    mus = np.zeros((ndraw, K))
    Lm = np.zeros((K, K))
    mm = np.zeros(K)
    for t in range(ndraw):
        rc = L().orc_nw_draw(Nb, K, ptr(X), ptr(mu0), beta0, nu0, ptr(W0inv), 21, t, 1028,
                             ptr(Lm), ptr(mm))
        assert rc == 0
        Lams[t] = Lm
        mus[t] = mm
    xbar = X.mean(0)
    Sunc = X.T @ X / Nb
    bs = beta0 + Nb
    mus_ = (beta0 * mu0 + Nb * xbar) / bs
    Winv = W0inv + Nb * Sunc + beta0 * np.outer(mu0, mu0) - bs * np.outer(mus_, mus_)
    Ws = np.linalg.inv(Winv)
    nus = nu0 + Nb
    mean = nus * Ws
    var = nus * (Ws ** 2 + np.outer(np.diag(Ws), np.diag(Ws)))
    se = np.sqrt(var / ndraw)
    assert np.all(np.abs(Lams.mean(0) - mean) < 5 * se)
    assert np.allclose(Lams.var(0), var, rtol=0.1)
    # mu | Lambda ~ N(mu*, (beta* Lambda)^-1): E[mu] = mu*, Cov = E[Lambda^-1] / beta*
    #   with E[Lambda^-1] = W*^-1 / (nu* - K - 1)
    cov_mu = Winv / (nus - K - 1) / bs
    assert np.all(np.abs(mus.mean(0) - mus_) < 5 * np.sqrt(np.diag(cov_mu) / ndraw))
    assert np.allclose(np.cov(mus.T), cov_mu, rtol=0.08, atol=1e-5)


def test_nw_three_footnote_forms_agree_numerically():
    """The oracle's centred form and the two alternatives of the footnote give the
    same W*^-1 (checked through the same Bartlett draw, which depends on W*^-1 only)."""
    rng = np.random.default_rng(7)
    K, Nb = 4, 25
    X = rng.standard_normal((Nb, K)) + 1.5
    mu0 = rng.standard_normal(K)
    W0inv = np.eye(K) * 0.7
    beta0, nu0 = 2.0, K
    Lm = np.zeros((K, K))
    mm = np.zeros(K)
    assert L().orc_nw_draw(Nb, K, ptr(X), ptr(mu0), beta0, nu0, ptr(W0inv), 1, 0, 4, ptr(Lm),
                           ptr(mm)) == 0
    # Re-derive the same draw from the second footnote form: Bartlett factors are a
    # deterministic function of the counters, so Lambda = T A A^T T^T must match.
    xbar = X.mean(0)
    Sunc = X.T @ X / Nb
    bs = beta0 + Nb
    Winv2 = W0inv + Nb * Sunc + beta0 * Nb / bs * np.outer(mu0 - xbar, mu0 - xbar) \
        - Nb * np.outer(xbar, xbar)
    R = np.linalg.cholesky(Winv2)
    T = np.linalg.inv(R).T
    A = np.zeros((K, K))
    nus = nu0 + Nb
    for k in range(1, K + 1):
        A[k - 1, k - 1] = np.sqrt(2.0 * native.gamma(1, k, 0, 4, 0.5 * (nus - k + 1)))
    zoff = native.normals(1, 0, 0, 4, K * (K - 1) // 2)
    q = 0
    for a in range(1, K):
        for b in range(a):
            A[a, b] = zoff[q]
            q += 1
    Lam2 = T @ A @ A.T @ T.T
    np.testing.assert_allclose(Lm, Lam2, rtol=1e-9)


# ---------------------------------------------------------------------- tau
def test_tau_draw_gamma_mean():
    sse, M, a0, b0 = 37.5, 120, 1.0, 1.0
    d = np.array([L().orc_tau_draw(sse, M, a0, b0, 5, t, 6) for t in range(20000)])
    shape, rate = a0 + M / 2, b0 + sse / 2
    assert abs(d.mean() - shape / rate) < 5 * np.sqrt(shape) / rate / np.sqrt(d.size)
    assert stats.kstest(d * rate, "gamma", args=(shape,)).pvalue > 1e-3


def test_sse_matches_dense_algebra():
    rng = np.random.default_rng(8)
    R, C, K = 30, 12, 3
    Y = rng.standard_normal((R, C))
    mask = rng.random((R, C)) < 0.4
    X = rng.standard_normal((R, K))
    W = rng.standard_normal((C, K))
    rows, cols = np.nonzero(mask)
    ptr_ = np.zeros(R + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=R), out=ptr_[1:])
    s = L().orc_sse(R, K, ptr(ptr_), ptr(cols.astype(np.int32)), ptr(Y[mask].copy()), ptr(X),
                    ptr(W))
    assert s == pytest.approx(np.sum(((Y - X @ W.T) ** 2)[mask]), rel=1e-12)


# ------------------------------------------------------------ moment matching
def test_mm_matches_numpy_cov_and_ridge():
    rng = np.random.default_rng(9)
    S, R, K = 30, 5, 4
    smp = rng.standard_normal((S, R, K)) * np.array([1.0, 2.0, 0.5, 1.5]) + 3.0
    mu = np.zeros((R, K))
    Lam = np.zeros((R, K, K))
    assert L().orc_mm(R, K, S, ptr(smp), ptr(mu), ptr(Lam)) == 0
    for n in range(R):
        np.testing.assert_allclose(mu[n], smp[:, n].mean(0), rtol=1e-13)
        np.testing.assert_allclose(Lam[n], np.linalg.inv(np.cov(smp[:, n].T)), rtol=1e-10)
    # S <= K: ridge with delta = 1e-6 tr / K
    S2 = 3
    smp2 = np.ascontiguousarray(smp[:S2])
    assert L().orc_mm(R, K, S2, ptr(smp2), ptr(mu), ptr(Lam)) == R
    for n in range(R):
        C = np.cov(smp2[:, n].T)
        C = C + (1e-6 * np.trace(C) / K + 1e-300) * np.eye(K)
        np.testing.assert_allclose(Lam[n], np.linalg.inv(C), rtol=1e-6)


# --------------------------------------------------------------- partition
def test_partition_sizes_pinned_by_paper(golden_dir):
    for l in open(os.path.join(golden_dir, "partition_ml1m_5x5.txt")):
        if l.startswith("#") or not l.strip():
            continue
        N, D, r, c, rp, cp = map(int, l.split())
        bs, sizes = part_sizes(N, r)
        assert bs == rp and sizes[0] == rp and sum(sizes) == N
        bs, sizes = part_sizes(D, c)
        assert bs == cp and sizes[0] == cp and sum(sizes) == D
    with pytest.raises(ValueError):
        part_sizes(10, 6)          # ceil(10/6)=2 leaves the 6th part empty


@pytest.mark.parametrize("order", ["given", "random", "decreasing"])
def test_plan_brute_force(order):
    rng = np.random.default_rng(10)
    N, D, I, J = 23, 17, 3, 2
    cells = rng.choice(N * D, size=120, replace=False)
    row, col = cells // D, cells % D
    p = Plan(N, D, row, col, I, J, order, seed=44)
    # positions are permutations
    assert sorted(p.row_pos.tolist()) == list(range(N))
    assert sorted(p.col_pos.tolist()) == list(range(D))
    if order == "decreasing":
        cnt = np.bincount(row, minlength=N)
        by_pos = cnt[np.argsort(p.row_pos)]
        assert np.all(np.diff(by_pos) <= 0)
    if order == "given":
        assert np.array_equal(p.row_pos, np.arange(N))
    # brute force: every entry in exactly one block, CSR and CSC transposes
    tot = 0
    for blk in p.blocks:
        i, j = blk["i"], blk["j"]
        dense = np.zeros((blk["R"], blk["C"]), dtype=int)
        for e in range(row.size):
            if p.row_block[row[e]] == i and p.col_block[col[e]] == j:
                dense[p.row_local[row[e]], p.col_local[col[e]]] += 1
        assert dense.max(initial=0) <= 1
        csr = np.zeros_like(dense)
        for n in range(blk["R"]):
            cols_n = blk["csr_idx"][blk["csr_ptr"][n]:blk["csr_ptr"][n + 1]]
            assert np.all(np.diff(cols_n) > 0)
            csr[n, cols_n] = 1
        csc = np.zeros_like(dense)
        for d in range(blk["C"]):
            rows_d = blk["csc_idx"][blk["csc_ptr"][d]:blk["csc_ptr"][d + 1]]
            assert np.all(np.diff(rows_d) > 0)
            csc[rows_d, d] = 1
        assert np.array_equal(dense, csr) and np.array_equal(dense, csc)
        tot += blk["M"]
    assert tot == row.size


def test_random_order_uses_philox_keys():
    N = 50
    p = Plan(N, 3, np.arange(N) % N, np.zeros(N, dtype=int), 1, 1, "random", seed=99)
    keys = [int(native.philox4x32_10([n, 0, counter_c2(0xFFFFFF, "PERM_ROW"), 0],
                                     [99, 0])[0]) for n in range(N)]
    expected = sorted(range(N), key=lambda n: (keys[n], n))
    assert [int(x) for x in np.argsort(p.row_pos)] == expected


# ----------------------------------------------------------------- aggregation
def _spd(rng, K, scale=1.0):
    B = rng.standard_normal((K, K))
    return scale * (B @ B.T + K * np.eye(K))


def test_aggregation_linear_gaussian_exactness():
    """Theorem 1 with X fixed and Gaussian W: base precision Lambda_W + tau G_0 and
    sibling precisions Lambda_base + tau G_i aggregate to the full-data posterior."""
    rng = np.random.default_rng(11)
    K, R, I, tau = 3, 6, 4, 1.7
    LamW = _spd(rng, K)
    m = rng.standard_normal(K)
    G = [[_spd(rng, K, 0.3) for _ in range(R)] for _ in range(I)]
    h = [[rng.standard_normal(K) for _ in range(R)] for _ in range(I)]
    Lb = np.array([LamW + tau * G[0][n] for n in range(R)])
    eb = [LamW @ m + tau * h[0][n] for n in range(R)]
    mub = np.array([np.linalg.solve(Lb[n], eb[n]) for n in range(R)])
    Ls, mus = [], []
    for i in range(1, I):
        Li = np.array([Lb[n] + tau * G[i][n] for n in range(R)])
        mi = np.array([np.linalg.solve(Li[n], Lb[n] @ mub[n] + tau * h[i][n]) for n in range(R)])
        Ls.append(Li)
        mus.append(mi)
    mu_star, ncor = aggregate_side(mub, Lb, mus, Ls, K)
    assert ncor == 0
    for n in range(R):
        Lfull = LamW + tau * sum(G[i][n] for i in range(I))
        mfull = np.linalg.solve(Lfull, LamW @ m + tau * sum(h[i][n] for i in range(I)))
        np.testing.assert_allclose(mu_star[n], mfull, rtol=1e-10, atol=1e-12)


def test_aggregation_eigen_correction_gives_spd():
    rng = np.random.default_rng(12)
    K, R = 4, 5
    Lb = np.array([_spd(rng, K, 2.0) for _ in range(R)])
    mub = rng.standard_normal((R, K))
    # siblings less precise than the base: differences are not PD
    Ls = [np.array([0.5 * Lb[n] for n in range(R)]) for _ in range(3)]
    mus = [rng.standard_normal((R, K)) for _ in range(3)]
    mu, ncor = aggregate_side(mub, Lb, mus, Ls, K)
    assert ncor == 3 * R
    for n in range(R):
        eps = 1e-6 * np.trace(Lb[n]) / K
        Lstar = -2 * Lb[n]
        rhs = -2 * Lb[n] @ mub[n]
        for Lj, mj in zip(Ls, mus):
            Dj = Lj[n] - Lb[n]
            Lsj = Dj + (abs(np.linalg.eigvalsh(Dj)[0]) + eps) * np.eye(K) + Lb[n]
            Lstar += Lsj
            rhs += Lsj @ mj[n]
        assert np.linalg.eigvalsh(Lstar)[0] > 0
        np.testing.assert_allclose(mu[n], np.linalg.solve(Lstar, rhs), rtol=1e-10)


def test_aggregation_two_forms_equal_without_correction():
    """Algorithm 2's (2 - J) form equals eq. post_marg_aggregation when no
    correction fires."""
    rng = np.random.default_rng(13)
    K, R, J = 3, 4, 5
    Lb = np.array([_spd(rng, K) for _ in range(R)])
    mub = rng.standard_normal((R, K))
    Ls = [np.array([Lb[n] + _spd(rng, K, 0.2) for n in range(R)]) for _ in range(J - 1)]
    mus = [rng.standard_normal((R, K)) for _ in range(J - 1)]
    mu, ncor = aggregate_side(mub, Lb, mus, Ls, K)
    assert ncor == 0
    for n in range(R):
        Lstar = Lb[n] + sum(Ls[j][n] - Lb[n] for j in range(J - 1))
        rhs = Lb[n] @ mub[n] + sum(Ls[j][n] @ mus[j][n] - Lb[n] @ mub[n] for j in range(J - 1))
        np.testing.assert_allclose(mu[n], np.linalg.solve(Lstar, rhs), rtol=1e-10)


# ------------------------------------------------------- chain-level checks
def test_chain_config1_rmse_between_noise_floor_and_column_means():
    d = synth.config(1, seed=1)
    o = Oracle(d["N"], d["D"], d["K"], d["row"], d["col"], d["val"], seed=101, burnin=20)
    o.run_stage(1, 50)
    o.aggregate()
    p = o.predict(d["test_row"], d["test_col"])
    rmse = np.sqrt(np.mean((p - d["test_val"]) ** 2))
    cnt = np.maximum(np.bincount(d["col"], minlength=d["D"]), 1)
    cm = np.bincount(d["col"], weights=d["val"], minlength=d["D"]) / cnt
    rmse_cm = np.sqrt(np.mean((cm[d["test_col"]] - d["test_val"]) ** 2))
    assert 0.5 < rmse < 0.6 * rmse_cm
    # tau should approach the true noise precision 1/0.5^2 = 4
    assert 2.5 < o.blocks[0]["tau"] < 6.0


def test_pp_linear_gaussian_monte_carlo():
    """PP with X frozen at the truth, fixed hyperparameters and tau, partition
    I x 1: the moment-matched and aggregated W means approach the exact
    full-data conditional means (Theorem 1) within Monte Carlo error."""
    rng = np.random.default_rng(14)
    N, D, K, I = 60, 8, 2, 3
    X = rng.standard_normal((N, K))
    Wt = rng.standard_normal((D, K))
    mask = rng.random((N, D)) < 0.5
    row, col = np.nonzero(mask)
    val = (np.sum(X[row] * Wt[col], 1) + 0.5 * rng.standard_normal(row.size)).astype(np.float32)
    o = Oracle(N, D, K, row, col, val, I=I, J=1, sample_tau=False, tau_fixed=4.0, seed=3,
               burnin=0, thin=1)
    nsw = 3000
    for s in (1, 2):
        o.begin_stage(s)
        for blk in o.stage_blocks(s):
            blk["X"] = np.ascontiguousarray(X[o.plan.row_ids[blk["i"]]])
            for t in range(nsw):
                o.update_cols(blk, t)
                blk["samples_w"].append(blk["W"].copy())
                blk["samples_x"].append(blk["X"].copy())
        o.finalize_stage()
    o.aggregate()
    r = val.astype(np.float64) - o.ybar
    for d in range(D):
        sel = col == d
        A = np.eye(K) + 4.0 * X[row[sel]].T @ X[row[sel]]
        mu = np.linalg.solve(A, 4.0 * X[row[sel]].T @ r[sel])
        got = o.mu_w[0][o.plan.col_local[d]]
        sd = np.sqrt(np.diag(np.linalg.inv(A)))
        assert np.all(np.abs(got - mu) < 6 * sd / np.sqrt(nsw) + 0.05 * sd)


def test_pp_linear_gaussian_monte_carlo_row_side():
    """The mirror of the I x 1 case: W frozen at the truth, partition 1 x J,
    X sampled; the X rows of blocks (0, j), j >= 1, run under the
    moment-matched prior of block (0, 0) (eq. stage2b), and the aggregated
    X means approach the full-data conditional means (Theorem 1)."""
    rng = np.random.default_rng(15)
    N, D, K, J = 8, 66, 2, 3
    Xt = rng.standard_normal((N, K))
    W = rng.standard_normal((D, K))
    mask = rng.random((N, D)) < 0.5
    row, col = np.nonzero(mask)
    val = (np.sum(Xt[row] * W[col], 1) + 0.5 * rng.standard_normal(row.size)).astype(np.float32)
    o = Oracle(N, D, K, row, col, val, I=1, J=J, sample_tau=False, tau_fixed=4.0, seed=4,
               burnin=0, thin=1)
    nsw = 3000
    for s in (1, 2):
        o.begin_stage(s)
        for blk in o.stage_blocks(s):
            assert blk["x_prop"] == (blk["j"] > 0) and not blk["w_prop"]
            blk["W"] = np.ascontiguousarray(W[o.plan.col_ids[blk["j"]]])
            for t in range(nsw):
                o.update_rows(blk, t)
                blk["samples_x"].append(blk["X"].copy())
                blk["samples_w"].append(blk["W"].copy())
        o.finalize_stage()
    o.aggregate()
    r = val.astype(np.float64) - o.ybar
    for n in range(N):
        sel = row == n
        A = np.eye(K) + 4.0 * W[col[sel]].T @ W[col[sel]]
        mu = np.linalg.solve(A, 4.0 * W[col[sel]].T @ r[sel])
        got = o.mu_x[0][o.plan.row_local[n]]
        sd = np.sqrt(np.diag(np.linalg.inv(A)))
        assert np.all(np.abs(got - mu) < 6 * sd / np.sqrt(nsw) + 0.05 * sd)


# ------------------------------------------ exact linear-Gaussian propagation
def _exact_side(ptr_, idx, r, other, prior, tau, K):
    """Exact Gaussian posterior (precision, mean) of every entity of one side of
    a block given the other side frozen: Lambda = P + tau G, mean solves
    Lambda mu = P m + tau s (the conjugate update of Sec. 2.1, in numpy)."""
    n = ptr_.size - 1
    P, m = prior
    lam = np.zeros((n, K, K))
    mu = np.zeros((n, K))
    for e in range(n):
        Pn = P[e] if P.ndim == 3 else P
        mn = m[e] if m.ndim == 2 else m
        w = other[idx[ptr_[e]:ptr_[e + 1]]]
        lam[e] = Pn + tau * w.T @ w
        mu[e] = np.linalg.solve(lam[e], Pn @ mn + tau * w.T @ r[ptr_[e]:ptr_[e + 1]])
    return lam, mu


def _exact_pp(oracle_mod, seed=16):
    """Run the three stages of a 3 x 3 partition with exact Gaussian stage
    posteriors in place of moment-matched samples: the X side of every block
    given the true W, the W side given the true X, each under the prior the
    oracle's begin_stage binds (eq. stage1-stage3).  Returns the oracle after
    aggregation, the truth and the data."""
    rng = np.random.default_rng(seed)
    N, D, K, I, J, tau = 43, 31, 2, 3, 3, 2.5
    X = rng.standard_normal((N, K))
    W = rng.standard_normal((D, K))
    mask = rng.random((N, D)) < 0.85
    row, col = np.nonzero(mask)
    val = (np.sum(X[row] * W[col], 1) + rng.standard_normal(row.size)).astype(np.float32)
    o = oracle_mod.Oracle(N, D, K, row, col, val, I=I, J=J, order="random", sample_tau=False,
                          tau_fixed=tau, seed=seed)
    for s in (1, 2, 3):
        o.begin_stage(s)
        for blk in o.stage_blocks(s):
            Xb = X[o.plan.row_ids[blk["i"]]]
            Wb = W[o.plan.col_ids[blk["j"]]]
            px = blk["x_prior"] if blk["x_prior"] is not None else blk["hx"]
            pw = blk["w_prior"] if blk["w_prior"] is not None else blk["hw"]
            xl, xm = _exact_side(blk["csr_ptr"], blk["csr_idx"], blk["csr_val"], Wb, px, tau, K)
            wl, wm = _exact_side(blk["csc_ptr"], blk["csc_idx"], blk["csc_val"], Xb, pw, tau, K)
            o.mm[blk["b"]] = dict(x_mu=xm, x_Lam=xl, w_mu=wm, w_Lam=wl, ridged=0)
    o.aggregate()
    return o, X, W, row, col, val, tau


def _exact_pp_check(o, X, W, row, col, val, tau):
    """Theorem 1: the aggregated precision and mean of every row and column
    equal the full-data conditional ones (prior (I, 0), all observed entries)."""
    K = X.shape[1]
    r = val.astype(np.float64) - o.ybar
    assert o.corrections == 0
    for n in range(o.N):
        sel = row == n
        lam = np.eye(K) + tau * W[col[sel]].T @ W[col[sel]]
        mu = np.linalg.solve(lam, tau * W[col[sel]].T @ r[sel])
        i, loc = o.plan.row_block[n], o.plan.row_local[n]
        np.testing.assert_allclose(o.lam_x[i][loc], lam, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(o.mu_x[i][loc], mu, rtol=1e-10, atol=1e-10)
    for d in range(o.D):
        sel = col == d
        lam = np.eye(K) + tau * X[row[sel]].T @ X[row[sel]]
        mu = np.linalg.solve(lam, tau * X[row[sel]].T @ r[sel])
        j, loc = o.plan.col_block[d], o.plan.col_local[d]
        np.testing.assert_allclose(o.lam_w[j][loc], lam, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(o.mu_w[j][loc], mu, rtol=1e-10, atol=1e-10)


def test_pp_exact_gaussian_stages_aggregate_to_full_posterior():
    """Both prior bindings of begin_stage (X of (i, j) from (i, 0), W from
    (0, j)) and both loops of Algorithm 2 reproduce the full-data conditional
    exactly when every stage posterior is the exact Gaussian (Theorem 1)."""
    from oracle import bpmf
    _exact_pp_check(*_exact_pp(bpmf))


def _mutant(old, new):
    """The oracle's bpmf module with one planted mistake (CPU only)."""
    import types
    from oracle import bpmf
    src = open(bpmf.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle._mutant")
    mod.__package__ = "oracle"
    mod.__file__ = bpmf.__file__
    exec(compile(src.replace(old, new), bpmf.__file__ + " (mutant)", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("old,new", [
    ("src = self.mm[i * self.J + 0]", "src = self.mm[0 * self.J + i]"),          # X binding
    ("src = self.mm[0 * self.J + j]", "src = self.mm[j * self.J + 0]"),          # W binding
    ("base = self.mm[i * J + 0]", "base = self.mm[0 * J + i]"),                  # X base
    ("sib = [self.mm[i * J + j] for j in range(1, J)]",
     "sib = [self.mm[j * J + i] for j in range(1, J)]"),                         # X siblings
    ("base = self.mm[0 * J + j]", "base = self.mm[j * J + 0]"),                  # W base
    ("sib = [self.mm[i * J + j] for i in range(1, I)]",
     "sib = [self.mm[j * J + i] for i in range(1, I)]"),                         # W siblings
    ("Lstar = (2 - Jn) * Lb", "Lstar = (1 - Jn) * Lb"),                          # (2 - J) term
])
def test_exact_pin_fails_on_planted_index_mistakes(old, new):
    with pytest.raises((AssertionError, KeyError, IndexError, ValueError, np.linalg.LinAlgError)):
        _exact_pp_check(*_exact_pp(_mutant(old, new)))


# ------------------------------------------------------------- P4, P5, P6
def test_conditional_precisions_are_spd_above_prior():
    """Every conditional precision the update forms passes Cholesky, and its
    smallest eigenvalue is at least the prior's (P + tau G with G PSD)."""
    rng = np.random.default_rng(17)
    K, R, C = 5, 40, 30
    deg = rng.integers(0, 9, size=R)
    ptr_ = np.zeros(R + 1, dtype=np.int64)
    np.cumsum(deg, out=ptr_[1:])
    idx = np.concatenate([np.sort(rng.choice(C, size=k, replace=False)) for k in deg]).astype(np.int32)
    val = rng.standard_normal(ptr_[-1])
    W = rng.standard_normal((C, K)) * rng.uniform(0.01, 3.0, size=(C, 1))
    P = np.zeros((R, K, K))
    for n in range(R):
        Q, _ = np.linalg.qr(rng.standard_normal((K, K)))
        P[n] = Q @ np.diag(10.0 ** rng.uniform(-6, 2, size=K)) @ Q.T
        P[n] = 0.5 * (P[n] + P[n].T)
    m = rng.standard_normal((R, K))
    tau = 0.7
    A = np.zeros((R, K, K))
    L().orc_cond_precision(R, K, ptr(ptr_), ptr(idx), ptr(val), ptr(W), 1, ptr(P), ptr(m), tau,
                           ptr(A))
    for n in range(R):
        w = W[idx[ptr_[n]:ptr_[n + 1]]]
        np.testing.assert_allclose(A[n], P[n] + tau * np.einsum("ea,eb->ab", w, w), rtol=1e-12,
                                   atol=1e-12 * np.abs(A[n]).max())
        assert native.cholesky(A[n]) is not None
        lo = np.linalg.eigvalsh(A[n])[0]
        assert lo > 0 and lo >= np.linalg.eigvalsh(P[n])[0] * (1 - 1e-9)
        if deg[n] == 0:
            assert np.array_equal(A[n], P[n])


def test_prediction_invariant_under_sign_flip():
    """Negating latent coordinate k of every X and W posterior (means, and the
    precisions conjugated by the sign matrix) leaves the predictions unchanged
    (the sign ambiguity of Sec. 2.1); negating X alone does not."""
    d = synth.make("ratings", 120, 70, 3, 3000, 0.8, 2)
    o = Oracle(d["N"], d["D"], 3, d["row"], d["col"], d["val"], I=2, J=2, order="random", seed=5,
               burnin=6)
    o.run_pp(20)
    o.aggregate()
    p1 = o.predict(d["test_row"], d["test_col"])
    k = 1
    S = np.ones(3)
    S[k] = -1.0
    saved = {b: {key: v.copy() if isinstance(v, np.ndarray) else v for key, v in mm.items()}
             for b, mm in o.mm.items()}
    for mm in o.mm.values():
        for side in ("x", "w"):
            mm[side + "_mu"] = mm[side + "_mu"] * S
            mm[side + "_Lam"] = mm[side + "_Lam"] * S[:, None] * S[None, :]
    o.aggregate()
    p2 = o.predict(d["test_row"], d["test_col"])
    np.testing.assert_allclose(p2, p1, rtol=1e-12, atol=1e-12)
    o.mm = saved
    for mm in o.mm.values():
        mm["x_mu"] = mm["x_mu"] * S
        mm["x_Lam"] = mm["x_Lam"] * S[:, None] * S[None, :]
    o.aggregate()
    p3 = o.predict(d["test_row"], d["test_col"])
    assert np.abs(p3 - p1).max() > 1e-3


def test_one_block_pp_is_plain_bpmf():
    """With a 1 x 1 partition, PP's stage 1 is plain BPMF (Theorem 1): the
    chain run as a PP stage equals the plain sweep loop, and the aggregated
    posterior mean is the kept-sample mean with its precision the inverse
    sample covariance."""
    d = synth.make("ratings", 150, 80, 4, 3000, 0.8, 3)
    a = Oracle(d["N"], d["D"], 4, d["row"], d["col"], d["val"], seed=9, burnin=5)
    a.run_pp(25)
    a.aggregate()
    b = Oracle(d["N"], d["D"], 4, d["row"], d["col"], d["val"], seed=9, burnin=5)
    b.begin_stage(1)
    for _ in range(25):
        b.sweep_block(b.blocks[0])
    assert np.array_equal(a.blocks[0]["X"], b.blocks[0]["X"])
    assert np.array_equal(a.blocks[0]["W"], b.blocks[0]["W"])
    sx = np.stack(b.blocks[0]["samples_x"])
    assert sx.shape[0] == 20
    np.testing.assert_allclose(a.mu_x[0], sx.mean(0), rtol=1e-13, atol=1e-14)
    for n in (0, 7, 31):
        np.testing.assert_allclose(a.lam_x[0][n], np.linalg.inv(np.cov(sx[:, n].T)), rtol=1e-9)
    p = a.predict(d["test_row"], d["test_col"])
    sw = np.stack(b.blocks[0]["samples_w"])
    q = a.ybar + np.einsum("ek,ek->e", sx.mean(0)[a.plan.row_local[d["test_row"]]],
                           sw.mean(0)[a.plan.col_local[d["test_col"]]])
    np.testing.assert_allclose(p, q, rtol=1e-12)


# ------------------------------------------------- the paper's simulated data
def _table4(golden_dir):
    out = {}
    for l in open(os.path.join(golden_dir, "table4_simulated_rmse.txt")):
        if l.startswith("#") or not l.strip():
            continue
        p, dec, rnd = l.split()
        out[int(p)] = {"decreasing": float(dec), "random": float(rnd)}
    return out


@pytest.mark.parametrize("IJ", [1, 3])
def test_simulated_data_rmse_in_table4_band(golden_dir, IJ):
    """The paper's simulated workload (Sec. 5.3: K = 5, tau = 1 fixed, 80 %
    missing at random) through the oracle's PP chain: the test RMSE of the
    posterior-mean prediction lies within 0.01 of the published value (Table 4)
    for the 1 x 1 and 3 x 3 partitions.  A shortened schedule (300 sweeps, 200
    burn-in, every second kept) keeps this CPU test short; the posterior of
    this data concentrates within far fewer sweeps."""
    want = _table4(golden_dir)[IJ]["random"]
    d = synth.simulated(1, "mar")
    o = Oracle(d["N"], d["D"], 5, d["row"], d["col"], d["val"], I=IJ, J=IJ, order="random",
               sample_tau=False, tau_fixed=1.0, seed=101, burnin=200, thin=2)
    o.run_pp(300)
    o.aggregate()
    p = o.predict(d["test_row"], d["test_col"])
    rmse = float(np.sqrt(np.mean((p - d["test_val"]) ** 2)))
    print("partition %dx%d: rmse %.5f (paper %.3f)" % (IJ, IJ, rmse, want))
    assert abs(rmse - want) <= 0.01
    # the noise floor: no predictor beats the noise standard deviation by much
    assert rmse > 0.99


def test_structured_missingness_recipe():
    """The second simulated scenario of Sec. 5.3: row and column weights equally
    spaced from 0.9 down to 0.005, cell (n, d) observed with probability
    w_n w_d.  The paper states that this leaves about 80 % of the cells
    missing, which fixes the reading of the product as the probability of
    being observed (as the probability of being missing it would leave about
    20 %).  Checked: the missing fraction, its closed-form expectation
    1 - mean(w)^2, and the density falling with the row and column index as
    the weights do."""
    d = synth.simulated(3, "structured")
    N, D = d["N"], d["D"]
    frac_missing = d["test_row"].size / (N * D)
    mean_w = np.linspace(0.9, 0.005, N).mean() * np.linspace(0.9, 0.005, D).mean()
    print("structured: %.4f missing, expected %.4f" % (frac_missing, 1.0 - mean_w))
    assert abs(frac_missing - 0.8) <= 0.01
    assert abs(frac_missing - (1.0 - mean_w)) <= 1e-3
    assert d["row"].size + d["test_row"].size == N * D
    # observed density per row decile and per column decile decreases
    rows = np.bincount(d["row"], minlength=N).astype(float)
    cols = np.bincount(d["col"], minlength=D).astype(float)
    rdec = np.array([c.mean() for c in np.array_split(rows, 10)])
    cdec = np.array([c.mean() for c in np.array_split(cols, 10)])
    assert np.all(np.diff(rdec) < 0) and np.all(np.diff(cdec) < 0)
    # first row's expected count: w_1 sum_d w_d
    assert abs(rows[0] / (0.9 * np.linspace(0.9, 0.005, D).sum()) - 1.0) <= 0.05
