"""Pins of the oracle's dominant-mode and mixture approximations (CPU only).

The clustering of the kept samples (lambda-means), the dominant-mode fit, the
pooled mixture moments used for aggregation (Sec. 4.2, eq. marginal_mixture)
and the responsibility choice of a mixture prior (Sec. 5.1) are checked
against facts fixed outside the oracle: clusters planted far apart, the
fixed-point property of a converged DP-means assignment, the plain sample
moments of the planted clusters (numpy), the law of total variance, and
closed-form responsibilities.
"""
import numpy as np

from oracle import native
from oracle.bpmf import LMEANS_CMAX, LMEANS_MAXIT, Oracle, gmm_choice
from oracle.native import ptr

import synth

L = native.lib


def _lmeans(smp, scale=2.0, cmax=LMEANS_CMAX, maxit=LMEANS_MAXIT):
    """smp: (S, R, K) -> labels (R, S), cluster counts (R,)."""
    S, R, K = smp.shape
    smp = np.ascontiguousarray(smp, dtype=np.float64)
    lab = np.zeros((R, S), dtype=np.int32)
    ncl = np.zeros(R, dtype=np.int32)
    L().orc_lmeans(R, K, S, ptr(smp), scale, cmax, maxit, ptr(lab), ptr(ncl))
    return lab, ncl


def _lam2(x, scale):
    d = np.diff(x, axis=0)
    return scale * scale * (d * d).sum() / (2.0 * (x.shape[0] - 1))


def _chain_of_blobs(rng, centres, sizes, sd, K):
    """A chain that stays at each planted centre for its run of samples."""
    xs, truth = [], []
    for c, (m, n) in enumerate(zip(centres, sizes)):
        xs.append(m + sd * rng.standard_normal((n, K)))
        truth += [c] * n
    return np.concatenate(xs), np.array(truth)


def test_lmeans_recovers_planted_runs():
    rng = np.random.default_rng(3)
    K = 5
    for sizes in ((120, 80), (50, 100, 50), (200,)):
        centres = [rng.standard_normal(K) * 6.0 for _ in sizes]
        x, truth = _chain_of_blobs(rng, centres, sizes, 0.1, K)
        lab, ncl = _lmeans(x[:, None, :])
        assert ncl[0] == len(set(truth.tolist())) or ncl[0] == len(sizes)
        # the same partition as the planted one (ids in order of first appearance)
        first = {}
        want = np.array([first.setdefault(t, len(first)) for t in truth])
        np.testing.assert_array_equal(lab[0], want)


def test_lmeans_fixed_point_property():
    """At convergence each sample's label is its nearest final centre (lowest
    index on ties), within lambda unless the cluster cap was reached, and each
    centre is the mean of its members."""
    rng = np.random.default_rng(11)
    S, R, K = 60, 40, 3
    # a random walk with occasional jumps: clusters of varied shapes
    steps = 0.3 * rng.standard_normal((S, R, K))
    steps[rng.random((S, R)) < 0.05] *= 12.0
    smp = np.cumsum(steps, axis=0)
    for scale in (1.0, 2.0, 4.0):
        lab, ncl = _lmeans(smp, scale)
        for n in range(R):
            x = smp[:, n, :]
            C = ncl[n]
            cent = np.array([x[lab[n] == c].mean(0) for c in range(C)])
            assert all((lab[n] == c).any() for c in range(C))
            d = ((x[:, None, :] - cent[None, :, :]) ** 2).sum(-1)
            np.testing.assert_array_equal(lab[n], np.argmin(d, axis=1))
            if C < LMEANS_CMAX:
                assert (d.min(1) <= _lam2(x, scale) * (1 + 1e-12)).all()


def test_lmeans_degenerate_cases():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((30, 1, 4))
    lab, ncl = _lmeans(x, scale=1e6)                   # lambda beyond every distance
    assert ncl[0] == 1 and (lab == 0).all()
    same = np.repeat(x[:1], 30, axis=0)                # every sample identical: lambda = 0
    lab, ncl = _lmeans(same)
    assert ncl[0] == 1 and (lab == 0).all()
    lab, ncl = _lmeans(x, scale=1e-9)                  # tiny lambda: the cap binds
    assert ncl[0] == LMEANS_CMAX
    assert lab.max() == LMEANS_CMAX - 1


def _oracle_for_fit(approx, K):
    d = synth.make("ratings", 20, 10, K, 100, 0.8, 1)
    return Oracle(d["N"], d["D"], K, d["row"], d["col"], d["val"], approx=approx)


def test_dominant_mode_is_moments_of_largest_cluster():
    rng = np.random.default_rng(8)
    K, R = 4, 6
    o = _oracle_for_fit("dm", K)
    runs = []
    for n in range(R):
        sizes = (70, 30) if n % 2 == 0 else (25, 75)
        centres = [rng.standard_normal(K) * 8.0 for _ in sizes]
        runs.append(_chain_of_blobs(rng, centres, sizes, 0.3, K))
    smp = np.stack([r[0] for r in runs], axis=1)        # (S, R, K)
    fit = o.cluster_fit(smp)
    for n, (x, truth) in enumerate(runs):
        big = np.bincount(truth).argmax()
        xs = x[truth == big]
        np.testing.assert_allclose(fit["mu"][n], xs.mean(0), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(np.linalg.inv(fit["Lam"][n]), np.cov(xs.T, ddof=1), rtol=1e-9, atol=1e-12)


def test_dominant_mode_of_one_cluster_is_moment_matching():
    rng = np.random.default_rng(9)
    K, S, R = 3, 50, 8
    smp = rng.standard_normal((S, R, K)) * 0.2 + rng.standard_normal((1, R, K))
    o = _oracle_for_fit("dm", K)
    fit = o.cluster_fit(np.ascontiguousarray(smp))
    lab, ncl = _lmeans(smp, scale=1e6)
    mu = np.zeros((R, K))
    Lam = np.zeros((R, K, K))
    L().orc_mm(R, K, S, ptr(np.ascontiguousarray(smp)), ptr(mu), ptr(Lam))
    o2 = Oracle(2, 2, K, np.array([0], np.int32), np.array([0], np.int32), np.array([1.0], np.float32),
                approx="dm", lambda_scale=1e6)
    fit2 = o2.cluster_fit(np.ascontiguousarray(smp))
    np.testing.assert_array_equal(fit2["mu"], mu)
    np.testing.assert_array_equal(fit2["Lam"], Lam)
    assert fit["mu"].shape == (R, K)


def test_mixture_pooled_moments_obey_total_variance():
    """Three planted clusters, all kept: the pooled mean is the overall sample
    mean, and the pooled covariance is the law of total variance over the
    components' own (unbiased) covariances."""
    rng = np.random.default_rng(21)
    K, R = 3, 4
    runs = []
    for n in range(R):
        sizes = (60, 50, 40)
        centres = [rng.standard_normal(K) * 10.0 for _ in sizes]
        runs.append(_chain_of_blobs(rng, centres, sizes, 0.5, K))
    smp = np.stack([r[0] for r in runs], axis=1)
    o = _oracle_for_fit("gmm", K)
    fit = o.cluster_fit(smp)
    for n, (x, truth) in enumerate(runs):
        np.testing.assert_allclose(fit["mu"][n], x.mean(0), rtol=1e-12, atol=1e-12)
        S = x.shape[0]
        within = sum((truth == c).sum() / S * np.cov(x[truth == c].T, ddof=1) for c in range(3))
        between = sum((truth == c).sum() / S * np.outer(x[truth == c].mean(0) - x.mean(0),
                                                         x[truth == c].mean(0) - x.mean(0)) for c in range(3))
        np.testing.assert_allclose(np.linalg.inv(fit["Lam"][n]), within + between, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(np.sort(fit["pi"][n])[::-1], [60 / 150, 50 / 150, 40 / 150], rtol=1e-15)
        # components sorted by size
        np.testing.assert_allclose(fit["cmu"][n, 0], x[truth == 0].mean(0), rtol=1e-12, atol=1e-12)


def test_mixture_choice_closed_form():
    K = 2
    g = dict(pi=np.array([[0.5, 0.5], [0.9, 0.1], [0.5, 0.5]]),
             mu=np.array([[[0.0, 0.0], [4.0, 0.0]]] * 3),
             Lam=np.array([[np.eye(K), np.eye(K)]] * 3),
             logdet=np.zeros((3, 2)))
    X = np.array([[3.0, 0.0],      # nearer the second mean, equal weights
                  [2.1, 0.0],      # nearer the second mean, but the first weighs 9x
                  [2.0, 0.0]])     # a tie: the lower index
    # log 0.9 - 2.1^2/2 = -2.3105 against log 0.1 - 1.9^2/2 = -4.1076
    np.testing.assert_array_equal(gmm_choice(g, X), [1, 0, 0])
    # a broad component wins far from both means through its log-determinant term
    g2 = dict(pi=np.array([[0.5, 0.5]]), mu=np.array([[[0.0, 0.0], [0.0, 0.0]]]),
              Lam=np.array([[np.eye(K), 0.01 * np.eye(K)]]), logdet=np.array([[0.0, 2 * np.log(0.01)]]))
    assert gmm_choice(g2, np.array([[0.5, 0.0]]))[0] == 0
    assert gmm_choice(g2, np.array([[5.0, 0.0]]))[0] == 1


def test_pp_dm_and_gmm_run_and_degenerate_to_mm_with_one_cluster():
    """Stages 1-3 at 2x2 run under every approximation; with a lambda beyond
    every distance each row keeps one cluster and DM and GMM reproduce the MM
    chain exactly."""
    d = synth.make("ratings", 40, 30, 4, 600, 0.8, 3)
    res = {}
    for approx, scale in (("mm", 2.0), ("dm", 1e6), ("gmm", 1e6), ("dm", 2.0), ("gmm", 2.0)):
        o = Oracle(d["N"], d["D"], 4, d["row"], d["col"], d["val"], I=2, J=2, order="random", seed=5, burnin=3,
                   thin=1, approx=approx, lambda_scale=scale)
        o.run_pp(12)
        o.aggregate()
        res[(approx, scale)] = o.predict(d["test_row"], d["test_col"])
        assert np.isfinite(res[(approx, scale)]).all()
    np.testing.assert_array_equal(res[("dm", 1e6)], res[("mm", 2.0)])
    # the pooled precision of a one-component mixture is Lambda^-1 inverted back: rounding only
    np.testing.assert_allclose(res[("gmm", 1e6)], res[("mm", 2.0)], rtol=1e-12, atol=1e-12)
