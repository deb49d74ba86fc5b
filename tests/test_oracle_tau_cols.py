"""Pins of the oracle's per-column noise precisions (CPU only).

The tau_d variant of Sec. 2.1 (y_nd ~ N(x_n^T w_d, 1/tau_d)): the row update
weights each observed entry by its column's tau_d, the column update uses its
own tau_d, and each tau_d is drawn from its Gamma posterior.  Checked against a
closed-form one-dimensional conditional with two differently weighted entries,
the scalar update when every tau_d is equal, the Gamma posterior of each
column separately (Kolmogorov-Smirnov), and a swapped-column planted mistake.
"""
import numpy as np
from scipy import stats

from oracle import native
from oracle.bpmf import Oracle
from oracle.native import ptr

import synth

L = native.lib


def test_weighted_row_conditional_closed_form():
    """K = 1, prior N(0, 1), two entries with w = (1, 2), r = (0.7, -0.4) and
    column precisions (3, 0.5): A = 1 + 3 + 0.5 * 4 = 6, h = 3 * 0.7 + 0.5 * (-0.4) * 2,
    x = h / A + z / sqrt(A) with the row's own normal z."""
    ptr_ = np.array([0, 2], dtype=np.int64)
    idx = np.array([0, 1], dtype=np.int32)
    val = np.array([0.7, -0.4])
    other = np.array([[1.0], [2.0]])
    wt = np.array([3.0, 0.5])
    P, m = np.array([1.0]), np.array([0.0])
    out = np.zeros(1)
    seed, t, c2 = 11, 4, 0x502
    assert L().orc_update_side_w(1, 1, ptr(ptr_), ptr(idx), ptr(val), ptr(other), ptr(wt), None, 0, ptr(P),
                                 ptr(m), 1.0, seed, t, c2, ptr(out), 1) == 0
    z = native.normals(seed, 0, t, c2, 1)[0]
    A = 1.0 + 3.0 * 1.0 + 0.5 * 4.0
    h = 3.0 * 0.7 * 1.0 + 0.5 * (-0.4) * 2.0
    assert abs(out[0] - (h / A + z / np.sqrt(A))) < 1e-14


def test_equal_column_precisions_reduce_to_the_scalar_update():
    d = synth.make("ratings", 60, 40, 3, 900, 0.8, 2)
    rng = np.random.default_rng(4)
    for which in ("rows", "cols"):
        o1 = Oracle(d["N"], d["D"], 3, d["row"], d["col"], d["val"], seed=9, tau_per_column=True)
        o2 = Oracle(d["N"], d["D"], 3, d["row"], d["col"], d["val"], seed=9)
        for o in (o1, o2):
            o.begin_stage(1)
        b1, b2 = o1.blocks[0], o2.blocks[0]
        X, W = rng.standard_normal((b1["R"], 3)), rng.standard_normal((b1["C"], 3))
        for b in (b1, b2):
            b["X"], b["W"] = X.copy(), W.copy()
        b1["tau"] = np.full(b1["C"], 1.7)
        b2["tau"] = 1.7
        getattr(o1, "update_" + which)(b1, 3)
        getattr(o2, "update_" + which)(b2, 3)
        key = "X" if which == "rows" else "W"
        np.testing.assert_allclose(b1[key], b2[key], rtol=1e-12, atol=1e-13)


def test_column_precision_draws_follow_their_own_posteriors():
    """Each column's draw over many sweeps is Gamma(a0 + M_d/2, b0 + SSE_d/2) of
    its own M_d and SSE_d; giving column 0 the counts of column 1 (a swapped
    index) fails the test."""
    C = 4
    sse = np.array([3.0, 40.0, 0.5, 12.0])
    cnt = np.array([10, 200, 3, 50], dtype=np.int64)
    a0, b0 = 1.0, 1.0
    draws = np.zeros((3000, C))
    for t in range(draws.shape[0]):
        out = np.zeros(C)
        L().orc_tau_cols(C, ptr(sse), ptr(cnt), a0, b0, 17, t, 0x306, ptr(out))
        draws[t] = out
    for dcol in range(C):
        shape, rate = a0 + cnt[dcol] / 2, b0 + sse[dcol] / 2
        assert stats.kstest(draws[:, dcol] * rate, "gamma", args=(shape,)).pvalue > 1e-3
    shape, rate = a0 + cnt[1] / 2, b0 + sse[1] / 2
    assert stats.kstest(draws[:, 0] * rate, "gamma", args=(shape,)).pvalue < 1e-6
    # distinct columns take distinct counters
    assert len(set(np.round(draws[0] * (b0 + sse / 2), 12))) == C


def test_pp_chain_with_column_precisions_runs():
    d = synth.make("ratings", 80, 50, 3, 1500, 0.8, 3)
    o = Oracle(d["N"], d["D"], 3, d["row"], d["col"], d["val"], I=2, J=2, order="random", seed=5, burnin=2,
               tau_per_column=True)
    o.run_pp(8)
    o.aggregate()
    p = o.predict(d["test_row"], d["test_col"])
    assert np.isfinite(p).all()
    taus = np.concatenate([blk["tau"] for blk in o.blocks])
    assert taus.size == sum(blk["C"] for blk in o.blocks) and (taus > 0).all()
