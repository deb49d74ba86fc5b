"""Shared helpers of the GPU parity tests: matched library/oracle pairs."""
import numpy as np

import synth
from oracle.bpmf import Oracle
from paper_1703_00734_amd import BMF

# single conditional step from an identical state and identical noise, the
# draw before any rounding to the state precision: in BF16 mode the inputs are
# the same BF16 values on both sides and the arithmetic is FP32, so the FP32
# bound applies (the stored BF16 state adds its own rounding, 2^-8 per entry,
# checked bit for bit as the rounding of the draw)
TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16": 1e-4}


def small_data(K, seed=1, N=600, D=300, nnz=20000, empty_rows=7, kind="ratings"):
    """Skewed ratings-shaped data plus a few rows with no entries at all."""
    d = synth.make(kind, N, D, K, nnz, 0.8, seed)
    d["N"] = N + empty_rows
    return d


def pair(d, K, precision="fp64", I=1, J=1, order="given", seed=11, burnin=0, thin=1, max_kept=4,
         sample_tau=True, tau_fixed=1.0, batched=True, pivot_theta=0.0, lane_nnz=0, approx="mm",
         lambda_scale=2.0, ncomp=3, tau_per_column=False):
    g = BMF(d["N"], d["D"], K, d["row"], d["col"], d["val"], I=I, J=J, order=order, seed=seed,
            burnin=burnin, thin=thin, max_kept=max_kept, precision=precision,
            sample_tau=sample_tau, tau_fixed=tau_fixed, batched=batched, pivot_theta=pivot_theta,
            lane_nnz=lane_nnz, approx=approx, lambda_scale=lambda_scale, ncomp=ncomp,
            tau_per_column=tau_per_column)
    o = Oracle(d["N"], d["D"], K, d["row"], d["col"], d["val"], I=I, J=J, order=order, seed=seed,
               burnin=burnin, thin=thin, sample_tau=sample_tau, tau_fixed=tau_fixed, approx=approx,
               lambda_scale=lambda_scale, ncomp=ncomp, tau_per_column=tau_per_column)
    return g, o


def random_state(rng, R, C, K, scale=0.7):
    X = scale * rng.standard_normal((R, K))
    W = scale * rng.standard_normal((C, K))
    B = rng.standard_normal((K, K))
    Lx = B @ B.T / K + np.eye(K)
    B = rng.standard_normal((K, K))
    Lw = B @ B.T / K + np.eye(K)
    return dict(X=X, W=W, hx=(Lx, 0.1 * rng.standard_normal(K)),
                hw=(Lw, 0.1 * rng.standard_normal(K)), tau=1.3)


def round_state(x, precision):
    """The values a state of the given precision holds (FP32: round to nearest;
    BF16: round to nearest even of the FP32 value)."""
    if precision in (0, "fp64"):
        return np.array(x, dtype=np.float64)
    f = np.asarray(x, dtype=np.float32)
    if precision in (1, "fp32"):
        return f.astype(np.float64)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def load_state(g, o, b, st):
    """Put the same state into block b of both sides (the oracle receives the
    values the library's state precision holds)."""
    g.set_state(b, X=st["X"], W=st["W"], hx=st["hx"], hw=st["hw"], tau=st["tau"])
    blk = o.blocks[b]
    blk["X"] = round_state(st["X"], g.cfg.precision)
    blk["W"] = round_state(st["W"], g.cfg.precision)
    blk["hx"] = (st["hx"][0].copy(), st["hx"][1].copy())
    blk["hw"] = (st["hw"][0].copy(), st["hw"][1].copy())
    blk["tau"] = st["tau"]


def rel_err_rows(x_gpu, x_or, A_inv_tr, K):
    """||dx_n|| / max(||x_n||, sqrt(tr(A_n^-1)/K)) per row."""
    num = np.linalg.norm(x_gpu - x_or, axis=1)
    den = np.maximum(np.linalg.norm(x_or, axis=1), np.sqrt(np.maximum(A_inv_tr, 0) / K))
    return num / den


def cond_precision_trace(blk, which, K, tau, prior_full):
    """tr(A_n^-1) for every entity of one side (A from the block's data)."""
    if which == "rows":
        ptr, idx, other = blk["csr_ptr"], blk["csr_idx"], blk["W"]
    else:
        ptr, idx, other = blk["csc_ptr"], blk["csc_idx"], blk["X"]
    n = ptr.size - 1
    out = np.empty(n)
    for e in range(n):
        Wn = other[idx[ptr[e]:ptr[e + 1]]]
        P = prior_full[e] if prior_full.ndim == 3 else prior_full
        out[e] = np.trace(np.linalg.inv(P + tau * Wn.T @ Wn))
    return out
