"""Seeded synthetic workloads shaped like the paper's matrix-completion data.

Shared input generator for the oracle and the GPU library.  It holds no part of
the method's arithmetic: it only draws a COO matrix, a train/test split and
ground-truth factors.  All draws use numpy's Generator(Philox(seed)).

Recipes (the paper's real datasets are not used; these stand in for their
shapes, sparsity and degree skew):

* ``uniform``: nnz distinct cells uniformly without replacement; X, W ~ N(0, 1);
  y = x^T w + N(0, sigma^2).
* ``ratings``: row and column degree targets Zipf(s) over random ranks,
  d = clip(round(c * rank^-s), dmin, cap), c found by bisection so that the
  targets sum to nnz; cells by a configuration-model pairing of row and column
  stubs, duplicates removed, topped up by degree-proportional pairs and
  trimmed to nnz, then every row and column raised to dmin entries;
  x, w ~ N(0, K^-1/2) entry-wise (var x^T w = 1);
  y = round(clip(x^T w + N(0, noise^2) + 3, 1, 5)).
* ``gaussian``: the ratings degree structure with x, w ~ N(0, 1) and
  y = K^-1/2 x^T w + N(0, noise^2).
* Split: a uniformly random 90 % of the observed cells are training data.
"""
import os

import numpy as np

CONFIGS = {
    1: dict(kind="uniform", N=1000, D=500, K=10, nnz=25_000, noise=0.5, I=1, J=1,
            order="given", precision="fp64", sweeps=50, burnin=20),
    2: dict(kind="ratings", N=70_000, D=10_700, K=10, nnz=10_000_000, noise=0.8, I=1, J=1,
            order="given", precision="fp32", sweeps=100, burnin=40),
    3: dict(kind="ratings", N=100_000, D=20_000, K=16, nnz=20_000_000, noise=0.8, I=4, J=4,
            order="random", precision="fp32", sweeps=60, burnin=20),
    4: dict(kind="gaussian", N=200_000, D=20_000, K=64, nnz=40_000_000, noise=1.0, I=1, J=1,
            order="given", precision="bf16", sweeps=60, burnin=20),
    5: dict(kind="ratings", N=480_000, D=17_800, K=32, nnz=100_000_000, noise=0.8, I=8, J=8,
            order="decreasing", precision="bf16", sweeps=60, burnin=20),
}


def _rng(seed):
    return np.random.Generator(np.random.Philox(int(seed)))


def zipf_targets(n, total, s, dmin, cap, rng):
    """Degree targets clip(round(c * rank^-s), dmin, cap) summing to ~total."""
    ranks = rng.permutation(n).astype(np.float64) + 1.0
    base = ranks ** (-s)

    def deg(c):
        return np.clip(np.rint(c * base), dmin, cap)

    lo, hi = 0.0, float(total) * 4.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if deg(mid).sum() < total:
            lo = mid
        else:
            hi = mid
    return deg(hi).astype(np.int64)


def _dedupe(keys):
    return np.unique(keys)


def _union(keys, new):
    """Sorted set union of a sorted unique key array and new keys: the new keys
    are deduplicated on their own, those already present dropped by binary
    search, and the two sorted runs merged (a stable sort of two runs is a
    linear merge), instead of re-sorting the whole set."""
    new = np.unique(new)
    if keys.size:
        pos = np.minimum(np.searchsorted(keys, new), keys.size - 1)
        new = new[keys[pos] != new]
    out = np.concatenate([keys, new])
    out.sort(kind="stable")
    return out


def _quiet(msg):
    pass


def ratings_cells(N, D, nnz, s, dmin, rng, progress=_quiet):
    """Configuration-model cells with Zipf row/column degree targets."""
    nnz = min(int(nnz), N * D)
    dr = zipf_targets(N, nnz, s, dmin, D, rng)
    dc = zipf_targets(D, nnz, s, dmin, N, rng)
    m = int(min(dr.sum(), dc.sum()))
    rs = np.repeat(np.arange(N, dtype=np.int64), dr)[:m]
    cs = np.repeat(np.arange(D, dtype=np.int64), dc)
    cs = cs[rng.permutation(cs.size)[:m]]
    keys = _dedupe(rs * D + cs)
    progress("cells: configuration model paired, %d distinct" % keys.size)
    pr = dr / dr.sum()
    pc = dc / dc.sum()
    for _ in range(50):
        if keys.size >= nnz:
            break
        extra = int((nnz - keys.size) * 1.3) + 1024
        r = rng.choice(N, size=extra, p=pr)
        c = rng.choice(D, size=extra, p=pc)
        keys = _union(keys, r * D + c)
        progress("cells: topped up to %d distinct" % keys.size)
    if keys.size > nnz:
        keys = np.sort(keys[rng.permutation(keys.size)[:nnz]])
    # raise every row and column to dmin entries
    for _ in range(20):
        row = keys // D
        col = keys % D
        rcnt = np.bincount(row, minlength=N)
        ccnt = np.bincount(col, minlength=D)
        need_r = np.nonzero(rcnt < min(dmin, D))[0]
        need_c = np.nonzero(ccnt < min(dmin, N))[0]
        if need_r.size == 0 and need_c.size == 0:
            break
        add = []
        if need_r.size:
            rr = np.repeat(need_r, dmin)
            add.append(rr * D + rng.choice(D, size=rr.size, p=pc))
        if need_c.size:
            cc = np.repeat(need_c, dmin)
            add.append(rng.choice(N, size=cc.size, p=pr) * D + cc)
        keys = _union(keys, np.concatenate(add))
        progress("cells: minimum degree pass, %d distinct" % keys.size)
    return keys // D, keys % D


def uniform_cells(N, D, nnz, rng):
    keys = np.sort(rng.choice(N * D, size=int(nnz), replace=False))
    return keys // D, keys % D


def _dot_rows(X, W, row, col, chunk=1 << 22):
    out = np.empty(row.size, dtype=np.float64)
    for a in range(0, row.size, chunk):
        b = min(row.size, a + chunk)
        out[a:b] = np.einsum("ij,ij->i", X[row[a:b]], W[col[a:b]])
    return out


def make(kind, N, D, K, nnz, noise, seed, zipf_s=1.2, dmin=5, train_frac=0.9, progress=_quiet, **_):
    """Draw one workload.  Returns a dict with the COO train and test sets.
    `progress(msg)` is called after each phase of a large draw."""
    rng = _rng(seed)
    if kind == "uniform":
        row, col = uniform_cells(N, D, nnz, rng)
        X = rng.standard_normal((N, K))
        W = rng.standard_normal((D, K))
        y = _dot_rows(X, W, row, col) + noise * rng.standard_normal(row.size)
    elif kind == "ratings":
        row, col = ratings_cells(N, D, nnz, zipf_s, dmin, rng, progress)
        sd = K ** -0.25
        X = sd * rng.standard_normal((N, K))
        W = sd * rng.standard_normal((D, K))
        y = _dot_rows(X, W, row, col) + noise * rng.standard_normal(row.size) + 3.0
        y = np.rint(np.clip(y, 1.0, 5.0))
    elif kind == "gaussian":
        row, col = ratings_cells(N, D, nnz, zipf_s, dmin, rng, progress)
        X = rng.standard_normal((N, K))
        W = rng.standard_normal((D, K))
        y = K ** -0.5 * _dot_rows(X, W, row, col) + noise * rng.standard_normal(row.size)
    else:
        raise ValueError(kind)
    progress("values drawn for %d cells" % row.size)
    perm = rng.permutation(row.size)
    ntr = int(round(train_frac * row.size))
    tr, te = np.sort(perm[:ntr]), np.sort(perm[ntr:])
    return dict(N=int(N), D=int(D), K=int(K),
                row=row[tr].astype(np.int32), col=col[tr].astype(np.int32),
                val=y[tr].astype(np.float32),
                test_row=row[te].astype(np.int32), test_col=col[te].astype(np.int32),
                test_val=y[te].astype(np.float32))


def simulated(seed, missing="mar", N=6040, D=3706, K=5, observed=0.2, progress=_quiet):
    """The simulated data of the paper's experiments (Sec. 5.3): X, W with
    standard-normal entries, Y = X W^T + E with standard-normal noise (so the
    true tau is 1), N = 6040 rows, D = 3706 columns, K = 5.  Missingness:

    * "mar": a uniformly random 80 % of the cells is missing (the test set),
      the remaining 20 % is the training set;
    * "structured": rows and columns get weights equally spaced from 0.9 down
      to 0.005, and cell (n, d) is observed (training) with probability
      w_n w_d, which leaves about 80 % missing (the paper's text says the
      product is the probability of being assigned to the test set, which
      would leave about 20 % missing; its own figure of 80 % fixes this
      reading).

    Every missing cell is a test cell.  Returns the COO train and test sets as
    ``make`` does."""
    rng = _rng(seed)
    X = rng.standard_normal((N, K))
    W = rng.standard_normal((D, K))
    Y = X @ W.T + rng.standard_normal((N, D))
    if missing == "mar":
        obs = np.zeros(N * D, dtype=bool)
        obs[rng.permutation(N * D)[:int(round(observed * N * D))]] = True
        obs = obs.reshape(N, D)
    elif missing == "structured":
        wn = np.linspace(0.9, 0.005, N)
        wd = np.linspace(0.9, 0.005, D)
        obs = rng.random((N, D)) < np.outer(wn, wd)
    else:
        raise ValueError(missing)
    progress("simulated %s: %d observed of %d cells" % (missing, int(obs.sum()), N * D))
    tr_r, tr_c = np.nonzero(obs)
    te_r, te_c = np.nonzero(~obs)
    return dict(N=int(N), D=int(D), K=int(K),
                row=tr_r.astype(np.int32), col=tr_c.astype(np.int32), val=Y[tr_r, tr_c].astype(np.float32),
                test_row=te_r.astype(np.int32), test_col=te_c.astype(np.int32),
                test_val=Y[te_r, te_c].astype(np.float32))


_CACHE = {}


def config(cid, seed=1, progress=_quiet):
    """Workload of one of the five benchmark configurations.  Draws are kept for
    the life of the process (the caller gets a fresh dict over the same arrays,
    which must not be written in place); with BMF_SYNTH_CACHE set to a
    directory they are also kept there as .npz files between processes."""
    key = (int(cid), int(seed))
    if key in _CACHE:
        return dict(_CACHE[key])
    path = None
    cache_dir = os.environ.get("BMF_SYNTH_CACHE")
    if cache_dir:
        path = os.path.join(cache_dir, "config%d_seed%d.npz" % key)
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                d = {k: (z[k].item() if z[k].ndim == 0 else z[k]) for k in z.files}
            progress("loaded %s" % path)
            _CACHE[key] = d
            return dict(d)
    c = CONFIGS[cid]
    d = make(c["kind"], c["N"], c["D"], c["K"], c["nnz"], c["noise"], seed, progress=progress)
    for k, v in d.items():
        if isinstance(v, np.ndarray):
            v.flags.writeable = False
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        tmp = path + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, **d)
        os.replace(tmp, path)
    _CACHE.clear()                       # one large workload at a time
    _CACHE[key] = d
    return dict(d)
