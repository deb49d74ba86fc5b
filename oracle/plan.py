"""Integer work of the oracle: ordering, r x c partition, per-block CSR/CSC.

TEST INFRASTRUCTURE ONLY.  Plain numpy, written for reading against the text:

* ordering (Sec. 5.2, "Test setup"): rows and columns are either permuted
  randomly, or sorted by decreasing number of observations.  The random order
  here is a stable sort on a Philox key per entity, counter
  (n, 0, (0xFFFFFF << 8) | purpose, 0), first output word, ties by id; the
  decreasing order is a stable sort on (-count, id); "given" keeps the ids.
* partition (Sec. 3, eq. joint_MF_posterior; Sec. 5.2): a scheme r x c splits
  the ordered rows into r parts and the ordered columns into c parts, of size
  ceil(N / r) (the last part takes the rest; an empty part is an error).
* observed sets Omega_n, Omega_d (Sec. 2.1, eq. BMF_likelihood): per block,
  CSR sorted by (local row, local col) and CSC sorted by (local col, local row).
"""
import numpy as np

from . import native

PURPOSE = dict(INIT_X=0, INIT_W=1, ROW=2, COL=3, HYPER_X=4, HYPER_W=5, TAU=6,
               PERM_ROW=7, PERM_COL=8)
ORDERS = ("given", "random", "decreasing")


def counter_c2(block, purpose):
    return ((int(block) & 0xFFFFFF) << 8) | PURPOSE[purpose]


def order_entities(n, counts, order, seed, purpose):
    """Return pos[n]: the position of entity n in the chosen order."""
    ids = np.arange(n, dtype=np.int64)
    if order == "given":
        perm = ids
    elif order == "random":
        ctr = np.zeros((n, 4), dtype=np.uint32)
        ctr[:, 0] = ids.astype(np.uint32)
        ctr[:, 2] = counter_c2(0xFFFFFF, purpose)
        key = native.philox_batch(ctr, seed)[:, 0].astype(np.int64)
        perm = np.lexsort((ids, key))          # by key, ties by id
    elif order == "decreasing":
        perm = np.lexsort((ids, -counts.astype(np.int64)))
    else:
        raise ValueError("unknown order %r" % (order,))
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = ids
    return pos


def part_sizes(n, parts):
    """Sizes of the r parts of n ordered entities, each ceil(n / r)."""
    bs = -(-n // parts)
    sizes = [min(bs, n - p * bs) for p in range(parts)]
    if parts < 1 or min(sizes) <= 0:
        raise ValueError("partition leaves an empty part (n=%d, parts=%d)" % (n, parts))
    return bs, sizes


class Plan:
    """Ordering + partition + per-block CSR/CSC of a COO training set."""

    def __init__(self, N, D, row, col, I, J, order, seed):
        row = np.asarray(row, dtype=np.int64)
        col = np.asarray(col, dtype=np.int64)
        self.N, self.D, self.I, self.J = int(N), int(D), int(I), int(J)
        rc = np.bincount(row, minlength=N)
        cc = np.bincount(col, minlength=D)
        self.row_pos = order_entities(N, rc, order, seed, "PERM_ROW")
        self.col_pos = order_entities(D, cc, order, seed, "PERM_COL")
        self.bs_r, self.R = part_sizes(N, I)
        self.bs_c, self.C = part_sizes(D, J)
        self.row_block = self.row_pos // self.bs_r
        self.row_local = self.row_pos % self.bs_r
        self.col_block = self.col_pos // self.bs_c
        self.col_local = self.col_pos % self.bs_c
        # entity id of every (block, local) slot
        self.row_ids = _inverse_ids(self.row_block, self.row_local, self.R)
        self.col_ids = _inverse_ids(self.col_block, self.col_local, self.C)
        # entries of every block, in CSR and CSC order
        eb = self.row_block[row] * J + self.col_block[col]
        lr = self.row_local[row]
        lc = self.col_local[col]
        self.blocks = []
        for b in range(I * J):
            i, j = divmod(b, J)
            sel = np.nonzero(eb == b)[0]
            r_, c_ = lr[sel], lc[sel]
            csr_perm = sel[np.lexsort((c_, r_))]
            csc_perm = sel[np.lexsort((r_, c_))]
            blk = dict(i=i, j=j, R=self.R[i], C=self.C[j], M=sel.size,
                       csr_entry=csr_perm, csc_entry=csc_perm)
            blk["csr_ptr"] = _ptr(self.row_local[row[csr_perm]], self.R[i])
            blk["csr_idx"] = self.col_local[col[csr_perm]].astype(np.int32)
            blk["csc_ptr"] = _ptr(self.col_local[col[csc_perm]], self.C[j])
            blk["csc_idx"] = self.row_local[row[csc_perm]].astype(np.int32)
            self.blocks.append(blk)


def _ptr(sorted_keys, n):
    counts = np.bincount(sorted_keys, minlength=n)
    p = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=p[1:])
    return p


def _inverse_ids(block, local, sizes):
    out = [np.empty(s, dtype=np.int64) for s in sizes]
    ids = np.arange(block.size, dtype=np.int64)
    for p, s in enumerate(sizes):
        m = block == p
        out[p][local[m]] = ids[m]
    return out


def stage_of(i, j):
    """Stage of block (i, j), 0-based (eq. stage1, stage2a/b, stage3)."""
    if i == 0 and j == 0:
        return 1
    if i == 0 or j == 0:
        return 2
    return 3
