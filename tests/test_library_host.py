"""Host-side checks of the HIP library (no GPU needed).

* every symbol include/bmf.h declares is exported by libbmf.so;
* the library's integer work (ordering, partition, CSR/CSC, entry maps) is
  bit-exact against the oracle's independent numpy plan;
* centering constant, validation errors and workspace sizing.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle.native import seq_mean
from oracle.plan import Plan
from paper_1703_00734_amd import BMF, BMFError, exported_symbols, load

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "bmf.h")).read()
    declared = set(re.findall(r"^(?:bmf_status|const char \*)\s*(bmf_\w+)\s*\(", hdr, re.M))
    assert declared == set(exported_symbols())
    L = load()
    for name in declared:
        assert hasattr(L, name), name


def _data(seed=3, N=97, D=61, nnz=900):
    rng = np.random.default_rng(seed)
    cells = rng.choice(N * D, size=nnz, replace=False)
    rng.shuffle(cells)
    row = (cells // D).astype(np.int32)
    col = (cells % D).astype(np.int32)
    val = rng.integers(1, 6, size=nnz).astype(np.float32)
    return N, D, row, col, val


@pytest.mark.parametrize("order", ["given", "random", "decreasing"])
@pytest.mark.parametrize("IJ", [(1, 1), (2, 3), (4, 4), (3, 1), (1, 5)])
def test_plan_bit_exact_against_oracle(order, IJ):
    N, D, row, col, val = _data()
    I, J = IJ
    m = BMF(N, D, 4, row, col, val, I=I, J=J, order=order, seed=77, device=False)
    p = Plan(N, D, row, col, I, J, order, 77)
    pr, pc = m.positions()
    assert np.array_equal(pr, p.row_pos)
    assert np.array_equal(pc, p.col_pos)
    tot = 0
    for b in range(I * J):
        info = m.block_info(b)
        ob = p.blocks[b]
        assert (info["R"], info["C"], info["M"]) == (ob["R"], ob["C"], ob["M"])
        for which, key in ((0, "csr"), (1, "csc")):
            ptr, idx, ent = m.block_csr(b, which)
            assert np.array_equal(ptr, ob[key + "_ptr"])
            assert np.array_equal(idx, ob[key + "_idx"])
            assert np.array_equal(ent, ob[key + "_entry"])
        tot += info["M"]
    assert tot == row.size


def test_plan_with_empty_rows_and_ragged_parts():
    rng = np.random.default_rng(4)
    N, D = 50, 23
    rows = rng.choice(np.arange(0, N, 3), size=80)       # two thirds of rows stay empty
    cols = rng.integers(0, D, size=80)
    cells = np.unique(rows * D + cols)
    row, col = (cells // D).astype(np.int32), (cells % D).astype(np.int32)
    val = np.ones(row.size, dtype=np.float32)
    m = BMF(N, D, 3, row, col, val, I=7, J=4, order="decreasing", device=False)
    p = Plan(N, D, row, col, 7, 4, "decreasing", 0)
    for b in range(28):
        ptr, idx, ent = m.block_csr(b, 0)
        assert np.array_equal(ptr, p.blocks[b]["csr_ptr"])
        assert np.array_equal(ent, p.blocks[b]["csr_entry"])


def test_global_mean_bit_exact():
    N, D, row, col, val = _data(seed=5)
    m = BMF(N, D, 4, row, col, val, device=False)
    assert m.global_mean() == seq_mean(val)


def test_partition_sizes_match_paper(golden_dir):
    # 6040 x 3706 at 5 x 5 gives 1208-row, 742-column subsets
    rng = np.random.default_rng(0)
    N, D = 6040, 3706
    cells = rng.choice(N * D, size=20000, replace=False)
    m = BMF(N, D, 2, cells // D, cells % D, np.ones(cells.size), I=5, J=5, device=False)
    info = m.block_info(0)
    assert info["R"] == 1208 and info["C"] == 742
    last = m.block_info(24)
    assert last["R"] == 6040 - 4 * 1208 and last["C"] == 3706 - 4 * 742


def _expect(status, **kw):
    N, D, row, col, val = _data(seed=6)
    args = dict(N=N, D=D, K=4, row=row, col=col, val=val)
    args.update(kw)
    with pytest.raises(BMFError) as e:
        BMF(device=False, **args)
    assert e.value.status == status


def test_validation_errors():
    N, D, row, col, val = _data(seed=6)
    _expect("BMF_EINVAL", row=np.concatenate([row, row[:1]]), col=np.concatenate([col, col[:1]]),
            val=np.concatenate([val, val[:1]]))                                  # duplicate cell
    bad = row.copy()
    bad[3] = N
    _expect("BMF_EINVAL", row=bad)                                                # out of range
    v = val.copy()
    v[7] = np.nan
    _expect("BMF_EINVAL", val=v)                                                  # non-finite
    _expect("BMF_EUNSUPPORTED", K=65)
    _expect("BMF_EINVAL", K=0)
    _expect("BMF_EINVAL", I=N + 1)
    _expect("BMF_EINVAL", nu0=2.0)                                                # nu0 <= K-1
    _expect("BMF_EINVAL", W0=np.array([[1, 2, 0, 0], [2, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]]))
    _expect("BMF_EINVAL", thin=0)
    _expect("BMF_EINVAL", approx=3)                                               # no such approximation
    _expect("BMF_EINVAL", approx="gmm", ncomp=5)                                  # at most 4 components
    _expect("BMF_EINVAL", approx="dm", lambda_scale=-1.0)
    _expect("BMF_EUNSUPPORTED", approx="dm", K=33, nu0=33.0)                      # clustering needs K <= 32
    _expect("BMF_EUNSUPPORTED", approx="gmm", max_kept=257)                       # labels of 256 samples at most
    _expect("BMF_EUNSUPPORTED", tau_per_column=True, precision="bf16")           # tau_d: FP32 and FP64 only
    # ceil partition that leaves the last part empty: N=10, I=6 -> parts of 2
    rng = np.random.default_rng(1)
    cells = rng.choice(100, size=30, replace=False)
    with pytest.raises(BMFError) as e:
        BMF(10, 10, 2, cells // 10, cells % 10, np.ones(30), I=6, device=False)
    assert e.value.status == "BMF_EINVAL"


def test_mixture_introspection_refused_without_device_or_clusters():
    N, D, row, col, val = _data(seed=7)
    m = BMF(N, D, 4, row, col, val, approx="gmm", device=False)
    for f in (lambda: m.get_clusters(0, 0, 2), lambda: m.get_component(0, 0, 0)):
        with pytest.raises(BMFError) as e:
            f()
        assert e.value.status == "BMF_ESTATE"


def test_device_calls_refused_on_host_context():
    N, D, row, col, val = _data(seed=7)
    m = BMF(N, D, 4, row, col, val, device=False)
    with pytest.raises(BMFError) as e:
        m.gibbs_sweep(1)
    assert e.value.status == "BMF_ESTATE"
    with pytest.raises(BMFError):
        m.predict([0], [0])


def test_workspace_size_grows_with_problem():
    L = load()
    from paper_1703_00734_amd.binding import bmf_config
    sizes = []
    for nnz, K, kept in ((1000, 4, 1), (5000, 4, 1), (5000, 16, 1), (5000, 16, 10)):
        N, D, row, col, val = _data(seed=8, N=200, D=100, nnz=nnz)
        c = bmf_config()
        L.bmf_config_defaults(ctypes.byref(c))
        c.N, c.D, c.K, c.nnz, c.nu0, c.max_kept = N, D, K, nnz, K, kept
        c.row = row.ctypes.data_as(ctypes.c_void_p)
        c.col = col.ctypes.data_as(ctypes.c_void_p)
        c.val = val.ctypes.data_as(ctypes.c_void_p)
        s = ctypes.c_size_t()
        assert L.bmf_workspace_size(ctypes.byref(c), ctypes.byref(s)) == 0
        sizes.append(s.value)
    assert sizes[0] < sizes[1] < sizes[2] < sizes[3]


def test_gather_offsets_that_would_wrap_are_rejected():
    # FP32, K = 16: 64-byte factor rows; a part of 2^26 rows reaches 2^32 bytes
    N, D, row, col, val = _data(seed=9)
    _expect("BMF_EUNSUPPORTED", N=1 << 26, K=16, nu0=16.0, precision="fp32")
    _expect("BMF_EUNSUPPORTED", D=1 << 27, K=16, nu0=16.0, precision="bf16")   # 32-byte rows
    # the same part split in two fits
    m = BMF(1 << 26, D, 16, row, col, val, I=2, nu0=16.0, precision="fp32", device=False)
    assert m.block_info(0)["R"] == 1 << 25


def test_checkpoint_header_checked_before_device(tmp_path):
    N, D, row, col, val = _data(seed=10)
    m = BMF(N, D, 4, row, col, val, device=False)
    with pytest.raises(BMFError) as e:
        m.load_state(str(tmp_path / "missing.bin"))
    assert e.value.status == "BMF_EINVAL"
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a checkpoint" * 40)
    with pytest.raises(BMFError) as e:
        m.load_state(str(junk))
    assert e.value.status == "BMF_EINVAL" and "not a checkpoint" in str(e.value)
    with pytest.raises(BMFError) as e:
        m.save_state(str(tmp_path / "x.bin"))
    assert e.value.status == "BMF_ESTATE"


def test_progress_callback_registers_on_host_context():
    N, D, row, col, val = _data(seed=11)
    m = BMF(N, D, 4, row, col, val, device=False)
    seen = []
    m.set_progress(lambda stage, sweep: seen.append((stage, sweep)) or False)
    m.set_progress(None)
    assert seen == []
    assert load().bmf_status_string(7).decode() == "BMF_EABORT"
