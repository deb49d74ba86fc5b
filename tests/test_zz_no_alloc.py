"""The allocation-free prediction entry point against bmf_predict (needs an MI355X).

bmf_predict_noalloc stages its pairs through the library's fixed device array
instead of the context's workspace; on two calls in a row, the second with a
smaller input, its outputs must equal bmf_predict's bit for bit (the same
kernel arithmetic).  Sizes beyond the array and calls before aggregation are
refused.
"""
import numpy as np
import pytest

from gpu_helpers import pair, small_data
from paper_1703_00734_amd import BMFError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision,K,IJ", [("fp64", 6, (1, 1)), ("bf16", 10, (2, 3)), ("fp32", 32, (3, 2))])
def test_predict_noalloc_equals_predict(precision, K, IJ):
    print("case noalloc", precision, K, IJ, flush=True)
    d = small_data(K, seed=50 + K, N=800, D=350, nnz=30000)
    g, _ = pair(d, K, precision, I=IJ[0], J=IJ[1], order="random", burnin=3, max_kept=8)
    for s in (1, 2, 3):
        g.pp_stage(s, 10)
    with pytest.raises(BMFError) as e:
        g.predict_noalloc(d["test_row"][:5], d["test_col"][:5])
    assert e.value.status == "BMF_ESTATE"
    g.aggregate()
    rng = np.random.default_rng(K)
    rows = np.concatenate([d["test_row"], rng.integers(0, d["N"], 20000)]).astype(np.int32)
    cols = np.concatenate([d["test_col"], rng.integers(0, d["D"], 20000)]).astype(np.int32)
    want = g.predict(rows, cols)
    got = g.predict_noalloc(rows, cols)
    assert np.array_equal(got, want)
    half = rows.size // 3
    got2 = g.predict_noalloc(rows[-half:], cols[-half:])
    assert np.array_equal(got2, want[-half:])
    assert g.predict_noalloc(rows[:0], cols[:0]).size == 0
    with pytest.raises(BMFError) as e:
        g.predict_noalloc(np.zeros((1 << 20) + 1, np.int32), np.zeros((1 << 20) + 1, np.int32))
    assert e.value.status == "BMF_EINVAL"
    bad = rows[:4].copy()
    bad[2] = d["N"]
    with pytest.raises(BMFError) as e:
        g.predict_noalloc(bad, cols[:4])
    assert e.value.status == "BMF_EINVAL"
    # a second context on the same GPU shares the array: sequential calls agree
    h, _ = pair(d, K, precision, I=IJ[0], J=IJ[1], order="random", burnin=3, max_kept=8, seed=12)
    for s in (1, 2, 3):
        h.pp_stage(s, 10)
    other = h.predict(rows, cols)
    assert np.array_equal(h.predict_noalloc(rows, cols), other)
    assert np.array_equal(g.predict_noalloc(rows[:half], cols[:half]), want[:half])
    g.close()
    h.close()
