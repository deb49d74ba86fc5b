"""The device planner against the host planner (needs an MI355X).

bmf_init lays out the ordering, the r x c partition and every block's CSR and
CSC (Sec. 5.2, Sec. 3, eq. BMF_likelihood) on the GPU by one radix sort of a
unique key per entry and order; the host planner (plan_on_host, and the host
contexts the oracle's plan is pinned against) does it with stable counting
sorts.  Both must give the same plan bit for bit -- positions, block sizes,
pointers, local ids, COO entries -- and the same chain; invalid input must be
refused with the host planner's messages.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import small_data
from paper_1703_00734_amd import BMF, BMFError

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ctx(d, K, I, J, order, host, **kw):
    # a fixed lane-group size: the autotuner's timed choice may differ between
    # two contexts, and with it the order of the FP32 sums
    return BMF(d["N"], d["D"], K, d["row"], d["col"], d["val"], I=I, J=J, order=order, seed=41, burnin=1,
               max_kept=4, precision="fp32", plan_on_host=host, lane_nnz=16, **kw)


@pytest.mark.parametrize("order", ["given", "random", "decreasing"])
@pytest.mark.parametrize("IJ", [(1, 1), (3, 2), (7, 5)])
def test_device_plan_equals_host_plan(order, IJ):
    K = 6
    d = small_data(K, seed=11, N=900, D=410, nnz=25000, empty_rows=9)
    I, J = IJ
    print("case", order, IJ, flush=True)
    g = _ctx(d, K, I, J, order, False)
    h = _ctx(d, K, I, J, order, True)
    for a, b in zip(g.positions(), h.positions()):
        np.testing.assert_array_equal(a, b)
    for blk in range(I * J):
        assert g.block_info(blk) == h.block_info(blk)
        for which in (0, 1):
            for a, b in zip(g.block_csr(blk, which), h.block_csr(blk, which)):
                np.testing.assert_array_equal(a, b)
    # the same chain from the same plan
    for s in (1, 2, 3):
        g.pp_stage(s, 3)
        h.pp_stage(s, 3)
    np.testing.assert_array_equal(g.predict(d["test_row"], d["test_col"]), h.predict(d["test_row"], d["test_col"]))
    g.close()
    h.close()


def test_device_plan_at_scale_equals_host_plan():
    """A 2M-entry ratings-shaped matrix on a 4 x 4 decreasing-order partition."""
    K = 8
    d = synth.make("ratings", 60000, 9000, K, 2000000, 0.8, 13)
    g = _ctx(d, K, 4, 4, "decreasing", False)
    h = _ctx(d, K, 4, 4, "decreasing", True)
    for blk in range(16):
        assert g.block_info(blk) == h.block_info(blk)
        for which in (0, 1):
            for a, b in zip(g.block_csr(blk, which), h.block_csr(blk, which)):
                np.testing.assert_array_equal(a, b)
    g.pp_stage(1, 2)
    h.pp_stage(1, 2)
    np.testing.assert_array_equal(g.get_state(0)["W"], h.get_state(0)["W"])
    g.close()
    h.close()


def test_device_plan_refuses_bad_input_like_the_host():
    d = small_data(4, seed=5, N=200, D=100, nnz=3000, empty_rows=0)
    row, col, val = d["row"], d["col"], d["val"]
    msgs = []
    for host in (False, True):
        with pytest.raises(BMFError) as e:
            BMF(d["N"], d["D"], 4, np.concatenate([row, row[5:6]]), np.concatenate([col, col[5:6]]),
                np.concatenate([val, val[5:6]]), I=2, J=2, plan_on_host=host)
        assert e.value.status == "BMF_EINVAL"
        msgs.append(str(e.value))
        bad = row.copy()
        bad[17] = d["N"] + 3
        with pytest.raises(BMFError) as e:
            BMF(d["N"], d["D"], 4, bad, col, val, plan_on_host=host)
        assert e.value.status == "BMF_EINVAL"
        msgs.append(str(e.value))
    assert msgs[0] == msgs[2] and msgs[1] == msgs[3]
