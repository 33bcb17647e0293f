"""ubf_far_mvm_noalloc: the product with its intermediates in the library's
static device array, checked against ubf_far_mvm (needs a GPU).

Both entry points run the same kernels on the same inputs, so results must
agree bit for bit. Two calls in a row, the second with a smaller input,
then the first again; a call too large for the array is refused before any
device work, and the plan's own entry point is unaffected.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import announce, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()


def _both(ff, x):
    xd = to_dev(x)
    y_ref = to_host(ff(xd))
    y = torch.empty_like(xd)
    U.far_mvm_noalloc(ff.plan, xd, y, x.shape[0])
    return to_host(y), y_ref


def test_noalloc_matches_far_mvm_large_then_small():
    w = W.config(2)
    announce("noalloc: shell, split-fp16, synthetic basis, nrhs 1")
    nb = np.full(w.n_box, 81)
    nb_ptr, S = W.random_basis(nb, w.n_u, 2)
    big = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=2, precision="split-fp16")
    Sd = to_dev(S)
    big.set_basis(nb_ptr, Sd)
    x1 = W.complex_normal((1, int(nb_ptr[-1])), 31)
    y, y_ref = _both(big, x1)
    assert np.isfinite(y).all() and np.any(y)
    assert np.array_equal(y, y_ref)

    # second call, smaller input: 6^3 grid, FP32, identity basis, 2 vectors
    small_w = W.config(1, nrhs=2)
    announce("noalloc: 6^3 grid, fp32, identity basis, nrhs 2")
    small = U.FarField(small_w.boxes, small_w.a, small_w.k, small_w.n_d, small_w.far_mode,
                       max_nrhs=2)
    y, y_ref = _both(small, small_w.coefficients())
    assert np.array_equal(y, y_ref)

    # the large call again: nothing left over from the smaller one matters
    announce("noalloc: shell again")
    x2 = W.complex_normal((1, int(nb_ptr[-1])), 32)
    y, y_ref = _both(big, x2)
    assert np.array_equal(y, y_ref)

    # too large for the array (two vectors on the shell: about 151 MB)
    x3 = to_dev(W.complex_normal((2, int(nb_ptr[-1])), 33))
    y3 = torch.empty_like(x3)
    with pytest.raises(U.UbfError) as e:
        U.far_mvm_noalloc(big.plan, x3, y3, 2)
    assert e.value.status == -1 and "static scratch" in str(e.value)
    # the plan's own entry point still runs on its workspace
    y_ws = to_host(big(x3))
    for r in range(2):
        assert np.array_equal(y_ws[r:r + 1], to_host(big(x3[r:r + 1].contiguous())))
    big.close()
    small.close()


def test_noalloc_argument_errors():
    w = W.config(1)
    announce("noalloc: argument errors")
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=1)
    x = to_dev(w.coefficients())
    with pytest.raises(U.UbfError) as e:
        U.far_mvm_noalloc(ff.plan, x, x, 1)
    assert e.value.status == -1 and "overlap" in str(e.value)
    y = torch.empty_like(x)
    with pytest.raises(U.UbfError) as e:
        U.far_mvm_noalloc(ff.plan, x, y, 2)
    assert e.value.status == -1
    ff.close()
