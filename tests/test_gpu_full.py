"""FULL far set at the shell's scale (needs a GPU): every pair with
Chebyshev offset >= 2 among 3,338 boxes (11,105,714 pairs over 148,018
distinct offsets, one operator each, 8 GB of table in device memory),
checked against the FP64 oracle on sampled test boxes."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import announce, parity, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("split-fp16", 1e-4)])
def test_full_far_set_shell_sampled(precision, tol):
    w = W.config(2, far_mode="full")
    announce("FULL shell", precision)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, "full", precision=precision)
    info = ff.info
    assert info["n_pairs"] == 11105714 and info["n_offsets"] == 148018
    P = w.coefficients(seed=21).reshape(1, w.n_box, w.n_u)
    Pd = to_dev(P)
    Ed = torch.empty_like(Pd)
    U.translate(ff.plan, Pd, Ed, 1)
    E = to_host(Ed)
    ff.close()
    rng = np.random.default_rng(22)
    sample = np.sort(rng.choice(w.n_box, size=4, replace=False))
    ref = O.translate(P.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode="full",
                      test_boxes=sample)
    parity(E[:, sample], ref[:, sample], tol, boxes=w.n_u, label=f"FULL {precision} sampled")
