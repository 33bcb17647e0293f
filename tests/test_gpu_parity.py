"""Parity of the HIP far-zone product with the FP64 oracle (needs a GPU).

Every case feeds both sides the same complex64 inputs (the oracle gets them
upcast to complex128) and bounds the relative error of the GPU result by
1e-4, the plain-FP32 target for this product, over the whole result, per
test box and element by element (max norm), for each right-hand side.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import announce, parity, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-4

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()


def make_field(w, max_nrhs=1):
    return U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=max_nrhs)


def run_translate(ff, P):
    Pd = to_dev(P.astype(np.complex64))
    Ed = torch.empty_like(Pd)
    U.translate(ff.plan, Pd, Ed, P.shape[0])
    return to_host(Ed)


@pytest.mark.parametrize("cfg", [1, 2])
def test_translate_parity(cfg):
    w = W.config(cfg)
    announce("translate", w.name)
    ff = make_field(w)
    P = w.coefficients().reshape(1, w.n_box, w.n_u)
    E = run_translate(ff, P)
    ref = O.translate(P.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, w.far_mode)
    parity(E, ref, TOL, boxes=w.n_u, label=f"{w.name} translate")


def test_far_mvm_identity_basis_and_nrhs():
    w = W.config(1, nrhs=3)
    announce("far_mvm identity nrhs=3", w.name)
    ff = make_field(w, max_nrhs=4)
    x = w.coefficients()
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode=w.far_mode)
    parity(y, ref, TOL, boxes=w.n_u, label="identity basis nrhs 3")


@pytest.mark.parametrize("explicit_T", [False, True])
def test_far_mvm_synthetic_basis(explicit_T):
    w = W.config(1)
    announce("far_mvm basis", w.name, "explicit_T", explicit_T)
    nb = np.full(w.n_box, 81)
    nb_ptr, S = W.random_basis(nb, w.n_u, 11)
    T = W.random_basis(nb, w.n_u, 12)[1] if explicit_T else None
    ff = make_field(w, max_nrhs=2)
    Sd = to_dev(S)
    Td = to_dev(T) if explicit_T else None
    ff.set_basis(nb_ptr, Sd, Td)
    x = W.complex_normal((2, int(nb_ptr[-1])), 13)
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, nb_ptr,
                    S.astype(np.complex128),
                    None if T is None else T.astype(np.complex128), w.far_mode)
    parity(y, ref, TOL, boxes=nb_ptr, label=f"basis explicit_T={explicit_T}")


@pytest.mark.parametrize("precision", ["fp32", "split-fp16"])
@pytest.mark.parametrize("nrhs", [3, 4, 5, 8])
def test_basis_rhs_blocks_match_single_vectors(precision, nrhs):
    # stages 1 and 3 read S once per block of up to four right-hand sides
    # (3: one partial block; 5: a full block and a block of one); every
    # vector's result equals the same vector run alone, bit for bit, and the
    # oracle within the bar
    w = W.config(1)
    announce("basis rhs blocks", w.name, precision, "nrhs", nrhs)
    nb = np.full(w.n_box, 81)
    nb_ptr, S = W.random_basis(nb, w.n_u, 21)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=nrhs, precision=precision)
    ff.set_basis(nb_ptr, to_dev(S))
    x = W.complex_normal((nrhs, int(nb_ptr[-1])), 22)
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, nb_ptr,
                    S.astype(np.complex128), mode=w.far_mode)
    for r in range(nrhs):
        y1 = to_host(ff(to_dev(x[r:r + 1])))
        assert np.array_equal(y[r:r + 1], y1), f"rhs {r} differs from its single run"
    parity(y, ref, TOL, boxes=nb_ptr, label=f"{precision} nrhs {nrhs}")
    ff.close()


def test_ragged_basis_with_empty_boxes():
    boxes = W.grid_boxes(4, 4, 5)
    rng = np.random.default_rng(3)
    nb = rng.integers(0, 120, size=len(boxes))
    nb[[0, 7, 33]] = 0
    announce("ragged basis", len(boxes), "boxes, max nb", nb.max())
    nb_ptr, S = W.random_basis(nb, 81, 4)
    ff = U.FarField(boxes, 0.25, 2 * np.pi, 3, "ilist", max_nrhs=2)
    ff.set_basis(nb_ptr, to_dev(S))
    x = W.complex_normal((2, int(nb_ptr[-1])), 5)
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), boxes, 0.25, 2 * np.pi, 3, nb_ptr,
                    S.astype(np.complex128))
    # boxes without functions produce no output entries and take no input
    assert y.shape == ref.shape
    parity(y, ref, TOL, boxes=nb_ptr, label="ragged basis")


def test_stages_separately():
    w = W.config(1)
    announce("stages separately", w.name)
    nb = np.full(w.n_box, 60)
    nb_ptr, S = W.random_basis(nb, w.n_u, 21)
    ff = make_field(w)
    Sd = to_dev(S)
    ff.set_basis(nb_ptr, Sd)
    x = W.complex_normal((1, int(nb_ptr[-1])), 22)
    xd = to_dev(x)
    Pd = torch.empty((1, w.n_box * w.n_u), dtype=torch.complex64, device="cuda")
    U.aggregate(ff.plan, xd, Pd)
    P = to_host(Pd)
    Pref = O.aggregate(x.astype(np.complex128), nb_ptr, S.astype(np.complex128), w.n_u)
    parity(P.reshape(Pref.shape), Pref, 1e-6, boxes=w.n_u, label="stage 1 alone")
    E = W.complex_normal((1, w.n_box * w.n_u), 23)
    yd = torch.empty_like(xd)
    U.disaggregate(ff.plan, to_dev(E), yd)
    Eref = E.astype(np.complex128).reshape(1, w.n_box, w.n_u)
    yref = O.disaggregate(Eref, nb_ptr, S.astype(np.complex128))
    parity(to_host(yd), yref, 1e-6, boxes=nb_ptr, label="stage 3 alone")
    # stage 2 alone ignores the basis
    Et = run_translate(ff, Pref.astype(np.complex64))
    Etref = O.translate(Pref.astype(np.complex64).astype(np.complex128), w.boxes,
                        w.a, w.k, w.n_d)
    parity(Et, Etref, TOL, boxes=w.n_u, label="stage 2 alone")


@pytest.mark.parametrize("n_d,boxes", [
    (1, W.grid_boxes(5, 5, 5)),
    (2, W.grid_boxes(4, 6, 4)),
    (4, W.grid_boxes(4, 4, 4)),
    (4, W.grid_boxes(4, 4, 5)),
])
def test_other_dipole_grids(n_d, boxes):
    announce("n_d", n_d, len(boxes), "boxes")
    n_u = 3 * n_d ** 3
    ff = U.FarField(boxes, 0.25, 2 * np.pi, n_d, "ilist", max_nrhs=2)
    P = W.complex_normal((2, len(boxes), n_u), 30 + n_d)
    E = run_translate(ff, P)
    ref = O.translate(P.astype(np.complex128), boxes, 0.25, 2 * np.pi, n_d)
    parity(E, ref, TOL, boxes=n_u, label=f"n_d {n_d}, {len(boxes)} boxes")


def test_nd4_sphere_full_size():
    # 762-box sphere at a = 0.125, n_d = 4 (192 coefficients per box): the
    # operator-table product with the box vectors staged in LDS, all 22,602
    # pairs, two right-hand sides
    w = W.config(6, nrhs=2)
    announce("n_d=4 sphere", w.name)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=2)
    assert ff.info["mfma"] == 1
    x = w.coefficients()
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode=w.far_mode)
    parity(y, ref, TOL, boxes=w.n_u, label=w.name)
    ff.close()


def test_full_far_set():
    boxes = W.grid_boxes(6, 6, 6)
    announce("full far set 6^3")
    ff = U.FarField(boxes, 0.25, 2 * np.pi, 3, "full")
    P = W.complex_normal((1, 216, 81), 41)
    E = run_translate(ff, P)
    ref = O.translate(P.astype(np.complex128), boxes, 0.25, 2 * np.pi, 3, "full")
    parity(E, ref, TOL, boxes=81, label="FULL 6^3")


def test_low_frequency_regime():
    # a = lambda/256 boxes (the low-frequency example of Sec. 5), 8x8x8 grid
    boxes = W.grid_boxes(8, 8, 8)
    a = 1.0 / 256
    announce("low frequency a=1/256")
    ff = U.FarField(boxes, a, 2 * np.pi, 3, "ilist")
    P = W.complex_normal((1, len(boxes), 81), 51)
    E = run_translate(ff, P)
    ref = O.translate(P.astype(np.complex128), boxes, a, 2 * np.pi, 3)
    parity(E, ref, TOL, boxes=81, label="a = 1/256")


@pytest.mark.parametrize("boxes", [
    np.array([[3, 3, 3]]),                       # one box: no far pair
    np.array([[0, 0, 0], [1, 1, 1]]),           # adjacent: no far pair
    np.array([[0, 0, 0], [9, 9, 9]]),           # far apart, parents not adjacent
])
def test_degenerate_geometries_give_zero(boxes):
    announce("degenerate", boxes.tolist())
    ff = U.FarField(boxes, 0.25, 2 * np.pi, 3, "ilist")
    x = to_dev(W.complex_normal((1, len(boxes) * 81), 61))
    y = to_host(ff(x))
    assert not np.any(y)


def test_two_far_boxes_exact_operator():
    boxes = np.array([[0, 0, 0], [0, 0, 2]])
    announce("two boxes")
    ff = U.FarField(boxes, 0.25, 2 * np.pi, 3, "ilist")
    P = W.complex_normal((1, 2, 81), 62)
    E = run_translate(ff, P)
    ref = O.translate(P.astype(np.complex128), boxes, 0.25, 2 * np.pi, 3)
    parity(E, ref, TOL, boxes=81, label="two boxes")


def test_deterministic_and_linear():
    w = W.config(1)
    announce("determinism/linearity", w.name)
    ff = make_field(w)
    x1 = to_dev(W.complex_normal((1, w.n_box * w.n_u), 71))
    x2 = to_dev(W.complex_normal((1, w.n_box * w.n_u), 72))
    y1a = to_host(ff(x1))
    y1b = to_host(ff(x1))
    assert np.array_equal(y1a, y1b)
    a, b = 0.5 - 2j, 1.5 + 0.25j
    y2 = to_host(ff(x2))
    y12 = to_host(ff((a * x1 + b * x2).to(torch.complex64)))
    assert rel_l2(y12, a * y1a + b * y2) <= 1e-5


def test_argument_errors_on_device():
    w = W.config(1)
    announce("argument errors")
    ff = make_field(w, max_nrhs=1)
    x = to_dev(W.complex_normal((2, w.n_box * w.n_u), 81))
    y = torch.empty_like(x)
    with pytest.raises(U.UbfError) as e:
        U.far_mvm(ff.plan, x, y, 2)          # nrhs beyond the binding
    assert e.value.status == -1
    with pytest.raises(U.UbfError) as e:
        U.far_mvm(ff.plan, x, x, 1)          # aliasing
    assert e.value.status == -1 and "overlap" in str(e.value)
    with pytest.raises(U.UbfError):
        U.far_mvm(ff.plan, x, y, 0)


def test_shell_full_size_three_stage():
    """The benchmarked workload: 3,338-box shell, 81 functions per box, nrhs 1."""
    w = W.config(2)
    announce("shell full size three-stage", w.name)
    nb = np.full(w.n_box, 81)
    nb_ptr, S = W.random_basis(nb, w.n_u, 2)
    ff = make_field(w)
    ff.set_basis(nb_ptr, to_dev(S))
    x = W.complex_normal((1, int(nb_ptr[-1])), 2)
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, nb_ptr,
                    S.astype(np.complex128), mode=w.far_mode)
    parity(y, ref, TOL, boxes=nb_ptr, label=f"{w.name} three-stage")


@pytest.mark.parametrize("variant", ["shell", "plate"])
def test_large_sampled(variant):
    """0.125-wavelength boxes (tens of thousands of boxes): sampled test boxes."""
    w = W.config(3, variant=variant)
    announce("large sampled", w.name, w.n_box)
    ff = make_field(w)
    P = w.coefficients().reshape(1, w.n_box, w.n_u)
    E = run_translate(ff, P)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(w.n_box, size=48, replace=False))
    ref = O.translate(P.astype(np.complex128), w.boxes, w.a, w.k, w.n_d,
                      test_boxes=sample)
    parity(E[:, sample], ref[:, sample], TOL, boxes=w.n_u, label=f"{w.name} sampled")


def test_benchmarked_configuration_after_tune():
    """Exactly what the benchmark times: the 3,338-box shell, 81 synthetic
    functions per box, split FP16, one right-hand side, the persistent
    stage-2 grid chosen by the tuner. Tuning changes no bit of the result."""
    w = W.config(2)
    announce("benchmarked configuration", w.name, "split-fp16 nrhs 1 tuned")
    nb = np.full(w.n_box, 81)
    nb_ptr, S = W.random_basis(nb, w.n_u, 2)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=1, precision="split-fp16")
    Sd = to_dev(S)
    ff.set_basis(nb_ptr, Sd)
    x = W.complex_normal((1, int(nb_ptr[-1])), 2)
    xd = to_dev(x)
    y0 = to_host(ff(xd))
    ff.tune(nrhs=1, reps=3)
    y = to_host(ff(xd))
    assert np.array_equal(y, y0)
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, nb_ptr,
                    S.astype(np.complex128), mode=w.far_mode)
    parity(y, ref, TOL, boxes=nb_ptr, label=f"{w.name} split-fp16 tuned")
    ff.close()
