"""Operators evaluated inside the translation kernel (needs a GPU).

With ``operators="generated"`` no operator table exists: each time the
stage-2 kernel stages an offset's operator it evaluates the dyadic Green's
function of Eq. (5)-(6) once per lattice difference of the dipole sites
(distance and phase in FP64, the rest in FP32) and fills the operator of
Eq. (12)-(13) in LDS, split as the host table is. The results are checked
against the FP64 oracle (same bars as the table forms: 1e-4 for the split
forms, 1e-3 for the single FP16 product, element by element and per test
box) and against the table path on the same inputs, whose operator values
were rounded to FP32 from FP64: the two differ by a few FP32 ulps per
entry, far below either form's error.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import announce, parity, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

FORMS = [("split-bf16", 1e-4), ("split-fp16", 1e-4), ("fp16", 1e-3)]
BOX_TOL = {"split-bf16": 1e-4, "split-fp16": 1e-4, "fp16": 3e-3}
# generated against table: the operator values agree to FP32 rounding, so
# the products agree far below the forms' own error
TABLE_DIFF = {"split-bf16": 1e-5, "split-fp16": 1e-5, "fp16": 2e-4}

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()


def _translate(ff, P, nrhs):
    Pd = to_dev(P)
    Ed = torch.empty_like(Pd)
    U.translate(ff.plan, Pd, Ed, nrhs)
    return to_host(Ed)


@pytest.mark.parametrize("form,tol", FORMS)
@pytest.mark.parametrize("far_mode", ["ilist", "full"])
def test_generated_grid_against_oracle_and_table(form, tol, far_mode):
    w = W.config(1)
    announce("generated operators", w.name, far_mode, form)
    P = W.complex_normal((2, w.n_box, w.n_u), 61)
    gen = U.FarField(w.boxes, w.a, w.k, w.n_d, far_mode, max_nrhs=2, precision=form,
                     operators="generated")
    assert gen.info["operators"] == U.OPERATORS_GENERATED and gen.info["table_bytes"] == 0
    E = _translate(gen, P, 2)
    ref = O.translate(P.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode=far_mode)
    parity(E, ref, tol, boxes=w.n_u, box_tol=BOX_TOL[form], label=f"generated {far_mode} {form}")
    tab = U.FarField(w.boxes, w.a, w.k, w.n_d, far_mode, max_nrhs=2, precision=form)
    Et = _translate(tab, P, 2)
    d = rel_l2(E, Et)
    print(f"generated vs table ({far_mode}, {form}): {d:.2e}")
    assert d <= TABLE_DIFF[form]
    # deterministic
    assert np.array_equal(_translate(gen, P, 2), E)
    gen.close()
    tab.close()


@pytest.mark.parametrize("form,tol", FORMS)
@pytest.mark.parametrize("n_d,boxes", [(1, W.grid_boxes(5, 5, 5)), (2, W.grid_boxes(4, 4, 5))])
def test_generated_small_dipole_grids(form, tol, n_d, boxes):
    # n_d = 1 (one lattice difference) and 2 (27), on grids where FULL and
    # ILIST differ, a = lambda / 8
    announce("generated n_d", n_d, form)
    a, k = 0.125, 2 * np.pi
    P = W.complex_normal((1, len(boxes), 3 * n_d ** 3), 62 + n_d)
    ff = U.FarField(boxes, a, k, n_d, "full", precision=form, operators="generated")
    E = _translate(ff, P, 1)
    ref = O.translate(P.astype(np.complex128), boxes, a, k, n_d, mode="full")
    parity(E, ref, tol, boxes=3 * n_d ** 3, box_tol=BOX_TOL[form],
           label=f"generated n_d={n_d} {form}")
    ff.close()


def test_generated_low_frequency_regime():
    # a = lambda / 256: the 1/(kR)^2 terms dominate and the operators span
    # many binades; the in-kernel FP16 scale per offset must follow them
    announce("generated low frequency")
    boxes = W.grid_boxes(5, 5, 5)
    a, k = 1.0 / 256, 2 * np.pi
    P = W.complex_normal((1, len(boxes), 81), 64)
    ff = U.FarField(boxes, a, k, 3, "full", precision="split-fp16", operators="generated")
    E = _translate(ff, P, 1)
    ref = O.translate(P.astype(np.complex128), boxes, a, k, 3, mode="full")
    parity(E, ref, 1e-4, boxes=81, label="generated lambda/256")
    ff.close()


@pytest.mark.parametrize("nrhs", [1, 3])
def test_generated_schedules_same_bits(nrhs):
    # the chunk kernel at several grids and the walk over right-hand sides
    # give identical bits; the round kernels (which read a table) are refused
    w = W.config(2)
    announce("generated schedules", w.name, nrhs)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, max_nrhs=nrhs, precision="split-fp16",
                    operators="generated")
    x = to_dev(W.complex_normal((nrhs, ff.nb_total), 65))
    y0 = to_host(ff(x))
    for kernel, groups in [(U.TRANSLATE_CHUNKS, 256), (U.TRANSLATE_CHUNKS, 4096),
                           (U.TRANSLATE_CHUNKS_WALK, 512)]:
        ff.schedule(kernel, groups)
        assert np.array_equal(to_host(ff(x)), y0), (kernel, groups)
    for kernel in (U.TRANSLATE_ROUNDS, U.TRANSLATE_ROUNDS_DOUBLE):
        with pytest.raises(U.UbfError) as e:
            ff.schedule(kernel, 512)
        assert e.value.status == -1
    g = ff.tune(nrhs=nrhs, reps=2)
    assert ff.info["translate_kernel"] in (U.TRANSLATE_CHUNKS, U.TRANSLATE_CHUNKS_WALK)
    assert ff.info["translate_groups"] == g
    assert np.array_equal(to_host(ff(x)), y0)
    sample = np.sort(np.random.default_rng(66).choice(w.n_box, size=32, replace=False))
    P = x.cpu().numpy().reshape(nrhs, w.n_box, w.n_u).astype(np.complex128)
    ref = O.translate(P, w.boxes, w.a, w.k, w.n_d, test_boxes=sample)
    parity(y0.reshape(nrhs, w.n_box, w.n_u)[:, sample], ref[:, sample], 1e-4, boxes=w.n_u,
           label=f"generated shell nrhs {nrhs}")
    ff.close()


def test_generated_three_stages_benchmarked_shell():
    # the headline configuration (3,338-box shell, synthetic basis, split
    # FP16, tuned) with generated operators, element by element
    w = W.config(2)
    announce("generated three stages", w.name)
    nb = np.full(w.n_box, 81)
    nb_ptr, S = W.random_basis(nb, w.n_u, 67)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, precision="split-fp16", operators="generated")
    ff.set_basis(nb_ptr, to_dev(S))
    ff.tune(nrhs=1, reps=2)
    x = W.complex_normal((1, int(nb_ptr[-1])), 68)
    y = to_host(ff(to_dev(x)))
    ref = O.far_mvm(x.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, nb_ptr,
                    S.astype(np.complex128))
    parity(y, ref, 1e-4, boxes=nb_ptr, label="generated three stages")
    ff.close()


@pytest.mark.parametrize("precision", ["split-fp16", "fp16"])
def test_generated_full_far_set_shell_sampled(precision):
    # FULL far set of the 3,338-box shell (11.1M pairs, 148,018 offsets)
    # without any table: sampled test boxes against the oracle
    w = W.config(2, far_mode="full")
    announce("generated FULL shell", precision)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, "full", precision=precision,
                    operators="generated")
    assert ff.info["n_pairs"] == 11105714 and ff.info["table_bytes"] == 0
    P = w.coefficients(seed=69).reshape(1, w.n_box, w.n_u)
    E = _translate(ff, P, 1)
    ff.close()
    sample = np.sort(np.random.default_rng(70).choice(w.n_box, size=4, replace=False))
    ref = O.translate(P.astype(np.complex128), w.boxes, w.a, w.k, w.n_d, mode="full",
                      test_boxes=sample)
    tol = 1e-4 if precision == "split-fp16" else 1e-3
    parity(E[:, sample], ref[:, sample], tol, boxes=w.n_u,
           box_tol=BOX_TOL[precision], label=f"generated FULL {precision} sampled")


def test_generated_beyond_the_table_limit():
    # 1,500 boxes scattered in a 300^3 region, FULL far set: 2,248,500 pairs
    # over 2,221,706 distinct offsets, whose table (127 GB) is refused; with
    # generated operators the plan needs 1.8 GB and every chunk evaluates
    # its own operator. Sampled test boxes against the oracle.
    rng = np.random.default_rng(5)
    boxes = np.unique(rng.integers(0, 300, size=(1500, 3)), axis=0)
    a, k = 0.25, 2 * np.pi
    announce("generated beyond the table limit", len(boxes))
    with pytest.raises(U.UbfError) as e:
        U.plan_create(boxes, a, k, 3, "full", precision="split-fp16")
    assert "16 GiB" in str(e.value)
    ff = U.FarField(boxes, a, k, 3, "full", precision="split-fp16", operators="generated")
    assert ff.info["n_pairs"] == len(boxes) * (len(boxes) - 1)
    assert ff.info["n_offsets"] > 2_000_000
    P = W.complex_normal((1, len(boxes), 81), 71)
    E = _translate(ff, P, 1)
    ff.close()
    sample = np.array([3, 777, 1234])
    ref = O.translate(P.astype(np.complex128), boxes, a, k, 3, mode="full", test_boxes=sample)
    parity(E[:, sample], ref[:, sample], 1e-4, boxes=81, label="generated beyond the table limit")
