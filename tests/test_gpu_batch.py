"""Batching several scatterers in one plan (needs a GPU).

A batched plan must give, for every scatterer, what a plan of that
scatterer alone gives (bit for bit: the per-pair arithmetic and the order of
the per-test-box sums are the same) and must match the FP64 oracle of that
scatterer to 1e-4. The captured HIP graph must reproduce the eager call, and
the stage-2 autotuner must not change any result.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import announce, parity, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-4
A, K = 0.25, 2 * np.pi

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()


def _small_parts():
    return [b for _, b in W.scatterer_set(6, seed=11, lo=40, hi=300)]


def _slices(parts, n_u):
    base = 0
    for b in parts:
        yield b, slice(base * n_u, (base + len(b)) * n_u)
        base += len(b)


@pytest.mark.parametrize("precision", ["fp32", "split-bf16"])
def test_small_batch_matches_oracle_and_solo(precision):
    parts = _small_parts()
    announce("small batch", precision, [len(b) for b in parts])
    ff = U.FarField(None, A, K, 3, max_nrhs=2, precision=precision, scatterers=parts)
    assert ff.info["n_scatterers"] == len(parts)
    n = sum(len(b) for b in parts) * 81
    x = W.complex_normal((2, n), 21)
    xd = to_dev(x)
    y = to_host(ff(xd))
    for b, sl in _slices(parts, 81):
        ref = O.far_mvm(x[:, sl].astype(np.complex128), b, A, K, 3)
        parity(y[:, sl], ref, TOL, boxes=81, label=f"{precision} scatterer of {len(b)} boxes")
        solo = U.FarField(b, A, K, 3, max_nrhs=2, precision=precision)
        ys = to_host(solo(xd[:, sl].contiguous()))
        assert np.array_equal(ys, y[:, sl])
        solo.close()


def test_batch_with_basis_matches_solo():
    parts = _small_parts()[:4]
    announce("small batch with basis", [len(b) for b in parts])
    nb = np.concatenate([np.random.default_rng(3).integers(0, 100, len(b)) for b in parts])
    nb_ptr, S = W.random_basis(nb, 81, 31)
    ff = U.FarField(None, A, K, 3, scatterers=parts)
    Sd = to_dev(S)
    ff.set_basis(nb_ptr, Sd)
    x = W.complex_normal((1, int(nb_ptr[-1])), 32)
    y = to_host(ff(to_dev(x)))
    ref_all = []
    base = 0
    for b in parts:
        lo, hi = nb_ptr[base], nb_ptr[base + len(b)]
        sub_ptr = nb_ptr[base:base + len(b) + 1] - lo
        S_sub = S[81 * lo:81 * hi]
        ref = O.far_mvm(x[:, lo:hi].astype(np.complex128), b, A, K, 3, sub_ptr,
                        S_sub.astype(np.complex128))
        parity(y[:, lo:hi], ref, TOL, boxes=sub_ptr, label=f"basis scatterer of {len(b)} boxes")
        solo = U.FarField(b, A, K, 3)
        S_dev = to_dev(S_sub)
        solo.set_basis(sub_ptr, S_dev)
        assert np.array_equal(to_host(solo(to_dev(x[:, lo:hi]))), y[:, lo:hi])
        solo.close()
        ref_all.append(ref)
        base += len(b)


def test_graph_replay_matches_eager():
    parts = _small_parts()
    announce("graph replay")
    ff = U.FarField(None, A, K, 3, max_nrhs=2, scatterers=parts)
    n = ff.nb_total
    x1 = to_dev(W.complex_normal((2, n), 41))
    x2 = to_dev(W.complex_normal((2, n), 42))
    y1 = to_host(ff(x1))
    y2 = to_host(ff(x2))
    xg = x1.clone()
    yg = torch.empty_like(xg)
    ff.capture(xg, yg)
    for rep in range(3):
        yg.zero_()
        ff.replay()
        assert np.array_equal(to_host(yg), y1), rep
        # eager use of the same plan between replays
        assert np.array_equal(to_host(ff(x2)), y2)
    xg.copy_(x2)              # the graph reads whatever xg holds at launch
    ff.replay()
    assert np.array_equal(to_host(yg), y2)
    ff.set_basis(None)        # discards the graph
    with pytest.raises(U.UbfError) as e:
        ff.replay()
    assert e.value.status == -4


@pytest.mark.parametrize("precision", ["fp32", "split-bf16", "split-fp16", "fp16"])
def test_tune_keeps_results(precision):
    w = W.config(2)
    announce("tune", w.name, precision)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, max_nrhs=2, precision=precision)
    x = to_dev(w.coefficients(seed=7))
    y0 = to_host(ff(x))
    g = ff.tune(nrhs=1, reps=3)
    assert g in (256, 512, 1024, 2048, 4096) or g <= ff.info["n_chunks"] + 7
    assert ff.info["translate_groups"] == g
    y1 = to_host(ff(x))
    assert np.array_equal(y0, y1)


@pytest.mark.parametrize("precision", ["split-fp16", "split-bf16", "fp16"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_every_stage2_schedule_gives_the_same_bits(precision, nrhs):
    # every kernel and grid the tuner may choose computes each column with
    # the same products in the same order: results agree bit for bit, and
    # with the oracle (sampled test boxes)
    w = W.config(2)
    announce("schedules", w.name, precision, "nrhs", nrhs)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, max_nrhs=nrhs, precision=precision)
    x = W.complex_normal((nrhs, ff.nb_total), 17)
    xd = to_dev(x)
    y0 = to_host(ff(xd))
    assert ff.info["translate_kernel"] == U.TRANSLATE_CHUNKS
    seen = []
    for kernel, groups in [(U.TRANSLATE_CHUNKS, 256), (U.TRANSLATE_CHUNKS, 4096),
                           (U.TRANSLATE_CHUNKS_WALK, 512), (U.TRANSLATE_ROUNDS, 512),
                           (U.TRANSLATE_ROUNDS, 1024), (U.TRANSLATE_ROUNDS_DOUBLE, 256),
                           (U.TRANSLATE_ROUNDS_DOUBLE, 8)]:
        ff.schedule(kernel, groups)
        assert ff.info["translate_kernel"] == kernel
        y = to_host(ff(xd))
        assert np.array_equal(y, y0), (kernel, groups)
        seen.append((kernel, ff.info["translate_groups"]))
    assert len(set(seen)) == len(seen)
    sample = np.sort(np.random.default_rng(3).choice(w.n_box, size=40, replace=False))
    P = x.reshape(nrhs, w.n_box, w.n_u).astype(np.complex128)
    ref = O.translate(P, w.boxes, w.a, w.k, w.n_d, test_boxes=sample)
    parity(y0.reshape(nrhs, w.n_box, w.n_u)[:, sample], ref[:, sample],
           1e-4 if precision != "fp16" else 1e-3, boxes=w.n_u,
           box_tol=1e-4 if precision != "fp16" else 3e-3, label=f"schedules {precision}")
    with pytest.raises(U.UbfError):
        ff.schedule(7, 512)
    ff.close()


def test_fp32_plan_has_only_the_chunk_kernel():
    w = W.config(1)
    announce("fp32 schedule")
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d)
    ff.schedule(U.TRANSLATE_CHUNKS, 256)
    assert ff.info["translate_groups"] <= 256
    with pytest.raises(U.UbfError) as e:
        ff.schedule(U.TRANSLATE_ROUNDS, 512)
    assert e.value.status == -1
    ff.close()


def test_tune_cache_is_reused(tmp_path, monkeypatch):
    w = W.config(2)
    announce("tune cache", w.name)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("UBF_TUNE_CACHE", str(cache))
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, max_nrhs=1, precision="split-fp16")
    x = to_dev(W.complex_normal((1, ff.nb_total), 5))
    y0 = to_host(ff(x))
    g = ff.tune(nrhs=1, reps=2)
    kernel = ff.info["translate_kernel"]
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[1].split()[:2] == [str(kernel), str(g)]
    # a second plan of the same statistics takes the cached schedule
    ff2 = U.FarField(w.boxes, w.a, w.k, w.n_d, max_nrhs=1, precision="split-fp16")
    assert ff2.tune(nrhs=1, reps=2) == g and ff2.info["translate_kernel"] == kernel
    assert len(cache.read_text().splitlines()) == 1
    assert np.array_equal(to_host(ff2(x)), y0)
    ff.close()
    ff2.close()


def test_batch64_full_size_against_solo_and_oracle():
    """64 scatterers (200 to 20k boxes), 4 right-hand sides, split precision,
    tuned and replayed from a graph: the benchmarked batch."""
    w = W.config(4)
    parts = w.extra["scatterers"]
    announce("batch64 full size", w.n_box)
    ff = U.FarField(None, w.a, w.k, w.n_d, max_nrhs=4, precision="split-bf16",
                    scatterers=parts)
    ff.tune(nrhs=4, reps=2)
    x = w.coefficients()
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    ff.capture(xd, yd)
    ff.replay()
    y = to_host(yd)
    assert np.isfinite(y).all()
    for s, (b, sl) in enumerate(_slices(parts, 81)):
        solo = U.FarField(b, w.a, w.k, w.n_d, max_nrhs=4, precision="split-bf16")
        ys = to_host(solo(xd[:, sl].contiguous()))
        assert np.array_equal(ys, y[:, sl]), s
        solo.close()
        del solo
    rng = np.random.default_rng(44)
    picks = [0, 1, 2, 3] + [int(i) for i in np.argsort([len(b) for b in parts])[-4:]]
    for s in picks:
        b, sl = list(_slices(parts, 81))[s]
        sample = np.sort(rng.choice(len(b), size=min(6, len(b)), replace=False))
        P = x[:, sl].reshape(4, len(b), 81).astype(np.complex128)
        ref = O.translate(P, b, w.a, w.k, w.n_d, test_boxes=sample)
        got = y[:, sl].reshape(4, len(b), 81)
        parity(got[:, sample], ref[:, sample], TOL, boxes=81, label=f"batch64 scatterer {s}")
