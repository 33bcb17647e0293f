"""Host checks of the network training helpers (no GPU): orbit
representatives, the DOF symmetry against the library's own FP64 operators,
the expansion of orbit networks to a plan's offsets, and a tiny training run.
"""
import numpy as np
import pytest

import paper_2501_04684_amd as U
from paper_2501_04684_amd import training as T

A, K = 0.125, 2 * np.pi


def _linear(G):
    n = G.shape[1]
    I = np.eye(n)
    return {"W1": np.vstack([I, -I]), "b1": np.zeros(2 * n), "W2": np.hstack([G, -G]),
            "b2": np.zeros(G.shape[0])}


def _forward(net, v):
    z = net["W1"] @ v + net["b1"]
    return net["W2"] @ (np.maximum(z.real, 0) + 1j * np.maximum(z.imag, 0)) + net["b2"]


def test_sixteen_orbits_among_316_vectors():
    offs = T.interaction_list_offsets()
    assert len(offs) == 316
    reps = set()
    for w in offs:
        r, M = T.representative(w)
        assert np.array_equal(M @ np.array(r), w)
        assert np.array_equal(np.abs(M).sum(0), [1, 1, 1]) and np.array_equal(np.abs(M).sum(1), [1, 1, 1])
        reps.add(r)
    assert len(reps) == 16          # the count printed in Sec. 2.2
    assert len(T.cube_symmetries()) == 48


@pytest.mark.parametrize("n_d", [2, 3, 4])
def test_dof_symmetry_against_library_operators(n_d):
    offs = T.interaction_list_offsets()[::23]
    ops = T.operators_for(np.vstack([offs] + [np.array(T.representative(w)[0])[None]
                                              for w in offs]), A, K, n_d)
    for w in offs:
        r, M = T.representative(w)
        Pi = T.dof_permutation(M, n_d)
        assert np.allclose(Pi @ Pi.T, np.eye(3 * n_d ** 3))
        Gw, Gr = ops[tuple(int(c) for c in w)], ops[r]
        assert np.linalg.norm(Gw - Pi @ Gr @ Pi.T) <= 1e-12 * np.linalg.norm(Gw)


def test_expansion_to_plan_offsets():
    n_d = 2
    boxes = np.indices((6, 6, 3)).reshape(3, -1).T.astype(np.int32)
    plan = U.plan_create(boxes, A, K, n_d, "ilist")
    try:
        offs = U.plan_offsets(plan)
        reps = sorted({T.representative(w)[0] for w in offs})
        ops = T.operators_for(np.array(reps), A, K, n_d)
        nets = {r: _linear(ops[r]) for r in reps}
        W1, b1, W2, b2 = T.networks_for_plan(plan, nets, n_d)
        assert W1.shape == (len(offs), 48, 24) and W2.shape == (len(offs), 24, 48)
        rng = np.random.default_rng(0)
        for o in range(0, len(offs), 7):
            v = rng.standard_normal(24) + 1j * rng.standard_normal(24)
            out = _forward({"W1": W1[o], "b1": b1[o], "W2": W2[o], "b2": b2[o]}, v)
            ref = U.plan_operator(plan, o) @ v
            assert np.linalg.norm(out - ref) <= 1e-5 * np.linalg.norm(ref)
    finally:
        U.plan_destroy(plan)


def test_tiny_training_run(tmp_path):
    pytest.importorskip("torch")
    G = T.operators_for(np.array([[2, 0, 0]]), A, K, 1)[(2, 0, 0)]
    net = T.train_network(G, hidden=8, epochs=30, n_train=2000, n_test=200, seed=1)
    assert net["W1"].shape == (8, 3) and net["W2"].shape == (3, 8)
    assert net["W1"].dtype == np.complex64
    assert np.isfinite(net["err_mean"]) and net["err_mean"] < 0.5
    T.save(str(tmp_path / "n.npz"), {(2, 0, 0): net}, {"a": A, "k": K, "n_d": 1, "hidden": 8,
                                                      "epochs": 30})
    nets, meta = T.load(str(tmp_path / "n.npz"))
    assert meta["hidden"] == 8 and np.array_equal(nets[(2, 0, 0)]["W2"], net["W2"])
