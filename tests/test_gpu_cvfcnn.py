"""Parity of the network translation (Sec. 3, Fig. 5) with the FP64 oracle.

Both sides take the same complex64 weights, biases and inputs (upcast to
complex128 in the oracle). The GPU runs both layers in FP32: matrix-core
products with FP32 accumulation over 2 N_u (layer 1) and 2 HP (layer 2)
terms, the l-inf norm in FP32. Each layer adds a relative error of about
sqrt(K) 2^-24 (below 1e-6 for K <= 384), CReLU is 1-Lipschitz and the
per-pair contributions add in FP32 in stage 3, so the relative l2 error of
the whole product stays below 1e-5, the bar used here. Exact linear networks
(W1 = [I; -I], W2 = [G_w, -G_w], which compute G_w v) must reproduce the
operator-table product within the FP32 bar of 1e-4.
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import announce, parity, to_dev, to_host
from oracle import cvfcnn as C

pytestmark = pytest.mark.gpu
TOL = 1e-5
TOL_FP32 = 1e-4

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()


def _nets(offsets, W1, b1, W2, b2):
    return {tuple(int(c) for c in offsets[o]): (W1[o], b1[o], W2[o], b2[o])
            for o in range(len(offsets))}


def _field(boxes, a, k, n_d, mode, hidden, seed, max_nrhs=1):
    ff = U.FarField(boxes, a, k, n_d, mode, max_nrhs=max_nrhs)
    offs = U.plan_offsets(ff.plan)
    weights = W.random_networks(len(offs), hidden, 3 * n_d ** 3, seed)
    ff.set_networks(*weights)
    return ff, _nets(offs, *weights)


# 1 and 7: widths that are not a multiple of the four hidden units of one
# k group; 33: the first width of the 64-unit image
@pytest.mark.parametrize("hidden", [1, 7, 16, 33, 50, 64])
def test_identity_basis_config1(hidden):
    w = W.config(1, nrhs=2)
    announce("cvfcnn identity basis", w.name, "hidden", hidden)
    ff, nets = _field(w.boxes, w.a, w.k, w.n_d, w.far_mode, hidden, seed=7, max_nrhs=2)
    x = w.coefficients()
    x[1, 5 * w.n_u:6 * w.n_u] = 0                      # a zero box vector
    y = to_host(ff(to_dev(x)))
    P = x.reshape(2, w.n_box, w.n_u).astype(np.complex128)
    ref = C.translate_cvfcnn(P, w.boxes, nets, w.far_mode).reshape(2, -1)
    parity(y, ref, TOL, boxes=w.n_u, label=f"networks hidden {hidden}")
    ff.close()


def test_three_stages_synthetic_basis_config1():
    w = W.config(1)
    announce("cvfcnn synthetic basis", w.name)
    ff, nets = _field(w.boxes, w.a, w.k, w.n_d, w.far_mode, 50, seed=11)
    nb = np.full(w.n_box, w.n_u)
    nb_ptr, S = W.random_basis(nb, w.n_u, seed=3)
    S_dev = to_dev(S)
    ff.set_basis(nb_ptr, S_dev)
    x = w.coefficients(int(nb_ptr[-1]))
    y = to_host(ff(to_dev(x)))
    P = O.aggregate(x.astype(np.complex128), nb_ptr, S.astype(np.complex128), w.n_u)
    E = C.translate_cvfcnn(P, w.boxes, nets, w.far_mode)
    ref = O.disaggregate(E, nb_ptr, S.astype(np.complex128))
    parity(y, ref, TOL, boxes=nb_ptr, label="networks, three stages")
    ff.close()


@pytest.mark.parametrize("hidden", [33, 50, 64])
def test_nd4_paper_shape(hidden):
    # 3 N_d = 192 inputs (box vectors staged in two k passes), 50 hidden units
    # as in the paper's networks and the edges of the 64-unit image; FULL =
    # ILIST on a 4^3 grid plus a ragged 4x4x5 grid
    for boxes in (W.grid_boxes(4, 4, 4), W.grid_boxes(4, 4, 5)):
        announce("cvfcnn n_d=4", len(boxes), "hidden", hidden)
        ff, nets = _field(boxes, 0.125, 2 * np.pi, 4, "ilist", hidden, seed=5)
        x = W.complex_normal((1, len(boxes) * 192), seed=9)
        y = to_host(ff(to_dev(x)))
        P = x.reshape(1, len(boxes), 192).astype(np.complex128)
        ref = C.translate_cvfcnn(P, boxes, nets, "ilist").reshape(1, -1)
        parity(y, ref, TOL, boxes=192, label=f"networks n_d=4 {len(boxes)} boxes, hidden {hidden}")
        ff.close()


@pytest.mark.parametrize("networks", [True, False])
def test_nd4_degenerate_and_single_pair(networks):
    # 192 coefficients per box, networks or the operator table staged in
    # LDS: no far pair (one box; two adjacent boxes) gives zero, also with
    # stage timing on; one far pair gives its single product
    k = 2 * np.pi
    for boxes in (np.array([[3, 3, 3]]), np.array([[0, 0, 0], [1, 1, 1]]),
                  np.array([[0, 0, 0], [0, 0, 2]])):
        announce("n_d=4 degenerate", boxes.tolist(), "networks", networks)
        if networks:
            ff, nets = _field(boxes, 0.125, k, 4, "ilist", 50, seed=11)
        else:
            ff = U.FarField(boxes, 0.125, k, 4, "ilist")
        # one item per offset here (each offset holds a single pair)
        assert ff.info["n_items"] == len(U.plan_offsets(ff.plan))
        x = W.complex_normal((1, len(boxes) * 192), seed=13)
        U.profile_begin(ff.plan, 2, 1)
        y = to_host(ff(to_dev(x)))
        torch.cuda.synchronize()
        _, calls = U.profile_end(ff.plan, 2)
        assert len(calls) == 1
        P = x.reshape(1, len(boxes), 192).astype(np.complex128)
        if ff.info["n_pairs"] == 0:
            assert not np.any(y)
        else:
            ref = (C.translate_cvfcnn(P, boxes, nets, "ilist") if networks
                   else O.translate(P, boxes, 0.125, k, 4))
            parity(y, ref.reshape(1, -1), TOL if networks else TOL_FP32, boxes=192,
                   label=f"single pair, networks {networks}")
        ff.close()


def test_linear_networks_reproduce_operator_table():
    # n_d = 2: W1 = [I; -I] and W2 = [G_w, -G_w] fit in 48 hidden units
    boxes = W.grid_boxes(6, 6, 4)
    a, k, n_d = 0.25, 2 * np.pi, 2
    announce("cvfcnn linear networks", len(boxes))
    ff = U.FarField(boxes, a, k, n_d, "ilist")
    x = W.complex_normal((1, len(boxes) * 24), seed=12)
    xd = to_dev(x)
    y_table = to_host(ff(xd)).copy()
    offs = U.plan_offsets(ff.plan)
    I = np.eye(24)
    W1 = np.stack([np.vstack([I, -I])] * len(offs)).astype(np.complex64)
    G = np.stack([O.translation_operator(wv, a, k, n_d) for wv in offs])
    W2 = np.concatenate([G, -G], axis=2).astype(np.complex64)
    ff.set_networks(W1, np.zeros((len(offs), 48), np.complex64), W2,
                    np.zeros((len(offs), 24), np.complex64))
    y_net = to_host(ff(xd))
    ref = O.translate(x.reshape(1, len(boxes), 24).astype(np.complex128), boxes, a, k, n_d,
                      "ilist").reshape(1, -1)
    parity(y_net, ref, TOL_FP32, boxes=24, label="linear networks vs oracle")
    parity(y_net, y_table, TOL_FP32, boxes=24, label="linear networks vs operator table")
    # back to the operator table: the same result as before, bit for bit
    ff.set_networks()
    assert np.array_equal(to_host(ff(xd)), y_table)
    ff.close()


def test_shell3338_full_size():
    # the 3,338-box shell: 108,888 pairs over 316 offsets, whole output
    w = W.config(2)
    announce("cvfcnn full size", w.name)
    ff, nets = _field(w.boxes, w.a, w.k, w.n_d, w.far_mode, 50, seed=21)
    x = w.coefficients()
    y = to_host(ff(to_dev(x)))
    P = x.reshape(1, w.n_box, w.n_u).astype(np.complex128)
    ref = C.translate_cvfcnn(P, w.boxes, nets, w.far_mode).reshape(1, -1)
    parity(y, ref, TOL, boxes=w.n_u, label=f"networks {w.name}")
    ff.close()


def test_sphere762_nd4_full_size_trained_networks():
    # the network workload as bench.py times it: the 762-box sphere at
    # a = 0.125 with the committed trained networks (16 orbit networks
    # expanded to the 316 offsets), all 22,602 pairs, two right-hand sides
    from paper_2501_04684_amd import training as T
    path = os.path.join(os.path.dirname(U.__file__), "data", "networks_nd4_h50_a0.125.npz")
    w = W.config(6, nrhs=2)
    announce("cvfcnn trained networks", w.name)
    orbit, meta = T.load(path)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, max_nrhs=2)
    offs = U.plan_offsets(ff.plan)
    weights = T.networks_for_plan(ff.plan, orbit, w.n_d)
    ff.set_networks(*weights)
    x = w.coefficients()
    y = to_host(ff(to_dev(x)))
    P = x.reshape(2, w.n_box, w.n_u).astype(np.complex128)
    ref = C.translate_cvfcnn(P, w.boxes, _nets(offs, *weights), w.far_mode).reshape(2, -1)
    parity(y, ref, TOL, boxes=w.n_u, label=f"{w.name} trained networks")
    ff.close()


def test_graph_replay_matches_eager():
    w = W.config(1)
    announce("cvfcnn graph replay", w.name)
    ff, _ = _field(w.boxes, w.a, w.k, w.n_d, w.far_mode, 50, seed=3)
    x = to_dev(w.coefficients())
    y_eager = to_host(ff(x)).copy()
    y = torch.empty_like(x)
    ff.capture(x, y)
    for _ in range(3):
        ff.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), y_eager)
        y.zero_()
        torch.cuda.synchronize()
    ff.close()


def test_rejected_forms():
    w = W.config(1)
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode, precision="split-fp16")
    n_off = ff.info["n_offsets"]
    weights = W.random_networks(n_off, 8, w.n_u, seed=1)
    with pytest.raises(U.UbfError) as e:
        ff.set_networks(*weights)
    assert "FP32" in str(e.value)
    ff.close()
    ff = U.FarField(w.boxes, w.a, w.k, w.n_d, w.far_mode)
    with pytest.raises(ValueError):
        ff.set_networks(*W.random_networks(n_off - 1, 8, w.n_u, seed=1))
    ff.close()
