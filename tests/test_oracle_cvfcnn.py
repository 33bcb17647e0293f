"""Pins of the network translation (Sec. 3, Fig. 5) in the oracle."""
import numpy as np
import pytest

import oracle as O
from oracle import cvfcnn as C

A, K = 0.25, 2 * np.pi


def _linear_net(G):
    # W1 = [I; -I], W2 = [G, -G], no biases: since CReLU(v) - CReLU(-v) = v
    # component by component, the network computes G v exactly.
    n = G.shape[1]
    I = np.eye(n)
    return (np.vstack([I, -I]), np.zeros(2 * n), np.hstack([G, -G]), np.zeros(G.shape[0]))


def _cplx(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_crelu_hand_values():
    z = np.array([1 + 2j, -1 + 2j, 1 - 2j, -1 - 2j, 0, -0.5j])
    assert np.array_equal(C.crelu(z), np.array([1 + 2j, 2j, 1, 0, 0, 0]))


def test_linf_is_largest_modulus():
    assert C.linf(np.array([3 + 4j, -1, 2j])) == 5.0
    assert np.array_equal(C.linf(np.array([[1j, -2], [0, 0]])), [2.0, 0.0])


def test_worked_constant_network():
    # W1 = 0: the hidden layer is CReLU(b1) = [1+1j, 2j]; with W2 = [[1, 1],
    # [2j, 0]] and b2 = [0.5, -1j] the network outputs [1.5+3j, -2+1j] for any
    # input, and the contribution of P is ||P||_inf times that.
    net = (np.zeros((2, 3)), np.array([1 + 1j, -1 + 2j]),
           np.array([[1, 1], [2j, 0], [0, 0]]), np.array([0.5, -1j, 0]))
    P = np.array([[0.3, -4j, 1 + 1j]])
    out = C.apply_network(net, P)
    assert np.allclose(out, 4.0 * np.array([[1.5 + 3j, -2 + 1j, 0]]), rtol=0, atol=1e-15)


def test_zero_box_vector_contributes_nothing():
    rng = np.random.default_rng(1)
    net = (_cplx(rng, 5, 6), _cplx(rng, 5), _cplx(rng, 6, 5), _cplx(rng, 6))
    out = C.apply_network(net, np.zeros((3, 6), dtype=complex))
    assert np.array_equal(out, np.zeros((3, 6)))


def test_positive_homogeneity_without_biases():
    # without biases f(c v) = c f(v) for real c > 0, so the l-inf scaling
    # cancels and the contribution is f(P) itself
    rng = np.random.default_rng(2)
    net = (_cplx(rng, 7, 6), np.zeros(7), _cplx(rng, 6, 7), np.zeros(6))
    P = _cplx(rng, 4, 6)
    ref = C.network_forward(net, P)
    assert np.allclose(C.apply_network(net, P), ref, rtol=1e-14, atol=0)
    assert np.allclose(C.network_forward(net, 3.5 * P), 3.5 * ref, rtol=1e-14, atol=0)
    # with a bias the scaling matters
    net_b = (net[0], _cplx(rng, 7), net[2], net[3])
    assert not np.allclose(C.apply_network(net_b, P), C.network_forward(net_b, P))


@pytest.mark.parametrize("boxes,n_d,mode", [
    (np.array([[x, y, z] for x in range(4) for y in range(4) for z in range(2)]), 2, "ilist"),
    (np.array([[x, y, z] for x in range(3) for y in range(3) for z in range(3)]), 1, "full"),
    (np.array([[x, y, z] for x in range(4) for y in range(4) for z in range(4)
               if (x + y + z) % 3]), 2, "ilist"),
])
def test_linear_networks_reproduce_dgfa(boxes, n_d, mode):
    # the network translation with the exact linear networks is the DGFA
    # translation (Eq. 13-14), which is pinned by brute force and closed forms
    rng = np.random.default_rng(3)
    n_u = 3 * n_d ** 3
    j, i, w = O.far_pairs(boxes, mode)
    uniq, _ = O.offset_ids(w)
    nets = {tuple(int(c) for c in wv): _linear_net(O.translation_operator(wv, A, K, n_d))
            for wv in uniq}
    P = _cplx(rng, 2, len(boxes), n_u)
    P[1, 3] = 0                                           # a zero box vector
    E_net = C.translate_cvfcnn(P, boxes, nets, mode)
    E_ref = O.translate(P, boxes, A, K, n_d, mode)
    assert np.linalg.norm(E_net - E_ref) <= 1e-13 * np.linalg.norm(E_ref)


def test_transposed_network_is_caught():
    # G_w is not symmetric, so a network built from G_w^T must not match:
    # guards the orientation of W1/W2 in the forward pass
    n_d = 2
    w = np.array([2, 1, 0])
    G = O.translation_operator(w, A, K, n_d)
    assert np.linalg.norm(G - G.T) > 1e-3 * np.linalg.norm(G)
    rng = np.random.default_rng(5)
    v = _cplx(rng, 24)
    assert np.allclose(C.network_forward(_linear_net(G), v), G @ v, rtol=1e-14, atol=0)
    assert not np.allclose(C.network_forward(_linear_net(G.T), v), G @ v)


@pytest.mark.parametrize("n_d", [2, 3])
def test_symmetry_map_of_networks(n_d):
    # the network of M w obtained from the network of w by the signed DOF
    # permutation computes the operator of M w evaluated directly
    rng = np.random.default_rng(6)
    w = np.array([3, 2, 1])
    net = _linear_net(O.translation_operator(w, A, K, n_d))
    v = _cplx(rng, 3, 3 * n_d ** 3)
    for M in O.symmetry.cube_group()[::5]:
        Pi = O.symmetry.dof_permutation(M, n_d)
        mapped = C.permuted_network(net, Pi)
        Gs = O.translation_operator(M @ w, A, K, n_d)
        out = C.network_forward(mapped, v)
        assert np.linalg.norm(out - v @ Gs.T) <= 1e-13 * np.linalg.norm(v @ Gs.T)


def test_relative_error_definition():
    E = np.array([[3.0, 4.0j], [1.0, 0.0]])
    O_ = np.array([[3.0, 4.0j + 0.5], [1.0, 0.25j]])
    assert np.allclose(C.relative_error(O_, E), [0.1, 0.25], rtol=1e-15, atol=0)
