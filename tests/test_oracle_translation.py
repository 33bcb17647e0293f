"""Pins of the translation operators (Eq. 12-13) and the translation sum (Eq. 14)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

A, K = 0.25, 2 * np.pi


@pytest.mark.parametrize("n_d", [1, 2, 3])
def test_reciprocity(n_d):
    # G(r, r') = G(r', r)^T: the operator of -w is the transpose of that of w
    rng = np.random.default_rng(0)
    for _ in range(6):
        w = rng.integers(-3, 4, size=3)
        if np.abs(w).max() < 2:
            continue
        G = O.translation_operator(w, A, K, n_d)
        Gm = O.translation_operator(-w, A, K, n_d)
        assert np.linalg.norm(Gm - G.T) <= 1e-14 * np.linalg.norm(G)


@pytest.mark.parametrize("n_d", [2, 3])
def test_cube_symmetries(n_d):
    # G_{Mw} = Pi_M G_w Pi_M^T for all 48 rotations/mirrors (Sec. 2.2)
    for w in ([2, 0, 0], [3, 2, 1], [2, 2, -3]):
        w = np.array(w)
        G = O.translation_operator(w, A, K, n_d)
        for M in O.symmetry.cube_group():
            Pi = O.symmetry.dof_permutation(M, n_d)
            Gs = O.translation_operator(M @ w, A, K, n_d)
            assert np.linalg.norm(Gs - Pi @ G @ Pi.T) <= 1e-13 * np.linalg.norm(G)


def test_operator_entry_is_dipole_field():
    # one entry against Eq. (12) with absolute positions of the two dipoles
    n_d = 3
    w = np.array([2, -1, 3])
    G = O.translation_operator(w, A, K, n_d)
    sites = O.site_offsets(A, n_d)
    rng = np.random.default_rng(4)
    for _ in range(20):
        l, s = rng.integers(0, 27, size=2)
        al, be = rng.integers(0, 3, size=2)
        src_c, tst_c = np.array([5, 5, 5]), np.array([5, 5, 5]) + w
        rt = O.box_centres(tst_c[None], A)[0] + sites[l]
        rs = O.box_centres(src_c[None], A)[0] + sites[s]
        D = O.dyadic_green(rt - rs, K)
        assert np.isclose(G[3 * l + al, 3 * s + be], D[al, be], rtol=1e-14, atol=0)


def test_site_layout():
    s = O.site_offsets(1.0, 3)
    assert s.shape == (27, 3)
    # uniform lattice of spacing a/n_d, centred on the box, inside it
    assert np.allclose(s[0], [-1 / 3, -1 / 3, -1 / 3])
    assert np.allclose(s[13], [0, 0, 0])
    assert np.allclose(s[1] - s[0], [0, 0, 1 / 3])      # z fastest
    assert np.allclose(s[9] - s[0], [1 / 3, 0, 0])      # x slowest
    assert np.abs(s).max() < 0.5


@pytest.mark.parametrize("boxes,n_d,mode", [
    (W.grid_boxes(2, 2, 4), 2, "ilist"),
    (W.grid_boxes(2, 2, 4), 2, "full"),
    (W.grid_boxes(4, 4, 4), 1, "ilist"),
    (W.mask_boxes(24, 0.5, 11), 2, "ilist"),
])
def test_grouped_equals_bruteforce(boxes, n_d, mode):
    n_u = 3 * n_d ** 3
    P = W.complex_normal((2, len(boxes), n_u), 5, np.complex128)
    Eg = O.translate(P, boxes, A, K, n_d, mode)
    Eb = O.translate_bruteforce(P, boxes, A, K, n_d, mode)
    assert np.linalg.norm(Eg - Eb) <= 1e-13 * np.linalg.norm(Eb)


def test_grouped_equals_bruteforce_nd3_small():
    boxes = np.array([[0, 0, 0], [0, 0, 2], [3, 1, 0], [2, 3, 3]])
    P = W.complex_normal((1, 4, 81), 6, np.complex128)
    Eg = O.translate(P, boxes, A, K, 3, "full")
    Eb = O.translate_bruteforce(P, boxes, A, K, 3, "full")
    assert np.linalg.norm(Eg - Eb) <= 1e-13 * np.linalg.norm(Eb)


def test_far_operator_complex_symmetric():
    # block (j,i) = G_{c_j - c_i}, block (i,j) = its transpose: u^T Z v = v^T Z u
    boxes = W.grid_boxes(4, 4, 4)
    u = W.complex_normal((1, 64, 24), 7, np.complex128)
    v = W.complex_normal((1, 64, 24), 8, np.complex128)
    Zv = O.translate(v, boxes, A, K, 2)
    Zu = O.translate(u, boxes, A, K, 2)
    lhs = np.sum(u * Zv)
    rhs = np.sum(v * Zu)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_linearity_and_empty():
    boxes = W.grid_boxes(3, 3, 3)
    P1 = W.complex_normal((1, 27, 24), 1, np.complex128)
    P2 = W.complex_normal((1, 27, 24), 2, np.complex128)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    E = O.translate(a * P1 + b * P2, boxes, A, K, 2)
    E12 = a * O.translate(P1, boxes, A, K, 2) + b * O.translate(P2, boxes, A, K, 2)
    assert np.linalg.norm(E - E12) <= 1e-13 * np.linalg.norm(E)
    # two adjacent boxes: no far pair, field is exactly zero
    adj = np.array([[0, 0, 0], [1, 1, 1]])
    E = O.translate(W.complex_normal((1, 2, 24), 3, np.complex128), adj, A, K, 2)
    assert not E.any()
