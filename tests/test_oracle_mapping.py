"""Pins of the uniform-basis mapping (Sec. 2.1) and inverse mapping (Sec. 2.3)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import mapping as M

A, K, ND = 0.25, 2 * np.pi, 3
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_constants():
    ref = json.load(open(os.path.join(GOLDEN, "sec2_paper_constants.json")))
    pts = M.sample_points(A, ND)
    assert len(pts) == ref["n_s_over_n_d"] * ND ** 3
    assert np.allclose(np.linalg.norm(pts, axis=1), ref["sphere_radius_over_a"] * A)
    Am = M.A_matrix(A, K, ND)
    assert Am.shape == (3 * len(pts), ref["n_u_over_n_d"] * ND ** 3)
    assert 3 * 4 ** 3 == ref["dofs_4x4x4"]


def test_fibonacci_lattice_structure():
    n = 54
    p = M.fibonacci_points(n, 1.0)
    z = np.sort(p[:, 2])
    # equal-area bands: z values equally spaced by 2/n, symmetric about 0
    assert np.allclose(np.diff(z), 2.0 / n)
    assert np.isclose(z.sum(), 0.0, atol=1e-12)
    # successive azimuths advance by 2 pi / golden ratio
    az = np.arctan2(p[:, 1], p[:, 0])
    d = np.mod(np.diff(az), 2 * np.pi)
    assert np.allclose(d, np.mod(2 * np.pi / M.GOLDEN, 2 * np.pi))


def test_pinv_left_inverse():
    Am = M.A_matrix(A, K, ND)
    Ap = M.pinv(Am)
    assert np.linalg.norm(Ap @ Am - np.eye(81)) < 1e-9
    At_p = M.pinv(Am.T)
    assert np.linalg.norm(Am.T @ At_p - np.eye(81)) < 1e-9


def test_site_dipole_maps_exactly():
    # a point element sitting on a uniform dipole site is reproduced exactly
    sites = O.site_offsets(A, ND)
    t = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    pos = sites[[4, 20]]
    S = M.aggregation_matrix(A, ND, K, pos, t)
    e = np.zeros((81, 2))
    e[3 * 4 + 2, 0] = 1.0
    e[3 * 20 + 0, 1] = 1.0
    assert np.abs(S - e).max() < 1e-9


def test_disaggregation_is_transpose_of_aggregation():
    rng = np.random.default_rng(0)
    pos = rng.uniform(-A / 2, A / 2, size=(30, 3))
    t = rng.normal(size=(30, 3))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    S = M.aggregation_matrix(A, ND, K, pos, t)
    T = M.disaggregation_matrix(A, ND, K, pos, t)
    assert np.linalg.norm(T - S.T) <= 1e-10 * np.linalg.norm(S)


def test_test_site_fields_reproduced():
    # E at the uniform sites -> Q -> field back at the sites is the identity
    rng = np.random.default_rng(1)
    E = rng.normal(size=81) + 1j * rng.normal(size=81)
    Am = M.A_matrix(A, K, ND)
    Q = M.pinv(Am.T) @ E
    sites = O.site_offsets(A, ND)
    back = M.field_matrix(sites, M.sample_points(A, ND), K) @ Q
    assert np.linalg.norm(back - E) <= 1e-9 * np.linalg.norm(E)


def test_mapped_field_outside_sphere():
    # the mapped dipoles reproduce the element's field beyond the sphere
    # (uniqueness argument of Sec. 2.1); accuracy, not exactness
    rng = np.random.default_rng(2)
    pos = rng.uniform(-A / 2, A / 2, size=(5, 3))
    t = rng.normal(size=(5, 3))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    coef = rng.normal(size=5) + 1j * rng.normal(size=5)
    S = M.aggregation_matrix(A, ND, K, pos, t)
    C = S @ coef
    obs = np.array([[3 * A, 0.4 * A, -0.2 * A], [0.1, 2.5 * A, 2 * A]])
    sites = O.site_offsets(A, ND)
    # field of the elements themselves: sum_k D(obs - rho_k) t_k coef_k
    ref = sum(O.dyadic_green(obs - pos[kk], K) @ t[kk] * coef[kk] for kk in range(5))
    got = (M.field_matrix(obs, sites, K) @ C).reshape(-1, 3)
    assert np.linalg.norm(got - ref) <= 3e-2 * np.linalg.norm(ref)


def test_three_stage_operator_complex_symmetric():
    # with T = S^T, y = S^T G S x is a complex-symmetric map
    import workloads as W
    boxes = W.grid_boxes(3, 3, 3)
    nb = np.full(27, 5)
    nb_ptr, S = W.random_basis(nb, 24, 9, np.complex128)
    u = W.complex_normal((1, 135), 1, np.complex128)
    v = W.complex_normal((1, 135), 2, np.complex128)
    Mv = O.far_mvm(v, boxes, A, K, 2, nb_ptr, S)
    Mu = O.far_mvm(u, boxes, A, K, 2, nb_ptr, S)
    assert abs(np.sum(u * Mv) - np.sum(v * Mu)) <= 1e-12 * abs(np.sum(u * Mv))


def test_explicit_T_equals_default():
    import workloads as W
    boxes = W.grid_boxes(2, 2, 4)
    nb = np.array([3, 1, 4, 2, 5, 2, 1, 3, 2, 2, 4, 1, 3, 2, 2, 1])
    nb_ptr, S = W.random_basis(nb, 24, 3, np.complex128)
    # build T blocks as the transposes of the S blocks, column-major
    Tblocks, off = [], 0
    for b in range(16):
        Sb = S[off:off + 24 * nb[b]].reshape(nb[b], 24).T
        off += 24 * nb[b]
        Tblocks.append(Sb.T)
    T = M.column_major_blocks(Tblocks)
    x = W.complex_normal((2, int(nb.sum())), 4, np.complex128)
    y0 = O.far_mvm(x, boxes, A, K, 2, nb_ptr, S)
    y1 = O.far_mvm(x, boxes, A, K, 2, nb_ptr, S, T)
    assert np.array_equal(y0, y1)
