"""Uniform-basis mapping and inverse mapping, Sec. 2.1 and Sec. 2.3.

Test infrastructure (see the package docstring). This is the preprocessing
that produces the per-box aggregation matrix S_i (Algorithm 1: the stored
A^dagger and B_k) and disaggregation matrix T_i (Algorithm 3: the stored
(A^T)^dagger and D_k) for synthetic point current elements, which stand in
for RWG/SWG basis functions when no mesh is available.

Readings: sample points are the spherical Fibonacci lattice of Sec. 2.1 with
polar angle arccos(1 - (2l+1)/N_s) and azimuth 2 pi l / golden ratio,
l = 0..N_s-1 (the text swaps the usual theta/phi names); N_s = 2 N_d; the
sphere S has radius 1.5a about the box centre. Testing a field with a point
element means taking its component along the element's orientation, so the
vectorised testing operator D_k of Algorithm 3 is the transpose of B_k by
reciprocity of Eq. (5).
"""
import numpy as np

from .green import dyadic_green, ETA0
from .geometry import site_offsets

GOLDEN = 0.5 + 0.5 * np.sqrt(5.0)


def fibonacci_points(n_s, radius):
    """Spherical Fibonacci lattice points (n_s, 3) on a sphere of ``radius``."""
    l = np.arange(n_s, dtype=np.float64)
    polar = np.arccos(1.0 - (2.0 * l + 1.0) / n_s)
    azim = 2.0 * np.pi * l / GOLDEN
    return radius * np.stack([np.sin(polar) * np.cos(azim),
                              np.sin(polar) * np.sin(azim),
                              np.cos(polar)], axis=-1)


def sample_points(a, n_d):
    """The N_s = 2 N_d sampling points on the sphere of radius 1.5a."""
    return fibonacci_points(2 * n_d ** 3, 1.5 * a)


def field_matrix(points, sources, k, eta=ETA0):
    """Rows (l, alpha) x columns (s, beta): D(x_l - r_s)[alpha, beta]."""
    R = points[:, None, :] - sources[None, :, :]
    D = dyadic_green(R, k, eta)
    n_p, n_s = len(points), len(sources)
    return D.transpose(0, 2, 1, 3).reshape(3 * n_p, 3 * n_s)


def A_matrix(a, k, n_d, eta=ETA0):
    """Eq. (10): the 3N_s x N_u field of each uniform dipole at the samples."""
    return field_matrix(sample_points(a, n_d), site_offsets(a, n_d), k, eta)


def pinv(M):
    """Moore-Penrose pseudo-inverse by SVD with cutoff max(m,n)*eps*sigma_max."""
    return np.linalg.pinv(M, rcond=max(M.shape) * np.finfo(np.float64).eps)


def element_field(a, n_d, k, positions, orientations, eta=ETA0):
    """B: column k = samples of the field of point element k (Eq. 4, 10)."""
    pts = sample_points(a, n_d)
    R = pts[:, None, :] - np.asarray(positions)[None, :, :]
    D = dyadic_green(R, k, eta)                          # (l, k, 3, 3)
    cols = np.einsum("lkab,kb->lak", D, np.asarray(orientations))
    return cols.reshape(3 * len(pts), len(positions))


def aggregation_matrix(a, n_d, k, positions, orientations, eta=ETA0):
    """S = A^dagger B (Eq. 11 applied to every element of the box)."""
    return pinv(A_matrix(a, k, n_d, eta)) @ element_field(
        a, n_d, k, positions, orientations, eta)


def disaggregation_matrix(a, n_d, k, positions, orientations, eta=ETA0):
    """T = [D_1; ...; D_Nb] (A^T)^dagger (Eq. 17 then Eq. 15, Algorithm 3).

    Q = (A^T)^dagger E gives the virtual-dipole excitations on S; the field
    they produce at element k, tested along its orientation, is D_k Q with
    D_k[(l, beta)] = t_k . D(rho_k - x_l)[:, beta].
    """
    pts = sample_points(a, n_d)
    R = np.asarray(positions)[:, None, :] - pts[None, :, :]
    D = dyadic_green(R, k, eta)                          # (k, l, 3, 3)
    rows = np.einsum("ka,klab->klb", np.asarray(orientations), D)
    Dk = rows.reshape(len(positions), 3 * len(pts))
    return Dk @ pinv(A_matrix(a, k, n_d, eta).T)


def column_major_blocks(mats):
    """Flatten a list of matrices column-major and concatenate them."""
    return np.concatenate([np.asarray(m).T.reshape(-1) for m in mats])
