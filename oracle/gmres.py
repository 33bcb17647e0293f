"""Restarted GMRES in FP64, and the dense far-zone matrix of small problems.

Test infrastructure (see the package docstring).

The paper solves its systems with unpreconditioned restarted GMRES
(Sec. 5: tolerance, restart length and iteration cap are given there); the
far-zone product of Algorithm 5 is the matrix-vector product inside it.
This is the textbook method: Arnoldi with modified Gram-Schmidt builds an
orthonormal Krylov basis V and the (j+1) x j Hessenberg matrix H; the
iterate minimises ||beta e_1 - H y|| (solved here with a library
least-squares routine, no Givens bookkeeping); x = x_0 + V y; after
``restart`` steps the process restarts from the current residual.
"""
import numpy as np

from .geometry import FAR_ILIST, far_pairs
from .green import ETA0
from .operators import translation_operator


def gmres(matvec, b, restart, tol, max_steps):
    """Solve A x = b for one right-hand side, x_0 = 0.

    Returns ``(x, history)``: ``history[s]`` is the relative residual
    ||b - A x_s|| / ||b|| after step s (the least-squares residual, equal to
    the true residual in exact arithmetic); ``history[0]`` = 1.
    """
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    history = [1.0 if bnorm > 0 else 0.0]
    if bnorm == 0:
        return x, history
    steps = 0
    while steps < max_steps:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        V = [r / beta]
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        y = np.zeros(0, dtype=np.complex128)
        for j in range(restart):
            w = matvec(V[j])
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y) / bnorm
            steps += 1
            history.append(float(res))
            if res <= tol or steps >= max_steps or H[j + 1, j] == 0:
                break
            V.append(w / H[j + 1, j])
        x = x + np.stack(V[:len(y)], axis=1) @ y
        if history[-1] <= tol or (H[len(y), len(y) - 1] == 0):
            break
    return x, history


def far_matrix(boxes, a, k, n_d, mode=FAR_ILIST, eta=ETA0):
    """Dense Z^F in the identity basis: block (j, i) is G_{c_j - c_i} for
    every far pair (Eq. 13-14), zero otherwise. For small grids only."""
    boxes = np.asarray(boxes)
    n_u = 3 * n_d ** 3
    n = len(boxes)
    Z = np.zeros((n * n_u, n * n_u), dtype=np.complex128)
    j, i, w = far_pairs(boxes, mode)
    cache = {}
    for jj, ii, ww in zip(j, i, map(tuple, w)):
        if ww not in cache:
            cache[ww] = translation_operator(np.array(ww), a, k, n_d, eta)
        Z[jj * n_u:(jj + 1) * n_u, ii * n_u:(ii + 1) * n_u] = cache[ww]
    return Z
