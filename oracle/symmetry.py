"""Rotation/mirror symmetries of the box lattice, Sec. 2.2 (after Eq. 14).

Test infrastructure (see the package docstring). The 48 signed permutation
matrices of the cube map translation vectors onto equivalent ones; for cell-
centred sites they also permute the dipole sites of a box among themselves,
which is why G for one vector of an orbit determines the others.
"""
import itertools

import numpy as np


def cube_group():
    """The 48 signed 3x3 permutation matrices (integer)."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), dtype=np.int64)
            for r, c in enumerate(perm):
                M[r, c] = signs[r]
            mats.append(M)
    return mats


def orbits(offsets):
    """Group integer offsets into orbits of the cube group.

    Returns a list of sorted tuples of offsets, one per orbit.
    """
    group = cube_group()
    remaining = {tuple(int(v) for v in w) for w in np.asarray(offsets)}
    out = []
    while remaining:
        w = min(remaining)
        orb = {tuple(int(v) for v in (M @ np.array(w))) for M in group}
        orb &= remaining | {w}
        remaining -= orb
        out.append(tuple(sorted(orb)))
    return out


def dof_permutation(M, n_d):
    """Signed permutation Pi (3N_d x 3N_d) acting on a box's dipole vector.

    A site at offset r from the box centre moves to M r, and a dipole moment
    p becomes M p, so (Pi v)[(s', alpha)] = sum_beta M[alpha, beta] v[(s, beta)]
    where site s' = site at M r_s.
    """
    m = np.arange(n_d)
    g = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3)
    centred = 2 * g - (n_d - 1)                     # integer, symmetric
    moved = centred @ M.T
    idx_of = {tuple(v): s for s, v in enumerate(centred)}
    nd3 = len(g)
    Pi = np.zeros((3 * nd3, 3 * nd3))
    for s in range(nd3):
        sp = idx_of[tuple(moved[s])]
        Pi[3 * sp:3 * sp + 3, 3 * s:3 * s + 3] = M
    return Pi
