"""Translation matrices G_w, Eq. (12)-(13) of Sec. 2.2.

Test infrastructure (see the package docstring).
"""
import numpy as np

from .green import dyadic_green, ETA0
from .geometry import site_offsets


def translation_operator(w, a, k, n_d, eta=ETA0):
    """G_w, the 3N_d x 3N_d complex128 matrix for integer box offset w.

    Column (s, beta) is the field at every test site l of the test box due to
    the beta-directed unit dipole at site s of the basis box, whose centre is
    a*w away:  G_w[(l, alpha), (s, beta)] = D(a w + r_l - r_s)[alpha, beta].
    """
    r = site_offsets(a, n_d)
    R = a * np.asarray(w, dtype=np.float64) + r[:, None, :] - r[None, :, :]
    D = dyadic_green(R, k, eta)                       # (l, s, alpha, beta)
    nd3 = len(r)
    return D.transpose(0, 2, 1, 3).reshape(3 * nd3, 3 * nd3)


def translation_operators(offsets, a, k, n_d, eta=ETA0):
    """Stack of G_w for each row of ``offsets``: (n_off, 3N_d, 3N_d)."""
    return np.stack([translation_operator(w, a, k, n_d, eta)
                     for w in np.asarray(offsets)])
