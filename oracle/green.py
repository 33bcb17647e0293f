"""Free-space dyadic Green's function, Eq. (5)-(6) of Sec. 2.1.

Test infrastructure (see the package docstring). Time convention exp(+j w t)
(Sec. 1, last paragraph), so fields carry exp(-j k R).
"""
import numpy as np

# Intrinsic impedance of free space (mu0 * c). The paper does not give a
# value; it is a pure scale factor of every operator.
ETA0 = 376.730313668


def dyadic_green(R, k, eta=ETA0):
    """D(R) for separation vectors ``R = r - r'`` of shape (..., 3).

    D = psi(R) * { I (1 - j/(kR) - 1/(kR)^2) - Rhat Rhat (1 - 3j/(kR) - 3/(kR)^2) }
    psi(R) = -j k eta exp(-j k R) / (4 pi R)                       (Eq. 5, 6)

    Returns complex128 of shape (..., 3, 3). R must be non-zero.
    """
    R = np.asarray(R, dtype=np.float64)
    r = np.sqrt(np.sum(R * R, axis=-1))
    if np.any(r == 0.0):
        raise ValueError("dyadic_green: zero separation")
    rhat = R / r[..., None]
    kr = k * r
    psi = np.asarray(-1j * k * eta * np.exp(-1j * kr) / (4.0 * np.pi * r))
    c_iso = np.asarray(1.0 - 1j / kr - 1.0 / kr ** 2)
    c_rr = np.asarray(1.0 - 3j / kr - 3.0 / kr ** 2)
    eye = np.eye(3)
    outer = rhat[..., :, None] * rhat[..., None, :]
    return psi[..., None, None] * (c_iso[..., None, None] * eye
                                   - c_rr[..., None, None] * outer)
