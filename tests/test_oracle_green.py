"""Pins of the dyadic Green's function (Eq. 5-6) against independent facts."""
import numpy as np
import pytest

from oracle import dyadic_green, ETA0


def hertzian_field_closed_form(R, axis, k, eta=ETA0):
    """Textbook field of a unit current element I*l = 1 along ``axis``.

    In spherical coordinates about the element (exp(+jwt) convention):
      E_r     = eta cos(t) / (2 pi r^2) (1 + 1/(jkr)) exp(-jkr)
      E_theta = j eta k sin(t) / (4 pi r) (1 + 1/(jkr) - 1/(kr)^2) exp(-jkr)
    returned in Cartesian components.
    """
    R = np.asarray(R, float)
    r = np.linalg.norm(R)
    rhat = R / r
    zhat = np.zeros(3)
    zhat[axis] = 1.0
    cos_t = rhat @ zhat
    # theta-hat = (cos t) rhat - zhat, normalised (points toward +theta)
    th = cos_t * rhat - zhat
    sin_t = np.linalg.norm(th)
    th = th / sin_t if sin_t > 0 else th
    e = np.exp(-1j * k * r)
    Er = eta * cos_t / (2 * np.pi * r ** 2) * (1 + 1 / (1j * k * r)) * e
    Et = 1j * eta * k * sin_t / (4 * np.pi * r) * (
        1 + 1 / (1j * k * r) - 1 / (k * r) ** 2) * e
    return Er * rhat + Et * th


@pytest.mark.parametrize("k", [2 * np.pi, 0.03, 40.0])
def test_matches_hertzian_dipole_closed_form(k):
    rng = np.random.default_rng(0)
    for _ in range(50):
        R = rng.normal(size=3) * rng.uniform(0.05, 3.0)
        D = dyadic_green(R, k)
        for axis in range(3):
            ref = hertzian_field_closed_form(R, axis, k)
            got = D[:, axis]
            assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_symmetric_and_even():
    rng = np.random.default_rng(1)
    R = rng.normal(size=(200, 3))
    D = dyadic_green(R, 2 * np.pi)
    assert np.allclose(D, np.swapaxes(D, -1, -2), rtol=0, atol=0)
    Dm = dyadic_green(-R, 2 * np.pi)
    assert np.array_equal(D, Dm)


def test_static_limit():
    # kR -> 0: D -> j eta (I - 3 Rhat Rhat) / (4 pi k R^3)
    rng = np.random.default_rng(2)
    for _ in range(20):
        R = rng.normal(size=3)
        r = np.linalg.norm(R)
        rh = R / r
        k = 1e-5
        stat = 1j * ETA0 * (np.eye(3) - 3 * np.outer(rh, rh)) / (4 * np.pi * k * r ** 3)
        D = dyadic_green(R, k)
        assert np.linalg.norm(D - stat) <= 1e-4 * np.linalg.norm(stat)


def test_far_field_limit():
    # kR -> inf: D -> psi (I - Rhat Rhat), transverse, decaying as 1/R
    rng = np.random.default_rng(3)
    k = 2 * np.pi
    for _ in range(20):
        rh = rng.normal(size=3)
        rh /= np.linalg.norm(rh)
        r = 1e5
        psi = -1j * k * ETA0 * np.exp(-1j * k * r) / (4 * np.pi * r)
        ff = psi * (np.eye(3) - np.outer(rh, rh))
        D = dyadic_green(r * rh, k)
        assert np.linalg.norm(D - ff) <= 1e-5 * np.linalg.norm(ff)


def test_zero_separation_rejected():
    with pytest.raises(ValueError):
        dyadic_green(np.zeros(3), 1.0)
