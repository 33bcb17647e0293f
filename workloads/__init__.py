"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds no arithmetic of the method itself: it only produces box
occupancy sets (integer box coordinates), random complex coefficient vectors
and random per-box basis matrices, all from ``numpy.random.default_rng(seed)``.
Both sides receive exactly the same arrays; the HIP path gets them rounded to
complex64 and the oracle gets those rounded values upcast to complex128.

Geometries stand in for the paper's meshes (PEC/dielectric spheres, flamme,
almond), which are not available: a box grid partition of the mother box
(Sec. 2, the 8^L child boxes of side ``a``) only needs the set of occupied
child boxes, which these generators produce directly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "grid_boxes",
    "shell_boxes",
    "plate_boxes",
    "mask_boxes",
    "hollow_cube_boxes",
    "scatterer_set",
    "serving_requests",
    "complex_normal",
    "random_basis",
    "config",
    "CONFIGS",
]


def grid_boxes(nx: int, ny: int, nz: int) -> np.ndarray:
    """All boxes of an ``nx x ny x nz`` grid, as an (n, 3) int32 array.

    Order: x slowest, z fastest (lexicographic), which is also the order the
    oracle and the library use to number boxes.
    """
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij"), axis=-1)
    return g.reshape(-1, 3).astype(np.int32)


def shell_boxes(radius: float, thickness: float, a: float) -> np.ndarray:
    """Boxes of side ``a`` whose centre lies in the spherical shell
    ``radius - thickness/2 <= |r| < radius + thickness/2``.

    The sphere is centred on the centre of the middle box of a cubic grid of
    ``2*ceil((radius + thickness/2)/a) + 1`` boxes per side, so box ``c`` has
    its centre at ``a*(c - m)`` relative to the sphere centre, ``m`` being the
    middle index. All lengths are in the same unit (wavelengths here).
    The integer test |d|^2 in [lo^2, hi^2) is exact for the half-integer
    radii used by the shipped workloads.
    """
    half = int(math.ceil((radius + thickness / 2) / a))
    n = 2 * half + 1
    c = grid_boxes(n, n, n)
    d = (c - half).astype(np.float64) * a
    r = np.sqrt((d * d).sum(axis=1))
    keep = (r >= radius - thickness / 2) & (r < radius + thickness / 2)
    return c[keep]


def plate_boxes(lx: float, ly: float, lz: float, a: float) -> np.ndarray:
    """A solid ``lx x ly x lz`` plate voxelised into boxes of side ``a``."""
    n = [max(1, int(round(v / a))) for v in (lx, ly, lz)]
    return grid_boxes(*n)


def mask_boxes(n_target: int, rho: float, seed: int) -> np.ndarray:
    """Bernoulli(rho) occupancy of a cube of side ``ceil((n_target/rho)^(1/3))``.

    At least one box is always kept so the set is never empty.
    """
    rng = np.random.default_rng(seed)
    side = max(1, int(math.ceil((n_target / rho) ** (1.0 / 3.0))))
    c = grid_boxes(side, side, side)
    keep = rng.random(len(c)) < rho
    if not keep.any():
        keep[rng.integers(len(c))] = True
    return c[keep]


def hollow_cube_boxes(n: int) -> np.ndarray:
    """The one-box-thick surface of an ``n x n x n`` cube of boxes."""
    c = grid_boxes(n, n, n)
    on = ((c == 0) | (c == n - 1)).any(axis=1)
    return c[on]


SCATTERER_KINDS = ("shell", "hollow_cube", "plate", "mask")


def scatterer_set(count: int, seed: int, lo: int = 200, hi: int = 20000,
                  a: float = 0.25) -> list[tuple[str, np.ndarray]]:
    """``count`` independent scatterers of uneven size for batched runs.

    Target box counts are log-uniform in ``[lo, hi]``; kinds cycle through
    one-box-thick spherical shells, hollow cubes, plates one or two boxes
    thick with aspect ratio in [1, 4], and Bernoulli(rho) occupancy masks
    with rho uniform in [0.1, 1.0]. Each scatterer has its own coordinates
    (they may overlap across scatterers). Returns ``[(kind, boxes), ...]``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        target = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        kind = SCATTERER_KINDS[s % len(SCATTERER_KINDS)]
        if kind == "shell":
            radius = a * math.sqrt(target / (4.0 * math.pi))
            b = shell_boxes(radius, a, a)
        elif kind == "hollow_cube":
            b = hollow_cube_boxes(max(2, int(round(math.sqrt(target / 6.0))) + 1))
        elif kind == "plate":
            thick = int(rng.integers(1, 3))
            ratio = rng.uniform(1.0, 4.0)
            nx = max(1, int(round(math.sqrt(target / thick * ratio))))
            ny = max(1, int(round(target / thick / nx)))
            b = grid_boxes(nx, ny, thick)
        else:
            rho = rng.uniform(0.1, 1.0)
            b = mask_boxes(int(round(target)), rho, int(rng.integers(1 << 31)))
        out.append((kind, b))
    return out


def serving_requests(count: int, rate: float, seed: int, lo: int = 500,
                     hi: int = 50000, max_nrhs: int = 8) -> list[dict]:
    """A Poisson stream of solve requests on random-occupancy grids.

    Inter-arrival times are exponential with mean ``1/rate`` seconds; box
    counts are log-uniform in ``[lo, hi]`` on Bernoulli(rho) masks with rho
    uniform in [0.1, 1.0]; 1..``max_nrhs`` right-hand sides (uniform).
    Returns dicts with ``arrival``, ``boxes``, ``nrhs`` and ``b_seed`` (the
    seed of the request's right-hand sides, see ``complex_normal``).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        target = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
        rho = float(rng.uniform(0.1, 1.0))
        boxes = mask_boxes(target, rho, int(rng.integers(1 << 31)))
        out.append({"arrival": t, "boxes": boxes,
                    "nrhs": int(rng.integers(1, max_nrhs + 1)),
                    "b_seed": int(rng.integers(1 << 31))})
    return out


def complex_normal(shape, seed: int, dtype=np.complex64) -> np.ndarray:
    """i.i.d. N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return z.astype(dtype)


def random_networks(n_off: int, hidden: int, n_u: int, seed: int,
                    bias: float = 0.1) -> tuple:
    """Seeded complex64 weights of one network per offset, shaped as the
    library takes them: W1 (n_off, hidden, n_u) with N(0, 1/n_u) parts,
    b1 (n_off, hidden), W2 (n_off, n_u, hidden) with N(0, 1/hidden) parts,
    b2 (n_off, n_u); biases have N(0, bias^2) parts."""
    W1 = complex_normal((n_off, hidden, n_u), seed) / np.float32(np.sqrt(n_u))
    b1 = complex_normal((n_off, hidden), seed + 1) * np.float32(bias)
    W2 = complex_normal((n_off, n_u, hidden), seed + 2) / np.float32(np.sqrt(hidden))
    b2 = complex_normal((n_off, n_u), seed + 3) * np.float32(bias)
    return (W1.astype(np.complex64), b1.astype(np.complex64), W2.astype(np.complex64),
            b2.astype(np.complex64))


def random_basis(nb: np.ndarray, n_u: int, seed: int,
                 dtype=np.complex64) -> tuple[np.ndarray, np.ndarray]:
    """Random per-box basis matrices ``S_i`` (``n_u x nb[i]``, column-major).

    Returns ``(nb_ptr, S)`` where ``nb_ptr`` is the (n_box+1,) int64 prefix
    sum of ``nb`` and ``S`` is the flat concatenation of the column-major
    blocks (length ``n_u * nb_ptr[-1]``). Entries are complex N(0,1)/sqrt(n_u)
    so that ``S_i x_i`` keeps unit scale.
    """
    nb = np.asarray(nb, dtype=np.int64)
    nb_ptr = np.zeros(len(nb) + 1, dtype=np.int64)
    np.cumsum(nb, out=nb_ptr[1:])
    total = int(nb_ptr[-1]) * n_u
    S = complex_normal((total,), seed, np.complex128) / math.sqrt(n_u)
    return nb_ptr, S.astype(dtype)


@dataclass
class Workload:
    """One synthetic far-zone MVM problem."""

    name: str
    boxes: np.ndarray            # (n_box, 3) int32, unique, >= 0
    a: float                     # box side, wavelengths
    k: float                     # wavenumber, rad per wavelength
    n_d: int                     # dipoles per box edge
    far_mode: str                # "ilist" or "full"
    nrhs: int = 1
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_box(self) -> int:
        return int(len(self.boxes))

    @property
    def n_u(self) -> int:
        return 3 * self.n_d ** 3

    def coefficients(self, nb_total: int | None = None, seed: int | None = None,
                     dtype=np.complex64) -> np.ndarray:
        """``[nrhs][sum N_b]`` coefficient vectors (identity basis: N_b = n_u)."""
        n = self.n_box * self.n_u if nb_total is None else nb_total
        return complex_normal((self.nrhs, n), self.seed if seed is None else seed,
                              dtype)


TWO_PI = 2.0 * math.pi


def config(idx: int, **over) -> Workload:
    """The named synthetic workloads.

    1: 6x6x6 full grid, a = 0.25 wavelength, k = 2 pi, n_d = 3, ILIST.
    2: spherical shell, radius 4, thickness 0.25, a = 0.25 (centre rule).
    3: the same shell at a = 0.125 (and ``variant="plate"``: a 0.5 x 2 x 8
       plate at a = 0.125).
    4: batching: 64 scatterers of 200 to 20k boxes (``scatterer_set``) at
       a = 0.25, four right-hand sides each; ``boxes`` is their
       concatenation and ``extra["scatterers"]`` the list of box arrays
       (``count=`` picks another number of scatterers).

    6: the network translation workload of Sec. 3 and Sec. 5: a sphere of
       diameter 2 wavelengths voxelised at a = 0.125 (its centre-rule shell,
       radius 1, thickness 0.125), n_d = 4 (3 N_d = 192), ILIST.

    The serving stream (Poisson arrivals of solves on random-occupancy
    grids) is ``serving_requests``.
    """
    if idx == 1:
        w = Workload("grid6_a0.25", grid_boxes(6, 6, 6), 0.25, TWO_PI, 3,
                     "ilist", seed=1)
    elif idx == 2:
        w = Workload("shell_r4_t0.25_a0.25", shell_boxes(4.0, 0.25, 0.25),
                     0.25, TWO_PI, 3, "ilist", seed=2)
    elif idx == 3:
        if over.pop("variant", "shell") == "plate":
            w = Workload("plate_0.5x2x8_a0.125",
                         plate_boxes(0.5, 2.0, 8.0, 0.125), 0.125, TWO_PI, 3,
                         "ilist", seed=3)
        else:
            w = Workload("shell_r4_t0.25_a0.125",
                         shell_boxes(4.0, 0.25, 0.125), 0.125, TWO_PI, 3,
                         "ilist", seed=3)
    elif idx == 4:
        count = int(over.pop("count", 64))
        parts = scatterer_set(count, seed=4)
        w = Workload(f"batch{count}_a0.25", np.concatenate([b for _, b in parts]),
                     0.25, TWO_PI, 3, "ilist", nrhs=4, seed=4,
                     extra={"scatterers": [b for _, b in parts],
                            "kinds": [k for k, _ in parts]})
    elif idx == 6:
        w = Workload("sphere_d2_a0.125_nd4", shell_boxes(1.0, 0.125, 0.125), 0.125,
                     TWO_PI, 4, "ilist", seed=6)
    else:
        raise ValueError(f"unknown workload {idx}")
    for key, v in over.items():
        setattr(w, key, v)
    return w


CONFIGS = (1, 2, 3, 4)
