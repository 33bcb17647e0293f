"""Plain FP64 CPU oracle for the far-zone matrix-vector product.

TEST INFRASTRUCTURE ONLY. This package is the independent reference that the
HIP path is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the library and its
Python binding never do, and it never imports them.

Everything here is written from the paper (arXiv 2501.04684, Koç, Kalfa,
Dogan, Ertürk): the dyadic Green's function (Eq. 5-6), the uniform-basis
mapping (Sec. 2.1, Eq. 9-11, Algorithm 1), the translation by the direct
Green's function approach (Sec. 2.2, Eq. 12-14, Algorithm 2) and the inverse
mapping (Sec. 2.3, Eq. 15-17, Algorithm 3), combined as in Algorithm 5, the
network translation of Sec. 3 (Fig. 5, Eq. 18-19) and the restarted GMRES the
paper's solutions use (Sec. 5).
Arithmetic is complex128 / float64 throughout; NumPy matmul/pinv serve as
library primitives, with no blocking, fusion or reordering beyond what the
definitions state.

Pins (see ``tests/test_oracle_*.py``): closed-form Hertzian-dipole fields,
static and far-field limits, reciprocity, the 48 cube symmetries, the
316/16 count printed in Sec. 2.2, closed-form far-set counts, brute-force
dipole sums on tiny grids, the least-squares identities of Eq. 11/17, exact
linear networks against the DGFA translation, and for GMRES exact dense
solves, finite termination and true-residual identities.
Parity unpinned: nothing in this package (every function has a pin).
"""
from .green import dyadic_green, ETA0
from .geometry import (site_offsets, box_centres, far_pairs, offset_ids,
                       FAR_ILIST, FAR_FULL)
from .operators import translation_operator, translation_operators
from .mvm import (aggregate, translate, translate_bruteforce, disaggregate,
                  far_mvm)
from . import cvfcnn, gmres, mapping, symmetry

__all__ = [
    "dyadic_green", "ETA0", "site_offsets", "box_centres", "far_pairs",
    "offset_ids", "FAR_ILIST", "FAR_FULL", "translation_operator",
    "translation_operators", "aggregate", "translate",
    "translate_bruteforce", "disaggregate", "far_mvm", "cvfcnn", "gmres",
    "mapping", "symmetry",
]
