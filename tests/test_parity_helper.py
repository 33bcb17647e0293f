"""The GPU tests' parity check on planted errors (CPU only).

A single coefficient off by a few per cent of the typical value hides in the
relative l2 norm of a large output; the per-box and max-norm grains of
``parity`` must catch it, and a zero box must stay exactly zero.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import parity, rel_l2


def _pair(n_box=3338, n_u=81, seed=0):
    ref = W.complex_normal((1, n_box * n_u), seed).astype(np.complex128)
    got = ref * (1 + 1e-7)
    return got, ref


def test_clean_result_passes():
    got, ref = _pair()
    w = parity(got, ref, 1e-4, boxes=81, label="clean")
    assert w["global"] < 1e-6


def test_one_coefficient_off_hides_in_l2_but_is_caught():
    got, ref = _pair()
    got[0, 12345] += 0.04 * np.sqrt(2)           # ~4% of a typical entry
    assert rel_l2(got, ref) <= 1e-4               # the old global check passes
    with pytest.raises(AssertionError, match="per-box|max-norm"):
        parity(got, ref, 1e-4, boxes=81, label="planted")


def test_one_box_off_is_caught_per_box():
    got, ref = _pair()
    got[0, 81 * 7:81 * 8] *= 1 + 5e-4             # a whole box 5e-4 off
    assert rel_l2(got, ref) <= 1e-4
    with pytest.raises(AssertionError, match="per-box"):
        parity(got, ref, 1e-4, boxes=81, label="box")


def test_zero_reference_box_must_be_zero():
    got, ref = _pair(n_box=10)
    ref[0, :81] = 0
    got[0, :81] = 1e-30
    with pytest.raises(AssertionError, match="zero reference"):
        parity(got, ref, 1e-4, boxes=81, label="zero box")


def test_ragged_boxes_and_scaled_bound():
    ref = W.complex_normal((2, 100), 3).astype(np.complex128)
    nb_ptr = np.array([0, 0, 30, 30, 100])        # empty boxes are skipped
    got = ref.copy()
    got[1, 40] += 1e-3
    with pytest.raises(AssertionError, match="max-norm"):
        parity(got, ref, 1e-4, boxes=nb_ptr, label="ragged")
    # a box whose field is small next to its terms: 1e-5 off is 1e-3 of its
    # own norm, but within the bar against the scale of the terms it sums
    ref[:, 0:30] *= 1e-3
    got = ref.copy()
    got[0, 3] += 1e-5
    with pytest.raises(AssertionError, match="per-box"):
        parity(got, ref, 1e-4, boxes=nb_ptr, label="own norm")
    parity(got, ref, 1e-4, boxes=nb_ptr, box_scale=np.array([0.0, 1.0, 0.0, 10.0]),
           label="scaled")


def test_non_finite_output_fails():
    got, ref = _pair(n_box=4)
    got[0, 3] = np.nan
    with pytest.raises(AssertionError, match="non-finite"):
        parity(got, ref, 1e-4, boxes=81)
