"""Pins of the far-zone pair set (Algorithm 2 and the interaction-list reading)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_pairs(boxes, mode):
    """Explicit double loop over ordered pairs with the stated conditions."""
    out = []
    for jj, cj in enumerate(boxes):
        for ii, ci in enumerate(boxes):
            w = [int(cj[d]) - int(ci[d]) for d in range(3)]
            if max(abs(v) for v in w) < 2:
                continue
            if mode == "ilist":
                pj = [int(cj[d]) // 2 for d in range(3)]
                pi = [int(ci[d]) // 2 for d in range(3)]
                if max(abs(pj[d] - pi[d]) for d in range(3)) > 1:
                    continue
            out.append((jj, ii, tuple(w)))
    return sorted(out)


def closed_form_count(n, mode):
    """Pairs on a full n^3 grid.

    Per axis, ordered coordinate pairs with |dc| <= 1 number n + 2(n-1);
    ordered pairs whose parents are adjacent number 4 * (p + 2(p-1)) with
    p = n/2 parents (n even). Near pairs are always parent-adjacent.
    """
    near = (n + 2 * (n - 1)) ** 3
    if mode == "full":
        return n ** 6 - near
    p = n // 2
    return (4 * (p + 2 * (p - 1))) ** 3 - near


@pytest.mark.parametrize("mode", ["ilist", "full"])
@pytest.mark.parametrize("boxes", [
    W.grid_boxes(2, 2, 4), W.grid_boxes(4, 4, 4), W.grid_boxes(3, 5, 2),
    W.mask_boxes(60, 0.4, 7), np.array([[0, 0, 0]], dtype=np.int32),
])
def test_matches_brute_force(boxes, mode):
    j, i, w = O.far_pairs(boxes, mode)
    got = sorted((int(a), int(b), tuple(int(v) for v in c)) for a, b, c in zip(j, i, w))
    assert got == brute_pairs(boxes, mode)


@pytest.mark.parametrize("n", [2, 4, 6, 8])
@pytest.mark.parametrize("mode", ["ilist", "full"])
def test_closed_form_counts(n, mode):
    j, _, _ = O.far_pairs(W.grid_boxes(n, n, n), mode)
    assert len(j) == closed_form_count(n, mode)


def test_paper_316_vectors_16_matrices():
    ref = json.load(open(os.path.join(GOLDEN, "sec2_2_offset_count.json")))
    # single-level far set of a 4^3 grid (L = 2) equals the interaction list
    b = W.grid_boxes(4, 4, 4)
    jf, if_, wf = O.far_pairs(b, "full")
    ji, ii, wi = O.far_pairs(b, "ilist")
    assert np.array_equal(jf, ji) and np.array_equal(if_, ii)
    uniq, _ = O.offset_ids(wf)
    assert len(uniq) == ref["n_translation_vectors"]
    assert len(O.symmetry.orbits(uniq)) == ref["n_unique_matrices"]
    # the same 316 vectors on any larger full grid under the interaction list
    uniq6, _ = O.offset_ids(O.far_pairs(W.grid_boxes(6, 6, 6), "ilist")[2])
    assert len(uniq6) == ref["n_translation_vectors"]
    assert np.array_equal(uniq6, uniq)


def test_ilist_offset_ranges_per_parity():
    # a test box with even coordinate sees offsets in [-3, 2], odd in [-2, 3]
    b = W.grid_boxes(8, 8, 8)
    j, i, w = O.far_pairs(b, "ilist")
    par = b[j] % 2
    assert np.all(w[par == 0] <= 2) and np.all(w[par == 0] >= -3)
    assert np.all(w[par == 1] >= -2) and np.all(w[par == 1] <= 3)
    counts = np.bincount(j, minlength=len(b))
    assert counts.max() == 189


def test_rejects_bad_boxes():
    with pytest.raises(ValueError):
        O.far_pairs(np.array([[0, 0, 0], [0, 0, 0]]))
    with pytest.raises(ValueError):
        O.far_pairs(np.array([[0, -1, 0]]))


def test_shell_workload_shape():
    w = W.config(2)
    assert w.n_box == 3338
    j, _, _ = O.far_pairs(w.boxes, "ilist")
    assert len(j) == 108888
