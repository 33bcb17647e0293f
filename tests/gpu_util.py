"""Helpers shared by the GPU tests (no method arithmetic)."""
import sys

import numpy as np


def rel_l2(got, ref):
    """Relative l2 error ||got - ref|| / ||ref|| (the Eq. 18-19 form)."""
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(got) - ref) / np.linalg.norm(ref))


def _box_bounds(n, boxes):
    """Start/stop of each box along a flattened per-RHS axis of length n."""
    if boxes is None:
        return np.array([0, n])
    if np.isscalar(boxes):
        assert n % int(boxes) == 0, (n, boxes)
        return np.arange(0, n + 1, int(boxes))
    ptr = np.asarray(boxes, dtype=np.int64)
    assert ptr[0] == 0 and ptr[-1] == n, (ptr[-1], n)
    return ptr


def parity(got, ref, tol, boxes=None, box_scale=None, label="", box_tol=None):
    """Compare a GPU result with the oracle at three grains and assert each.

    got, ref: complex arrays whose first axis is the right-hand side (any
    trailing shape is flattened per RHS). ``boxes`` splits the flattened axis
    into test boxes: coefficients per box (int) or a prefix array such as
    nb_ptr (ragged boxes; empty boxes are skipped). Asserted, per RHS:

    * whole result: ||got - ref|| <= tol ||ref|| (Eq. 18-19);
    * every test box b: ||got_b - ref_b|| <= box_tol ||ref_b|| (box_tol
      defaults to tol; a form whose per-product error is near the bar itself
      states a larger one), or, where
      ``box_scale`` is given (one value per box, e.g. the sum of the norms
      of the contributions the box receives), ||got_b - ref_b|| <=
      box_tol * box_scale[b]; a box whose reference is exactly zero must be
      exactly zero;
    * every element e: |got_e - ref_e| <= tol * max|ref| (max norm).

    Returns the worst values seen (for printing) and prints them.
    """
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.isfinite(got).all(), f"{label}: non-finite output"
    R = got.shape[0] if got.ndim > 1 else 1
    g = got.reshape(R, -1)
    r = ref.reshape(R, -1)
    ptr = _box_bounds(g.shape[1], boxes)
    box_tol = tol if box_tol is None else box_tol
    worst = {"global": 0.0, "box": 0.0, "elem": 0.0}
    for q in range(R):
        d = g[q] - r[q]
        nref = np.linalg.norm(r[q])
        if nref == 0.0:
            assert not np.any(g[q]), f"{label}: rhs {q} must be exactly zero"
            continue
        e_glob = float(np.linalg.norm(d) / nref)
        e_elem = float(np.abs(d).max() / np.abs(r[q]).max())
        # per-box sums over the non-empty boxes only: with strictly
        # increasing starts each reduceat segment ends where its box ends
        live = np.diff(ptr) > 0
        starts = ptr[:-1][live]
        dn = np.sqrt(np.add.reduceat(np.abs(d) ** 2, starts))
        rn = np.sqrt(np.add.reduceat(np.abs(r[q]) ** 2, starts))
        if box_scale is None:
            den = rn
        else:
            bs = np.asarray(box_scale, dtype=np.float64).reshape(-1)
            assert len(bs) == len(ptr) - 1, (len(bs), len(ptr) - 1)
            den = bs[live]
        zero = rn == 0.0
        assert not np.any(dn[zero]), f"{label}: rhs {q}: a box with zero reference is not zero"
        chk = den > 0.0
        e_box = float((dn[chk] / den[chk]).max()) if np.any(chk) else 0.0
        worst["global"] = max(worst["global"], e_glob)
        worst["elem"] = max(worst["elem"], e_elem)
        worst["box"] = max(worst["box"], e_box)
        assert e_glob <= tol, f"{label}: rhs {q}: rel_l2 {e_glob:.3e} > {tol:g}"
        assert e_box <= box_tol, \
            f"{label}: rhs {q}: worst per-box error {e_box:.3e} > {box_tol:g}"
        assert e_elem <= tol, f"{label}: rhs {q}: max-norm error {e_elem:.3e} > {tol:g}"
    print(f"{label}: rel_l2 {worst['global']:.2e}, worst box {worst['box']:.2e}, "
          f"max-norm {worst['elem']:.2e} (bar {tol:g}, per box {box_tol:g})")
    return worst


def announce(*parts):
    """Print and flush what names the case before a GPU step."""
    print("[gpu-case]", *parts, file=sys.stderr, flush=True)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()
