"""Box grid, uniform dipole sites and the far-zone interaction set.

Test infrastructure (see the package docstring).

Readings of the paper used here (each is listed in the design notes):
  * Sites (Sec. 2.1, "n_d dipoles along each of x, y, z with uniform
    separation"): cell-centred, at a*((m + 1/2)/n_d - 1/2) from the box
    centre, m in {0..n_d-1}^3; site index s = (m_x*n_d + m_y)*n_d + m_z and
    degree of freedom u = 3*s + alpha (alpha = x, y, z).
  * Box centre: a*(c + 1/2) for integer box coordinate c, so the translation
    vector between boxes is a*(c_test - c_source) (Sec. 2.2, w_ij = r_j - r_i).
  * FULL far set: every pair with ||w|| >= 2a (Algorithm 2), which for integer
    offsets is Chebyshev norm >= 2.
  * ILIST far set: FULL restricted to pairs whose parents floor(c/2) are
    Chebyshev-adjacent -- the one-box-buffer interaction list of a two-level
    tree. The 316 translation vectors counted in Sec. 2.2 are exactly this
    set's offsets.
"""
import numpy as np

FAR_ILIST = "ilist"
FAR_FULL = "full"


def site_offsets(a, n_d):
    """(n_d^3, 3) site positions relative to the box centre."""
    m = np.arange(n_d)
    g = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3)
    return a * ((g + 0.5) / n_d - 0.5)


def box_centres(boxes, a):
    """(n_box, 3) box centres a*(c + 1/2)."""
    return a * (np.asarray(boxes, dtype=np.float64) + 0.5)


def _check_boxes(boxes):
    b = np.asarray(boxes, dtype=np.int64)
    if b.ndim != 2 or b.shape[1] != 3:
        raise ValueError("boxes must be (n, 3)")
    if len(b) and b.min() < 0:
        raise ValueError("box coordinates must be >= 0")
    if len(np.unique(b, axis=0)) != len(b):
        raise ValueError("duplicate boxes")
    return b


def far_pairs(boxes, mode=FAR_ILIST):
    """All far-zone (test j, source i) pairs, sorted by (j, i).

    Returns (j, i, w) with w = c_j - c_i of shape (n_pairs, 3).
    FULL mode enumerates every ordered pair; ILIST scans the 7^3 offsets
    within Chebyshev distance 3, which contains every ILIST pair.
    """
    b = _check_boxes(boxes)
    n = len(b)
    if n == 0:
        z = np.zeros(0, dtype=np.int64)
        return z, z, np.zeros((0, 3), dtype=np.int64)
    if mode == FAR_FULL:
        w = b[:, None, :] - b[None, :, :]
        keep = np.abs(w).max(axis=-1) >= 2
        j, i = np.nonzero(keep)
        return j, i, w[j, i]
    if mode != FAR_ILIST:
        raise ValueError(f"unknown far mode {mode!r}")
    hi = b.max(axis=0) + 1
    index = -np.ones(tuple(hi), dtype=np.int64)
    index[b[:, 0], b[:, 1], b[:, 2]] = np.arange(n)
    js, is_, ws = [], [], []
    rng = np.arange(-3, 4)
    for wx in rng:
        for wy in rng:
            for wz in rng:
                w = np.array([wx, wy, wz])
                if np.abs(w).max() < 2:
                    continue
                src = b - w
                ok = np.all((src >= 0) & (src < hi), axis=1)
                jj = np.nonzero(ok)[0]
                ii = index[src[jj, 0], src[jj, 1], src[jj, 2]]
                occ = ii >= 0
                jj, ii = jj[occ], ii[occ]
                par = np.abs(b[jj] // 2 - b[ii] // 2).max(axis=1) <= 1
                jj, ii = jj[par], ii[par]
                js.append(jj)
                is_.append(ii)
                ws.append(np.broadcast_to(w, (len(jj), 3)))
    j = np.concatenate(js)
    i = np.concatenate(is_)
    w = np.concatenate(ws).astype(np.int64)
    order = np.lexsort((i, j))
    return j[order], i[order], w[order]


def offset_ids(w):
    """Distinct offsets (lexicographically sorted) and each pair's index."""
    uniq, inv = np.unique(np.asarray(w, dtype=np.int64), axis=0,
                          return_inverse=True)
    return uniq, inv.reshape(-1)
