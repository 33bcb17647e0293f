"""The three stages of the far-zone MVM (Algorithm 5) in FP64.

Test infrastructure (see the package docstring).

Vectors are complex128 arrays of shape (nrhs, n_box, N_u) for the uniform
basis coefficients P and fields E, and (nrhs, sum N_b) for the subdomain
coefficients x and tested values y.
"""
import numpy as np

from .green import dyadic_green, ETA0
from .geometry import far_pairs, offset_ids, site_offsets, box_centres, FAR_ILIST
from .operators import translation_operator


def _blocks(nb_ptr):
    nb_ptr = np.asarray(nb_ptr, dtype=np.int64)
    return nb_ptr[:-1], np.diff(nb_ptr)


def aggregate(x, nb_ptr, S, n_u):
    """Stage 1 (Algorithm 1, Eq. 11): P_i = S_i x_i per box.

    ``S`` is the flat concatenation of column-major n_u x N_b,i blocks
    (S_i = A^dagger [B_1 ... B_Nb]); ``S is None`` means the identity basis
    (x already holds the uniform-basis coefficients, N_b,i = n_u).
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.complex128))
    nrhs = x.shape[0]
    if S is None:
        return x.reshape(nrhs, -1, n_u).copy()
    start, nb = _blocks(nb_ptr)
    P = np.zeros((nrhs, len(nb), n_u), dtype=np.complex128)
    soff = 0
    for b in range(len(nb)):
        Si = np.asarray(S[soff:soff + n_u * nb[b]], dtype=np.complex128)
        Si = Si.reshape(nb[b], n_u).T                 # column-major n_u x N_b
        soff += n_u * nb[b]
        P[:, b, :] = (Si @ x[:, start[b]:start[b] + nb[b]].T).T
    return P


def translate(P, boxes, a, k, n_d, mode=FAR_ILIST, eta=ETA0, pairs=None,
              test_boxes=None):
    """Stage 2 (Algorithm 2 with Eq. 13-14): E_j = sum_{i in F_j} G_{c_j-c_i} P_i.

    Grouped form: one G_w per distinct offset, applied with one complex128
    matmul to every pair at that offset. ``test_boxes`` restricts the output
    to a subset of test boxes (rows of other boxes are left zero).
    """
    P = np.asarray(P, dtype=np.complex128)
    j, i, w = far_pairs(boxes, mode) if pairs is None else pairs
    if test_boxes is not None:
        keep = np.isin(j, np.asarray(test_boxes))
        j, i, w = j[keep], i[keep], w[keep]
    E = np.zeros_like(P)
    if len(j) == 0:
        return E
    uniq, inv = offset_ids(w)
    for o, wv in enumerate(uniq):
        sel = np.nonzero(inv == o)[0]
        G = translation_operator(wv, a, k, n_d, eta)
        contrib = P[:, i[sel], :] @ G.T              # (nrhs, pairs, N_u)
        np.add.at(E, (slice(None), j[sel]), contrib)
    return E


def translate_bruteforce(P, boxes, a, k, n_d, mode=FAR_ILIST, eta=ETA0):
    """Stage 2 dipole by dipole, without forming any G_w (tiny grids only).

    For every far pair and every (test site, source site) the field of the
    source dipole at the absolute test position is evaluated with Eq. (5).
    """
    P = np.asarray(P, dtype=np.complex128)
    boxes = np.asarray(boxes)
    nrhs = P.shape[0]
    j, i, _ = far_pairs(boxes, mode)
    centres = box_centres(boxes, a)
    sites = site_offsets(a, n_d)
    nd3 = len(sites)
    E = np.zeros_like(P)
    for jj, ii in zip(j, i):
        for l in range(nd3):
            rt = centres[jj] + sites[l]
            for s in range(nd3):
                rs = centres[ii] + sites[s]
                D = dyadic_green(rt - rs, k, eta)
                for r in range(nrhs):
                    E[r, jj, 3 * l:3 * l + 3] += D @ P[r, ii, 3 * s:3 * s + 3]
    return E


def disaggregate(E, nb_ptr, S, T=None):
    """Stage 3 (Algorithm 3, Eq. 15-17): y_j = T_j E_j per box.

    ``T`` is the flat concatenation of column-major N_b,j x n_u blocks; when
    it is None, T_j = S_j^T (point testing of the Galerkin pair, see
    ``mapping.disaggregation_matrix``). ``S is None`` means the identity basis.
    """
    E = np.asarray(E, dtype=np.complex128)
    nrhs, n_box, n_u = E.shape
    if S is None and T is None:
        return E.reshape(nrhs, -1).copy()
    start, nb = _blocks(nb_ptr)
    y = np.zeros((nrhs, int(np.sum(nb))), dtype=np.complex128)
    off = 0
    for b in range(n_box):
        if T is None:
            Sb = np.asarray(S[off:off + n_u * nb[b]], dtype=np.complex128)
            Tb = Sb.reshape(nb[b], n_u)               # rows = columns of S_b
        else:
            Tb = np.asarray(T[off:off + n_u * nb[b]], dtype=np.complex128)
            Tb = Tb.reshape(n_u, nb[b]).T             # column-major N_b x n_u
        off += n_u * nb[b]
        y[:, start[b]:start[b] + nb[b]] = (Tb @ E[:, b, :].T).T
    return y


def far_mvm(x, boxes, a, k, n_d, nb_ptr=None, S=None, T=None,
            mode=FAR_ILIST, eta=ETA0):
    """Algorithm 5: y = T G_far S x (stages 1, 2, 3 in order)."""
    n_u = 3 * n_d ** 3
    P = aggregate(x, nb_ptr, S, n_u)
    E = translate(P, boxes, a, k, n_d, mode, eta)
    return disaggregate(E, nb_ptr, S, T)
