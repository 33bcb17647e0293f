"""Translation by complex-valued fully connected networks (Sec. 3, Fig. 5).

Test infrastructure (see the package docstring).

Sec. 3 replaces the DGFA product G_w P_i of Eq. 13 by one network per
translation vector w: a feed-forward complex network with one hidden layer
of H units, input and output dimension 3N_d, and the Cartesian ReLU on the
hidden layer. The input box vector is divided by its l-infinity norm first.

Readings (each is listed in the design notes):
  * l-infinity norm of a complex vector: its largest modulus.
  * Layers are affine: f_w(v) = W2 CReLU(W1 v + b1) + b2, W1 (H x 3N_d),
    W2 (3N_d x H), complex weights and biases.
  * CReLU(z) = max(Re z, 0) + j max(Im z, 0), component by component.
  * The network predicts G_w applied to the normalised input, so the
    contribution of source box i is ||P_i||_inf * f_w(P_i / ||P_i||_inf); a
    zero box vector contributes zero.
  * E_j sums these contributions over the far set exactly as Eq. 14 sums
    the DGFA products.
The relative error of Eq. 18 and Eq. 19 (e^u, e^sp) is ``relative_error``
below.

Pins (``tests/test_oracle_cvfcnn.py``): CReLU on hand values; a network built
as W1 = [I; -I], W2 = [G, -G] computes G v exactly, so its translation equals
the DGFA translation; positive homogeneity without biases; constant networks;
the cube-symmetry map of networks against the pinned operator symmetry.
"""
import numpy as np

from .geometry import FAR_ILIST, far_pairs, offset_ids


def crelu(z):
    """Cartesian ReLU, applied to the real and imaginary parts separately."""
    z = np.asarray(z, dtype=np.complex128)
    return np.maximum(z.real, 0.0) + 1j * np.maximum(z.imag, 0.0)


def linf(v):
    """Largest modulus along the last axis."""
    return np.max(np.abs(np.asarray(v)), axis=-1)


def network_forward(net, v):
    """f_w(v) = W2 CReLU(W1 v + b1) + b2 for rows v (..., 3N_d)."""
    W1, b1, W2, b2 = (np.asarray(t, dtype=np.complex128) for t in net)
    v = np.asarray(v, dtype=np.complex128)
    hidden = crelu(v @ W1.T + b1)
    return hidden @ W2.T + b2


def apply_network(net, P):
    """||P||_inf f_w(P / ||P||_inf) per row of P (..., 3N_d); zero rows give 0."""
    P = np.asarray(P, dtype=np.complex128)
    s = linf(P)
    out = np.zeros(P.shape[:-1] + (np.asarray(net[2]).shape[0],), dtype=np.complex128)
    nz = s > 0
    if np.any(nz):
        out[nz] = s[nz][..., None] * network_forward(net, P[nz] / s[nz][..., None])
    return out


def translate_cvfcnn(P, boxes, nets, mode=FAR_ILIST, pairs=None):
    """Stage 2 with networks: E_j = sum_{i in F_j} ||P_i|| f_{c_j-c_i}(P_i/||P_i||).

    ``P`` is (nrhs, n_box, 3N_d); ``nets`` maps an offset tuple (w_x, w_y,
    w_z) to its network (W1, b1, W2, b2).
    """
    P = np.asarray(P, dtype=np.complex128)
    j, i, w = far_pairs(boxes, mode) if pairs is None else pairs
    n_out = np.asarray(next(iter(nets.values()))[2]).shape[0] if nets else P.shape[-1]
    E = np.zeros(P.shape[:2] + (n_out,), dtype=np.complex128)
    if len(j) == 0:
        return E
    uniq, inv = offset_ids(w)
    for o, wv in enumerate(uniq):
        sel = np.nonzero(inv == o)[0]
        net = nets[tuple(int(c) for c in wv)]
        contrib = apply_network(net, P[:, i[sel], :])   # (nrhs, pairs, 3N_d)
        np.add.at(E, (slice(None), j[sel]), contrib)
    return E


def permuted_network(net, Pi):
    """Network of the vector M w from the network of w, where Pi is the signed
    DOF permutation of M: f_{Mw}(v) = Pi f_w(Pi^T v), i.e. W1 Pi^T, b1,
    Pi W2, Pi b2 (Pi is real and orthogonal)."""
    W1, b1, W2, b2 = (np.asarray(t, dtype=np.complex128) for t in net)
    Pi = np.asarray(Pi, dtype=np.float64)
    return W1 @ Pi.T, b1.copy(), Pi @ W2, Pi @ b2


def relative_error(O, E):
    """Eq. 18-19: ||O - E||_2 / ||E||_2 per row."""
    O = np.asarray(O, dtype=np.complex128)
    E = np.asarray(E, dtype=np.complex128)
    return np.linalg.norm(O - E, axis=-1) / np.linalg.norm(E, axis=-1)
