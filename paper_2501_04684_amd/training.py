"""Offline training of the translation networks (Sec. 3, first stage).

One complex-valued network per orbit of translation vectors under the 48
rotations and mirrors of the cube (Sec. 2.2 counts 16 orbits among the 316
vectors of the interaction list); the network of any other vector of the
orbit is the representative's with its inputs and outputs permuted (the
signed DOF permutation of the symmetry), which is exact for the operators
themselves: G_{Mw} = Pi_M G_w Pi_M^T.

Training follows the paper's first stage: inputs are box vectors with real
and imaginary parts uniform in [-1, 1], divided by their l-inf norm (largest
modulus); labels are the DGFA products G_w v with G_w evaluated in FP64 by
the library (``ubf_plan_operator``); Adam on the mean squared error; the
error reported is Eq. 18 (relative l2 per test vector, mean and standard
deviation as in Table 1). The second stage (vectors from an RWG sphere
mesh) needs a mesh that is not available and is not done.

This is preprocessing: it uses PyTorch autograd on the host or a GPU and is
never on the product's path; the trained weights go to the library through
``ubf_plan_set_networks``.

    python -m paper_2501_04684_amd.training --n-d 4 --a 0.125 --hidden 50 \\
        --out networks.npz
"""
from __future__ import annotations

import argparse
import itertools
import math
import time

import numpy as np

from . import plan_create, plan_destroy, plan_offsets, plan_operator


def cube_symmetries() -> list[np.ndarray]:
    """The 48 signed 3x3 permutation matrices."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), dtype=np.int64)
            M[np.arange(3), perm] = signs
            out.append(M)
    return out


def representative(w) -> tuple[tuple[int, int, int], np.ndarray]:
    """(r, M) with r = |w| sorted in descending order and M r = w."""
    w = np.asarray(w, dtype=np.int64)
    order = np.argsort(-np.abs(w), kind="stable")     # r[j] = |w[order[j]]|
    r = np.abs(w)[order]
    M = np.zeros((3, 3), dtype=np.int64)
    for j, i in enumerate(order):
        M[i, j] = -1 if w[i] < 0 else 1
    return tuple(int(v) for v in r), M


def dof_permutation(M: np.ndarray, n_d: int) -> np.ndarray:
    """Signed permutation of a box's 3 n_d^3 dipole coefficients under M:
    the site at centred lattice position c moves to M c and its moment p to
    M p (site s = (m_x n_d + m_y) n_d + m_z, coefficient 3 s + alpha)."""
    m = np.indices((n_d, n_d, n_d)).reshape(3, -1).T          # sites in index order
    c = 2 * m - (n_d - 1)
    c_new = c @ M.T
    m_new = (c_new + (n_d - 1)) // 2
    s_new = (m_new[:, 0] * n_d + m_new[:, 1]) * n_d + m_new[:, 2]
    n = 3 * n_d ** 3
    Pi = np.zeros((n, n))
    for s, t in enumerate(s_new):
        Pi[3 * t:3 * t + 3, 3 * s:3 * s + 3] = M
    return Pi


def interaction_list_offsets() -> np.ndarray:
    """The 316 vectors of [-3, 3]^3 outside [-1, 1]^3 (Sec. 2.2)."""
    g = np.array(list(itertools.product(range(-3, 4), repeat=3)))
    return g[np.abs(g).max(axis=1) >= 2]


def operators_for(offsets, a: float, k: float, n_d: int) -> dict:
    """G_w in FP64 from the library for each vector of ``offsets``: a plan
    over a cube of boxes large enough to hold every vector supplies them."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n = int(np.abs(offsets).max()) + 1
    boxes = np.indices((n, n, n)).reshape(3, -1).T.astype(np.int32)
    plan = plan_create(boxes, a, k, n_d, "full")
    try:
        have = {tuple(int(c) for c in w): o for o, w in enumerate(plan_offsets(plan))}
        return {tuple(int(c) for c in w): plan_operator(plan, have[tuple(int(c) for c in w)])
                for w in offsets}
    finally:
        plan_destroy(plan)


def train_network(G: np.ndarray, hidden: int = 50, epochs: int = 300, n_train: int = 20000,
                  n_test: int = 2000, batch: int = 256, lr: float = 3e-3, seed: int = 0,
                  device: str = "cpu") -> dict:
    """Fit f(v) = W2 CReLU(W1 v + b1) + b2 to v -> G v on l-inf normalised
    uniform inputs. Returns complex64 weights and the Eq. 18 test error."""
    import torch
    gen = torch.Generator().manual_seed(seed)
    rng = np.random.default_rng(seed)
    n = G.shape[1]

    def sample(count):
        x = rng.uniform(-1, 1, (count, n)) + 1j * rng.uniform(-1, 1, (count, n))
        v = x / np.abs(x).max(axis=1, keepdims=True)
        return v, v @ G.T

    v_tr, t_tr = sample(n_train)
    v_te, t_te = sample(n_test)
    scale = float(np.sqrt(np.mean(np.abs(t_tr) ** 2)))   # labels scaled to O(1)
    dev = torch.device(device)
    as_t = lambda a: torch.tensor(a, dtype=torch.complex64, device=dev)
    V, T = as_t(v_tr), as_t(t_tr / scale)
    Vt, Tt = as_t(v_te), as_t(t_te / scale)
    W1 = (torch.randn(hidden, n, dtype=torch.complex64, generator=gen) / math.sqrt(n)).to(dev)
    W2 = (torch.randn(n, hidden, dtype=torch.complex64, generator=gen) / math.sqrt(hidden)).to(dev)
    b1 = torch.zeros(hidden, dtype=torch.complex64, device=dev)
    b2 = torch.zeros(n, dtype=torch.complex64, device=dev)
    params = [p.requires_grad_() for p in (W1, b1, W2, b2)]

    def forward(v):
        z = v @ W1.T + b1
        return torch.complex(torch.relu(z.real), torch.relu(z.imag)) @ W2.T + b2

    opt = torch.optim.Adam(params, lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, epochs, eta_min=lr * 3e-3)
    for _ in range(epochs):
        perm = torch.randperm(n_train, generator=gen).to(dev)
        for i in range(0, n_train, batch):
            idx = perm[i:i + batch]
            loss = (forward(V[idx]) - T[idx]).abs().pow(2).mean()
            opt.zero_grad()
            loss.backward()
            opt.step()
        sched.step()
    with torch.no_grad():
        err = ((forward(Vt) - Tt).abs().pow(2).sum(1).sqrt()
               / Tt.abs().pow(2).sum(1).sqrt()).cpu().numpy()
    host = lambda p: p.detach().cpu().numpy().astype(np.complex64)
    return {"W1": host(W1), "b1": host(b1), "W2": host(W2) * np.float32(scale),
            "b2": host(b2) * np.float32(scale), "err_mean": float(err.mean()),
            "err_std": float(err.std())}


def networks_for_plan(plan, orbit_nets: dict, n_d: int) -> tuple:
    """Per-offset weights in the plan's offset order from the orbit
    representatives' networks: W1 Pi^T, b1, Pi W2, Pi b2."""
    offs = plan_offsets(plan)
    out = [[], [], [], []]
    for w in offs:
        r, M = representative(w)
        net = orbit_nets[r]
        Pi = dof_permutation(M, n_d)
        out[0].append(net["W1"] @ Pi.T)
        out[1].append(net["b1"])
        out[2].append(Pi @ net["W2"])
        out[3].append(Pi @ net["b2"])
    return tuple(np.stack(t).astype(np.complex64) for t in out)


def save(path: str, nets: dict, meta: dict):
    reps = sorted(nets)
    np.savez(path, reps=np.array(reps, dtype=np.int32),
             W1=np.stack([nets[r]["W1"] for r in reps]),
             b1=np.stack([nets[r]["b1"] for r in reps]),
             W2=np.stack([nets[r]["W2"] for r in reps]),
             b2=np.stack([nets[r]["b2"] for r in reps]),
             err_mean=np.array([nets[r]["err_mean"] for r in reps]),
             err_std=np.array([nets[r]["err_std"] for r in reps]),
             **{k: np.array(v) for k, v in meta.items()})


def load(path: str) -> tuple[dict, dict]:
    """(orbit networks keyed by representative, metadata)."""
    z = np.load(path, allow_pickle=False)
    nets = {tuple(int(c) for c in r): {"W1": z["W1"][i], "b1": z["b1"][i], "W2": z["W2"][i],
                                       "b2": z["b2"][i], "err_mean": float(z["err_mean"][i]),
                                       "err_std": float(z["err_std"][i])}
            for i, r in enumerate(z["reps"])}
    meta = {k: z[k].item() for k in ("a", "k", "n_d", "hidden", "epochs") if k in z}
    return nets, meta


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n-d", type=int, default=4)
    ap.add_argument("--a", type=float, default=0.125, help="box side in wavelengths")
    ap.add_argument("--k", type=float, default=2 * math.pi)
    ap.add_argument("--hidden", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--n-train", type=int, default=20000)
    ap.add_argument("--device", default="cpu")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    import torch
    if args.threads:
        torch.set_num_threads(args.threads)
    reps = sorted({representative(w)[0] for w in interaction_list_offsets()}, reverse=True)
    ops = operators_for(reps, args.a, args.k, args.n_d)
    nets = {}
    for i, r in enumerate(reps):
        t0 = time.time()
        nets[r] = train_network(ops[r], args.hidden, args.epochs, args.n_train,
                                seed=1000 + i, device=args.device)
        print(f"{r}: e mean {nets[r]['err_mean']:.3e} std {nets[r]['err_std']:.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    save(args.out, nets, {"a": args.a, "k": args.k, "n_d": args.n_d, "hidden": args.hidden,
                          "epochs": args.epochs})


if __name__ == "__main__":
    main()
