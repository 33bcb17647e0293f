"""Helpers shared by the GPU tests (no method arithmetic)."""
import sys

import numpy as np


def rel_l2(got, ref):
    """Relative l2 error ||got - ref|| / ||ref|| (the Eq. 18-19 form)."""
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(got) - ref) / np.linalg.norm(ref))


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
