"""Helpers for the GPU tests: device transfer and the case banner."""
import sys

import numpy as np


def banner(*parts):
    print("\n[case]", *parts, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def zeros(shape):
    import torch

    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)
