"""Helpers of the GPU tests: device tensors from NumPy, and a printed case name
before each GPU step."""
import sys

import numpy as np


def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def say(*args):
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def host(r):
    """NumPy copies of a binding Result."""
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}
    return type("R", (), out)
