"""Shared helpers of the GPU parity tests: the same law description is turned
into the oracle's law and the binding's law (inputs only, no arithmetic)."""
import sys

import numpy as np


def flush(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def laws(orc, desc, device, mean=None, stdev=None):
    """desc: ("normal"|"uniform", loc, scale) or ("reparam",) with FP32 numpy
    mean/stdev in the binding's layout ((n, m) for A, (n, p) for B)."""
    import torch
    from paper_1904_00429_amd import Law
    if desc[0] == "normal":
        return orc.Law.normal(desc[1], desc[2]), Law.normal(desc[1], desc[2])
    if desc[0] == "uniform":
        return orc.Law.uniform(desc[1], desc[2]), Law.uniform(desc[1], desc[2])
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    stdev = np.ascontiguousarray(stdev, dtype=np.float32)
    ld = mean.shape[1] if mean.ndim == 2 else 1
    o = orc.Law.reparam(mean.astype(np.float64).ravel(), stdev.astype(np.float64).ravel(), ld)
    g = Law.reparam(torch.from_numpy(mean).to(device), torch.from_numpy(stdev).to(device))
    return o, g


def rel_frob(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
