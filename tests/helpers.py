"""Shared test helpers (no method arithmetic)."""
import numpy as np


def to_dev(a, dev="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# stated parity bounds for the reduced-precision operator (a few unit roundoffs)
PREC_TOL = {"fp64": 1e-12, "fp32": 1e-6, "fp16": 2e-3, "bf16": 2e-2}
