"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
(via the thin torch binding) and compare with the FP64 oracle."""
import os
import sys

import numpy as np

TOL = 1e-5          # relative L2, FP32 path vs FP64 oracle (stated target)


def require_gpu():
    import torch
    from paper_2008_02478_amd import lib
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible GPU")
    if not os.path.exists(lib.LIB_PATH):
        raise RuntimeError("libdemag.so is not built")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def max_cell(a, b):
    """Largest per-cell error, max over cells of |a - b| (the 3-vector norm),
    relative to the largest cell value max |b|: a point-wise check beside
    the aggregate rel-L2."""
    a = np.asarray(a, np.float64).reshape(3, -1)
    b = np.asarray(b, np.float64).reshape(3, -1)
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


def to_dev(x, torch):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
