"""Shared helpers of the GPU parity tests."""
import sys

import numpy as np
import pytest
import torch

# Parity bars: FP32 GPU results against the FP64 oracle.
FWD_TOL = 1e-6      # relative L2 per signal and level
GRAD_TOL = 1e-5     # relative L2 of gradients


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    nr = np.linalg.norm(ref)
    d = np.linalg.norm(got - ref)
    if nr == 0:
        return 0.0 if d == 0 else float("inf")
    return float(d / nr)


def worst_level_err(Y_gpu: np.ndarray, Y_ref: np.ndarray) -> float:
    """Worst relative L2 over levels (rows of an (m, N) array)."""
    return max(rel_l2(Y_gpu[i], Y_ref[i]) for i in range(Y_ref.shape[0]))


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()
