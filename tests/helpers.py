"""Shared helpers of the GPU parity tests."""
import numpy as np
import pytest
import torch

import oracle


def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def as_prec(a, dtype):
    """The values the device sees, as float64 numpy (float32 rounding applied)."""
    return np.asarray(a, dtype=np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def colrel(got, ref):
    """Per-column normwise relative error ‖got_c − ref_c‖ / ‖ref_c‖."""
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    den = np.linalg.norm(ref, axis=0)
    return np.linalg.norm(got - ref, axis=0) / np.where(den > 0, den, 1.0)


def oracle_rows(X, V, kernel, l, f, s, rows):
    """Rows `rows` (a slice) of K̂·V from the dense oracle block."""
    return oracle.khat_block(X, rows, kernel, l, f, s) @ V


TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def colrel_cond(got, ref, refabs):
    """Per-column error normalised by the magnitude of the summands,
    ‖got_c − ref_c‖ / ‖(|K̂||V|)_c‖: the natural bound of a floating-point
    product, for columns whose result cancels (sum ≪ sum of magnitudes)."""
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    den = np.linalg.norm(np.asarray(refabs).reshape(ref.shape[0], -1), axis=0)
    return np.linalg.norm(got - ref, axis=0) / np.where(den > 0, den, 1.0)
