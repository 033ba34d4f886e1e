"""Helpers for the GPU tests: device checks and tensor <-> numpy moves."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2505_07158_amd import vcipher  # noqa: F401  (fails loudly without the library)
    return torch.device("cuda:0")


def to_dev(a: np.ndarray, dev) -> torch.Tensor:
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def to_np(t: torch.Tensor) -> np.ndarray:
    a = t.detach().cpu().numpy()
    return a.view(np.uint16) if a.dtype == np.int16 else a
