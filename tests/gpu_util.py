"""Helpers for the GPU tests: device placement and the native binding."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_06326_amd import native  # raises if the library is missing
    return native


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
