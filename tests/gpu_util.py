"""Helpers of the GPU tests: device arrays from host arrays and back."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def log_case(**kw):
    print("CASE " + " ".join("%s=%s" % (k, v) for k, v in kw.items()), flush=True)
