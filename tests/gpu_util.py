"""Helpers for GPU parity tests: device copies of seeded problems and a context."""
import numpy as np
import pytest


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU (select them with -m gpu on a machine with an MI355X)"
    return torch


def dev(a, dtype=None):
    torch = torch_cuda()
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b, axis=0):
    """Norm-wise relative error per column (axis=0) or overall (axis=None)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if axis is None:
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return np.linalg.norm(a - b, axis=axis) / np.maximum(np.linalg.norm(b, axis=axis), 1e-300)


class GpuProblem:
    """A seeded problem with its device arrays and the binding's Problem."""

    def __init__(self, p):
        from paper_1602_06693_amd import binding
        self.p = p
        self.X = dev(p.X)
        self.prob = binding.Problem(self.X, p.lengthscales, p.sigma2, p.lam)
        self.B = dev(p.B)
        self.idx = dev(p.idx)


@pytest.fixture(scope="module")
def ctx():
    from paper_1602_06693_amd import binding
    torch = torch_cuda()
    torch.cuda.set_device(0)
    c = binding.pkm_create(0, binding.current_stream_handle())
    yield c
    torch.cuda.synchronize()
    binding.pkm_destroy(c)
