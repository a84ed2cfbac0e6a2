"""Helpers for GPU tests: device copies in column-major layout and result checks
done with torch on the GPU (for sizes where numpy on the host would be slow)."""
import sys

import numpy as np


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def torch_mod():
    import torch

    return torch


def to_dev(a):
    torch = torch_mod()
    a = np.asarray(a, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def to_host(t):
    return np.asfortranarray(t.detach().cpu().numpy())


def gpu_backward_error(H0, S, Z):
    """||H0 - Z S Z^T||_F / ||H0||_F with all three on the GPU (torch matmul,
    float64): a check, not part of the product path."""
    torch = torch_mod()
    nh = torch.linalg.norm(H0)
    R = H0 - Z @ S @ Z.t()
    return float(torch.linalg.norm(R) / nh)


def gpu_orthogonality(Z):
    torch = torch_mod()
    n = Z.shape[0]
    return float(torch.linalg.norm(Z.t() @ Z - torch.eye(n, dtype=Z.dtype, device=Z.device)))
