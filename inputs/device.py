"""Seeded device-side recipes for the full-size workloads (torch on the GPU).

Same distributions as inputs.matrices but drawn with torch's generator on the
device, because building B B^T at n = 16384 on the host would take minutes.
Nothing here factors, solves or pivots.
"""
from __future__ import annotations


def _gen(seed: int, device):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def spd_bbt(n: int, seed: int = 0, device="cuda"):
    """A = B B^T + n I with B ~ N(0, 1) (row-major float64 on `device`)."""
    import torch

    b = torch.randn(n, n, generator=_gen(seed, device), dtype=torch.float64, device=device)
    a = b @ b.T.contiguous()
    del b
    a.diagonal().add_(float(n))
    return a


def uniform01(n: int, seed: int = 0, device="cuda"):
    """Entries uniform in (0, 1) (torch.rand draws [0, 1); exact zeros are lifted)."""
    import torch

    a = torch.rand(n, n, generator=_gen(seed + 7, device), dtype=torch.float64, device=device)
    a.clamp_(min=torch.finfo(torch.float64).tiny)
    return a
