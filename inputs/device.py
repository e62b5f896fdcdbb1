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


def haar_orthogonal(n: int, seed: int = 0, device="cuda"):
    """Q Haar-distributed orthogonal: QR of a Gaussian matrix with the column
    signs fixed by diag(R) (float64 on `device`)."""
    import torch

    g = torch.randn(n, n, generator=_gen(seed + 11, device), dtype=torch.float64, device=device)
    q, r = torch.linalg.qr(g)
    del g
    q.mul_(torch.sign(torch.diagonal(r))[None, :])
    return q


def spectrum_matrix(q, cond: float):
    """A = Q diag(sv) Q^T with sv log-spaced from 1 to 1/cond."""
    import math

    import torch

    n = q.shape[0]
    sv = torch.logspace(0.0, -math.log10(float(cond)), n, dtype=torch.float64, device=q.device)
    return (q * sv[None, :]) @ q.T.contiguous()


def haar_spectrum(n: int, cond: float, seed: int = 0, device="cuda"):
    """A = Q diag(sv) Q^T, Q Haar orthogonal, sv log-spaced from 1 to 1/cond."""
    return spectrum_matrix(haar_orthogonal(n, seed, device), cond)


def gaussian_rhs(n: int, nrhs: int = 1, seed: int = 1, device="cuda"):
    import torch

    return torch.randn(n, nrhs, generator=_gen(seed + 13, device), dtype=torch.float64, device=device)
