"""Seeded synthetic inputs generated on a torch device, for lattices too large
to build on the host.

The recipes are those of the host generators (complex Gaussian N(0,1) real and
imaginary parts; random SU(3) by Gram-Schmidt of two Gaussian rows with the
third row conj(r0 x r1)), but the numbers come from torch's generator on the
device, one t-slab at a time: the same seed gives other values than the host
generators. Like the rest of this package it holds none of the operator's
arithmetic.
"""

from __future__ import annotations

import torch

__all__ = ["gaussian_spinor", "random_gauge"]


def _complex_gaussian(gen, shape, device):
    z = torch.randn(tuple(shape) + (2,), generator=gen, dtype=torch.float64, device=device)
    return torch.complex(z[..., 0], z[..., 1])


def _generator(seed, device):
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    return gen


def gaussian_spinor(dims, seed: int, device="cuda") -> torch.Tensor:
    """psi[T][Z][Y][X][4][3], complex128 on the device."""
    X, Y, Z, T = (int(d) for d in dims)
    gen = _generator(seed, device)
    out = torch.empty((T, Z, Y, X, 4, 3), dtype=torch.complex128, device=device)
    for t in range(T):
        out[t] = _complex_gaussian(gen, (Z, Y, X, 4, 3), device)
    return out


def _su3_rows(a):
    r0 = a[..., 0, :]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = a[..., 1, :]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                      r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                      r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], dim=-1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def random_gauge(dims, seed: int, device="cuda") -> torch.Tensor:
    """U[T][Z][Y][X][4][3][3] of independent random SU(3) links, complex128 on the device."""
    X, Y, Z, T = (int(d) for d in dims)
    gen = _generator(seed, device)
    out = torch.empty((T, Z, Y, X, 4, 3, 3), dtype=torch.complex128, device=device)
    for t in range(T):
        out[t] = _su3_rows(_complex_gaussian(gen, (Z, Y, X, 4, 3, 3), device))
    return out
