"""Seeded synthetic inputs for the Wilson-Dirac operator.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws input fields; it holds none of the operator's arithmetic.

Canonical layout (C order, x fastest), complex128:
  spinor  psi[T][Z][Y][X][spin 4][colour 3]
  gauge   U  [T][Z][Y][X][mu 4][row 3][col 3]   (mu = 0,1,2,3 <-> x,y,z,t)

``dims`` is always given as (X, Y, Z, T).

Random-number recipe (the paper prints no workload data; these stand in for
the Wilson-fermion lattices it describes in Sec. II-A):
  * complex Gaussian: real and imaginary parts i.i.d. N(0,1), drawn as
    ``standard_normal((..., 2))`` from ``numpy.random.default_rng(seed)`` in
    canonical order, one t-slab at a time (identical to one big draw);
  * random SU(3): Gram-Schmidt of a complex Gaussian 3x3 on rows 0 and 1,
    third row = conj(r0 x r1), so that det U = 1 exactly in exact arithmetic;
  * near-unity SU(3): U = exp(i eps H) with H the traceless Hermitian part of
    a complex Gaussian 3x3, evaluated through its eigen-decomposition.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "lattice_shape", "complex_gaussian", "gaussian_spinor",
    "gaussian_spinors", "random_su3_matrices", "near_unity_su3_matrices",
    "random_gauge", "near_unity_gauge", "unit_gauge", "random_su3_field",
    "seed_gauge", "seed_spinor", "seed_transform",
]


def volume(dims) -> int:
    X, Y, Z, T = (int(d) for d in dims)
    return X * Y * Z * T


def lattice_shape(dims) -> tuple:
    """Array shape of the site axes, slowest first: (T, Z, Y, X)."""
    X, Y, Z, T = (int(d) for d in dims)
    if min(X, Y, Z, T) < 1:
        raise ValueError(f"lattice extents must be >= 1, got {dims}")
    return (T, Z, Y, X)


# Seeds for configuration n (1-based): gauge, right-hand side k, gauge transform.
def seed_gauge(n: int) -> int:
    return 1000 * n + 1


def seed_spinor(n: int, k: int = 0) -> int:
    return 1000 * n + 100 + k


def seed_transform(n: int) -> int:
    return 1000 * n + 900


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    z = rng.standard_normal(tuple(shape) + (2,))
    return z[..., 0] + 1j * z[..., 1]


def _slabbed(dims, per_site_shape, seed, make):
    """Fill a field one t-slab at a time from one generator stream."""
    T, Z, Y, X = lattice_shape(dims)
    rng = np.random.default_rng(seed)
    out = None
    for t in range(T):
        slab = make(rng, (Z, Y, X) + tuple(per_site_shape))
        if out is None:
            out = np.empty((T,) + slab.shape, dtype=np.complex128)
        out[t] = slab
    return out


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """One spinor field psi[T][Z][Y][X][4][3], complex N(0,1) entries."""
    return _slabbed(dims, (4, 3), seed, complex_gaussian)


def gaussian_spinors(dims, seeds) -> np.ndarray:
    """Several spinor fields stacked on a leading right-hand-side axis."""
    return np.stack([gaussian_spinor(dims, s) for s in seeds])


def random_su3_matrices(rng: np.random.Generator, shape) -> np.ndarray:
    """Haar-like random SU(3) matrices by Gram-Schmidt of Gaussian rows.

    Rows 0 and 1 are orthonormalised; row 2 = conj(r0 x r1). For orthonormal
    r0, r1 this row is orthogonal to both and makes det = |r0 x r1|^2 = 1.
    """
    a = complex_gaussian(rng, tuple(shape) + (3, 3))
    r0 = a[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = a[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def near_unity_su3_matrices(rng: np.random.Generator, shape, eps: float) -> np.ndarray:
    """U = exp(i eps H), H = traceless Hermitian part of a complex Gaussian 3x3."""
    return _exp_i_eps_h(complex_gaussian(rng, tuple(shape) + (3, 3)), eps)


def _exp_i_eps_h(a: np.ndarray, eps: float) -> np.ndarray:
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    lam, v = np.linalg.eigh(h)
    phase = np.exp(1j * eps * lam)
    return (v * phase[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def random_gauge(dims, seed: int) -> np.ndarray:
    """Gauge field U[T][Z][Y][X][4][3][3] of independent random SU(3) links."""
    return _slabbed(dims, (4,), seed, random_su3_matrices)


def near_unity_gauge(dims, seed: int, eps: float = 0.3) -> np.ndarray:
    """Gauge field of links exp(i eps H) close to the identity."""
    return _slabbed(dims, (4,), seed,
                    lambda rng, shape: near_unity_su3_matrices(rng, shape, eps))


def unit_gauge(dims) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    T, Z, Y, X = lattice_shape(dims)
    u = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3_field(dims, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site, Omega[T][Z][Y][X][3][3] (gauge transforms)."""
    return _slabbed(dims, (), seed, random_su3_matrices)
