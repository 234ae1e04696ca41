"""Solving the Wilson system D x = b, plain and even-odd preconditioned
(test infrastructure only).

Sec. II-A of the paper says that iterative solvers such as conjugate gradient
spend most of a lattice QCD run applying the Dirac operator of eq. (1) to a
quark field. The system those solvers face is D x = b with the Wilson-Dirac
operator D (the (4+m) - H/2 normalisation of ``wilson_ref``). The paper spells
out neither the solver nor a preconditioner; this module states two standard
ways to solve it, in FP64 and in the plainest form:

* the normal equations: D^dag D x = D^dag b, solved with conjugate gradient;
* even-odd (red-black) preconditioning. Colour every site by the parity of
  x+y+z+t. On a lattice whose four extents are even, every hop of D joins
  sites of opposite parity, so in the (even, odd) block order

      D = [[ A      , -H_eo/2 ],
           [ -H_oe/2, A       ]],   A = (4+m) on every site,

  where H_pq is the hopping term H = sum_mu [(1-g) U psi(x+mu) +
  (1+g) U^dag psi(x-mu)] restricted to outputs of parity p and inputs of
  parity q. Eliminating the even block leaves the odd-site Schur complement

      S = A - (-H_oe/2) A^{-1} (-H_eo/2) = (4+m) - H_oe H_eo / (4 (4+m)),

  with source  b^_o = b_o - (-H_oe/2) A^{-1} b_e = b_o + H_oe b_e / (2 (4+m)).
  Solving S x_o = b^_o (here through S^dag S x_o = S^dag b^_o) and then

      x_e = A^{-1} (b_e - (-H_eo/2) x_o) = (b_e + H_eo x_o / 2) / (4+m)

  gives the full solution x. S is gamma5-Hermitian like D.

Fields are full-lattice arrays in the canonical layout; a field "of parity p"
is zero on the sites of the other parity.
"""

from __future__ import annotations

import numpy as np

from .wilson_ref import dslash, dslash_dagger, gamma5_apply


def parity(dims) -> np.ndarray:
    """(x + y + z + t) mod 2 on the site axes (T, Z, Y, X)."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return (x + y + z + t) % 2


def _dims_of(field) -> tuple:
    T, Z, Y, X = field.shape[:4]
    return (X, Y, Z, T)


def restrict(field: np.ndarray, p: int) -> np.ndarray:
    """The field on the sites of parity p, zero elsewhere."""
    mask = parity(_dims_of(field)) == p
    return np.where(mask[..., None, None], field, 0)


def hopping(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """H psi = sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)].

    From the definition D = (4+m) - H/2 at m = -4, where D = -H/2.
    """
    return -2.0 * dslash(U, psi, -4.0)


def hopping_dagger(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """H^dag psi, from D^dag = (4+m) - H^dag/2 at m = -4."""
    return -2.0 * dslash_dagger(U, psi, -4.0)


def _check_even(dims):
    if any(d % 2 for d in dims):
        raise ValueError(f"even-odd preconditioning needs even extents, got {dims}")


def schur_odd(U: np.ndarray, m: float, psi: np.ndarray) -> np.ndarray:
    """S psi_o = (4+m) psi_o - H_oe H_eo psi_o / (4(4+m)) for the odd part of psi.

    The result is a field of parity 1 (zero on even sites).
    """
    _check_even(_dims_of(psi))
    psi_o = restrict(np.asarray(psi, dtype=np.complex128), 1)
    t_e = restrict(hopping(U, psi_o), 0)              # H_eo psi_o
    h_o = restrict(hopping(U, t_e), 1)                # H_oe H_eo psi_o
    return (4.0 + m) * psi_o - h_o / (4.0 * (4.0 + m))


def schur_odd_dagger(U: np.ndarray, m: float, psi: np.ndarray) -> np.ndarray:
    """S^dag psi_o = (4+m) psi_o - (H_oe H_eo)^dag psi_o / (4(4+m)).

    (H_oe H_eo)^dag = H_eo^dag H_oe^dag, and the restriction of H^dag to an
    output parity p and input parity q is (H_qp)^dag, so the product is again
    odd -> even -> odd, with H^dag in place of H.
    """
    _check_even(_dims_of(psi))
    psi_o = restrict(np.asarray(psi, dtype=np.complex128), 1)
    t_e = restrict(hopping_dagger(U, psi_o), 0)
    h_o = restrict(hopping_dagger(U, t_e), 1)
    return (4.0 + m) * psi_o - h_o / (4.0 * (4.0 + m))


def eo_source(U: np.ndarray, m: float, b: np.ndarray) -> np.ndarray:
    """b^_o = b_o + H_oe b_e / (2(4+m)) (parity 1)."""
    _check_even(_dims_of(b))
    b = np.asarray(b, dtype=np.complex128)
    return restrict(b, 1) + restrict(hopping(U, restrict(b, 0)), 1) / (2.0 * (4.0 + m))


def eo_reconstruct(U: np.ndarray, m: float, b: np.ndarray, x_o: np.ndarray) -> np.ndarray:
    """The full solution: x_e = (b_e + H_eo x_o / 2) / (4+m), and x_o itself."""
    b = np.asarray(b, dtype=np.complex128)
    x_o = restrict(np.asarray(x_o, dtype=np.complex128), 1)
    x_e = (restrict(b, 0) + 0.5 * restrict(hopping(U, x_o), 0)) / (4.0 + m)
    return x_e + x_o


def _dot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def cg_hpd(apply_a, rhs: np.ndarray, tol: float, max_iter: int = 20000, x0=None):
    """Conjugate gradient (Hestenes-Stiefel) for a Hermitian positive definite
    operator apply_a, from x0 (default 0). Stops once the recomputed residual
    |rhs - A x| is at most tol |rhs|. Returns (x, iterations, relative residual).
    """
    rhs = np.asarray(rhs, dtype=np.complex128)
    norm = np.sqrt(_dot(rhs, rhs).real)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.complex128)
    r = rhs - apply_a(x)
    p = r.copy()
    rr = _dot(r, r).real
    it = 0
    while it < max_iter:
        if np.sqrt(rr) <= tol * norm:
            true_r = rhs - apply_a(x)
            if np.sqrt(_dot(true_r, true_r).real) <= tol * norm:
                break
            r = true_r
            p = r.copy()
            rr = _dot(r, r).real
        ap = apply_a(p)
        alpha = rr / _dot(p, ap).real
        x = x + alpha * p
        r = r - alpha * ap
        rr_new = _dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    true_r = rhs - apply_a(x)
    rel = float(np.sqrt(_dot(true_r, true_r).real) / norm) if norm > 0 else 0.0
    return x, it, rel


def wilson_residual(U: np.ndarray, m: float, b: np.ndarray, x: np.ndarray) -> float:
    """|b - D x| / |b|."""
    r = np.asarray(b, dtype=np.complex128) - dslash(U, x, m)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def solve_wilson(U: np.ndarray, m: float, b: np.ndarray, tol: float = 1e-10,
                 max_iter: int = 20000):
    """x with D x = b through the normal equations D^dag D x = D^dag b.

    Returns (x, CG iterations, |b - D x| / |b|). tol bounds the residual of
    the normal equations relative to |D^dag b|.
    """
    b = np.asarray(b, dtype=np.complex128)
    rhs = dslash_dagger(U, b, m)
    x, it, _ = cg_hpd(lambda v: dslash_dagger(U, dslash(U, v, m), m), rhs, tol, max_iter)
    return x, it, wilson_residual(U, m, b, x)


def solve_wilson_eo(U: np.ndarray, m: float, b: np.ndarray, tol: float = 1e-10,
                    max_iter: int = 20000):
    """x with D x = b by even-odd preconditioning (module doc): CG on
    S^dag S x_o = S^dag b^_o, then the even sites from x_o.

    Returns (x, CG iterations, |b - D x| / |b|). tol bounds the residual of
    the odd-site normal equations relative to |S^dag b^_o|.
    """
    b = np.asarray(b, dtype=np.complex128)
    rhs = schur_odd_dagger(U, m, eo_source(U, m, b))
    x_o, it, _ = cg_hpd(lambda v: schur_odd_dagger(U, m, schur_odd(U, m, v)), rhs, tol, max_iter)
    x = eo_reconstruct(U, m, b, x_o)
    return x, it, wilson_residual(U, m, b, x)


def gamma5_schur(U: np.ndarray, m: float, psi: np.ndarray) -> np.ndarray:
    """gamma5 S psi_o, the Hermitian form of the Schur complement."""
    return gamma5_apply(schur_odd(U, m, psi))
