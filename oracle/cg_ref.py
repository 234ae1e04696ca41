"""FP64 conjugate-gradient solve of the normal equations (test infrastructure).

The paper (Sec. II-A) says that most of the time of a lattice QCD application
goes into iterative solvers such as conjugate gradient, whose dominant cost is
the Dirac operator applied to a quark field. It does not spell out the solver.
The oracle solves D^dag D x = b (D^dag D is Hermitian positive definite for
m > 0) with the textbook conjugate-gradient method of Hestenes and Stiefel,
from x0 = 0, stopping on the recomputed residual ||b - D^dag D x|| / ||b||.
"""

from __future__ import annotations

import numpy as np

from .wilson_ref import dslash, dslash_dagger


def normal_op(U: np.ndarray, m: float, v: np.ndarray) -> np.ndarray:
    """D^dag D v."""
    return dslash_dagger(U, dslash(U, v, m), m)


def _dot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.ravel(), b.ravel()))


def cg_normal(U: np.ndarray, m: float, b: np.ndarray, tol: float = 1e-10,
              max_iter: int = 20000, x0: np.ndarray | None = None):
    """Solve D^dag D x = b; returns (x, iterations, true relative residual).

    Iterates r <- r - alpha A p, x <- x + alpha p, p <- r + beta p with
    alpha = <r,r>/<p,Ap>, beta = <r',r'>/<r,r>, and stops once the iterated
    residual reaches tol * ||b||, confirmed by the true residual.
    """
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.sqrt(_dot(b, b).real)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - normal_op(U, m, x)
    p = r.copy()
    rr = _dot(r, r).real
    it = 0
    while it < max_iter:
        if np.sqrt(rr) <= tol * bnorm:
            true_r = b - normal_op(U, m, x)
            if np.sqrt(_dot(true_r, true_r).real) <= tol * bnorm:
                break
            r = true_r
            p = r.copy()
            rr = _dot(r, r).real
        Ap = normal_op(U, m, p)
        alpha = rr / _dot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = _dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    true_r = b - normal_op(U, m, x)
    rel = float(np.sqrt(_dot(true_r, true_r).real) / bnorm) if bnorm > 0 else 0.0
    return x, it, rel
