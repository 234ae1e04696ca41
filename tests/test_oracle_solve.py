"""Pins for the oracle's solvers of D x = b and its even-odd preconditioning.

Each check is fixed by something other than the oracle's own formulas: the
Schur complement computed by dense block linear algebra from the brute-force
matrix (itself pinned in test_oracle.py), numpy's dense solve of D x = b, a
closed form on plane waves with unit links, gamma5-hermiticity, and the mass
bookkeeping of the multi-right-hand-side operator. The mutation tests show
that plausible slips (the wrong parity, a sign or a factor of two in the
source or the complement) fail at least one pin.
"""

import numpy as np
import pytest

import lattice_inputs as li
import oracle
import oracle.solve_ref as sr


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def inner(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def parity_rows(dims):
    """Rows of the dense matrix (12 per site) of the even and of the odd sites,
    from the site coordinates (not from the oracle's parity helper)."""
    V = li.volume(dims)
    x, y, z, t = oracle.site_coords(dims, np.arange(V))
    par = (x + y + z + t) % 2
    rows = [np.concatenate([12 * s + np.arange(12) for s in np.nonzero(par == p)[0]])
            for p in (0, 1)]
    return rows


def dense_schur(U, m):
    M = oracle.dense_matrix(U, m)
    dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])
    e, o = parity_rows(dims)
    S = M[np.ix_(o, o)] - M[np.ix_(o, e)] @ np.linalg.solve(M[np.ix_(e, e)], M[np.ix_(e, o)])
    return S, o


def err_schur_dense(schur_fn, dims=(4, 2, 2, 2), m=0.13, seed=301):
    U = li.random_gauge(dims, seed)
    psi = li.gaussian_spinor(dims, seed + 1)
    S, o = dense_schur(U, m)
    expect = S @ psi.ravel()[o]
    got = schur_fn(U, m, psi).ravel()
    return rel(got[o], expect), float(np.abs(np.delete(got, o)).max())


def err_solve_dense(solve_fn, dims=(2, 2, 2, 2), m=0.05, seed=311, tol=1e-12):
    U = li.near_unity_gauge(dims, seed, 0.3)
    b = li.gaussian_spinor(dims, seed + 1)
    x, it, res = solve_fn(U, m, b, tol=tol)
    x_ref = np.linalg.solve(oracle.dense_matrix(U, m), b.ravel())
    return rel(x.ravel(), x_ref), it, res


# ------------------------------------------------------------------ the pins

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2), (2, 2, 4, 2)])
def test_schur_complement_equals_dense_block_elimination(dims):
    err, off = err_schur_dense(sr.schur_odd, dims)
    assert err < 1e-13 and off == 0.0


def test_schur_dagger_equals_dense_adjoint():
    dims = (2, 4, 2, 2)
    U = li.random_gauge(dims, 321)
    psi = li.gaussian_spinor(dims, 322)
    S, o = dense_schur(U, 0.2)
    got = sr.schur_odd_dagger(U, 0.2, psi).ravel()
    assert rel(got[o], S.conj().T @ psi.ravel()[o]) < 1e-13


def test_schur_gamma5_hermiticity():
    dims = (4, 4, 2, 6)
    U = li.random_gauge(dims, 331)
    phi = sr.restrict(li.gaussian_spinor(dims, 332), 1)
    psi = sr.restrict(li.gaussian_spinor(dims, 333), 1)
    g5 = oracle.gamma5_apply
    lhs = inner(phi, sr.schur_odd(U, 0.1, psi))
    rhs = inner(g5(sr.schur_odd(U, 0.1, g5(phi))), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14
    # and the adjoint helper agrees with gamma5 S gamma5
    assert rel(sr.schur_odd_dagger(U, 0.1, phi), g5(sr.schur_odd(U, 0.1, g5(phi)))) < 1e-14


def test_schur_free_field_closed_form():
    """Unit links, psi = P_o e^{ipx} chi: S psi = P_o e^{ipx} [(4+m) - (C^2 - 2iC g.s - s.s)/(4+m)] chi
    with C = sum cos p_mu and s_mu = sin p_mu (H e^{ipx} = e^{ipx}(2C - 2i g.s), and the
    staggered sign (-1)^(x+y+z+t) maps p to p + pi, which flips H's symbol)."""
    dims = (4, 6, 2, 8)
    X, Y, Z, T = dims
    n = (1, 2, 1, 3)
    m = 0.27
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    odd = ((x + y + z + t) % 2 == 1)[..., None, None]
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[..., None, None]
    chi = li.complex_gaussian(np.random.default_rng(341), (4, 3))
    psi = np.where(odd, phase * chi, 0)
    C = sum(np.cos(pm) for pm in p)
    gs = sum(oracle.GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    ss = sum(np.sin(pm) ** 2 for pm in p)
    sym = (4 + m) * np.eye(4) - (C * C * np.eye(4) - 2j * C * gs - ss * np.eye(4)) / (4 + m)
    expect = np.where(odd, phase * (sym @ chi), 0)
    assert rel(sr.schur_odd(li.unit_gauge(dims), m, psi), expect) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_even_odd_solve_equals_dense_solve(dims):
    err, it, res = err_solve_dense(sr.solve_wilson_eo, dims)
    assert err < 1e-9 and it > 0 and res < 1e-10


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 2, 1, 2)])
def test_normal_equation_solve_equals_dense_solve(dims):
    err, it, res = err_solve_dense(sr.solve_wilson, dims)
    assert err < 1e-9 and it > 0 and res < 1e-10


def test_even_odd_and_plain_solves_agree_on_a_larger_lattice():
    dims = (4, 4, 4, 4)
    U = li.near_unity_gauge(dims, 351, 0.3)
    b = li.gaussian_spinor(dims, 352)
    x1, it1, r1 = sr.solve_wilson(U, 0.1, b, tol=1e-11)
    x2, it2, r2 = sr.solve_wilson_eo(U, 0.1, b, tol=1e-11)
    assert r1 < 1e-9 and r2 < 1e-9
    assert rel(x2, x1) < 1e-8
    assert it2 < it1  # the Schur complement is better conditioned


def test_wilson_residual_is_zero_for_the_dense_solution():
    dims = (2, 2, 2, 2)
    U = li.random_gauge(dims, 361)
    b = li.gaussian_spinor(dims, 362)
    x = np.linalg.solve(oracle.dense_matrix(U, 0.3), b.ravel()).reshape(b.shape)
    assert sr.wilson_residual(U, 0.3, b, x) < 1e-13


def test_dslash_multi_assigns_each_mass_to_its_field():
    """Slot k of dslash_multi is D(m_k) psi_k: the same psi in two slots differs by
    (m1 - m2) psi, and every slot equals the brute-force matrix of its own mass."""
    dims = (2, 2, 2, 4)
    U = li.random_gauge(dims, 371)
    a = li.gaussian_spinor(dims, 372)
    c = li.gaussian_spinor(dims, 373)
    masses = [0.9, -0.35, 0.05]
    out = oracle.dslash_multi(U, np.stack([a, a, c]), masses)
    assert rel(out[0] - out[1], (masses[0] - masses[1]) * a) < 1e-14
    for k, psi in enumerate([a, a, c]):
        M = oracle.dense_matrix(U, masses[k])
        assert rel(out[k].ravel(), M @ psi.ravel()) < 1e-14


# ----------------------------------------------------- the pins catch mistakes

def test_mutation_wrong_parity_is_caught(monkeypatch):
    def bad_parity(dims):
        X, Y, Z, T = dims
        t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                                 indexing="ij")
        return (x + y + z) % 2
    monkeypatch.setattr(sr, "parity", bad_parity)
    err, _ = err_schur_dense(sr.schur_odd, (2, 2, 2, 2))
    assert err > 1e-2


def test_mutation_source_sign_is_caught(monkeypatch):
    good = sr.eo_source
    monkeypatch.setattr(sr, "eo_source",
                        lambda U, m, b: 2 * sr.restrict(b, 1) - good(U, m, b))  # b_o - H b_e/(2(4+m))
    err, _, _ = err_solve_dense(sr.solve_wilson_eo)
    assert err > 1e-3


def test_mutation_schur_factor_is_caught(monkeypatch):
    good = sr.schur_odd

    def bad(U, m, psi):  # (4+m) - H H / (2(4+m)) instead of / (4(4+m))
        return 2 * good(U, m, psi) - (4 + m) * sr.restrict(psi, 1)
    err, _ = err_schur_dense(bad)
    assert err > 1e-2


def test_mutation_reconstruction_factor_is_caught(monkeypatch):
    good = sr.eo_reconstruct

    def bad(U, m, b, x_o):  # x_e = (b_e - H x_o / 2) / (4+m)
        x = good(U, m, b, x_o)
        x_e = sr.restrict(x, 0)
        return x + (sr.restrict(b, 0) / (4 + m) - x_e) * 2
    monkeypatch.setattr(sr, "eo_reconstruct", bad)
    err, _, _ = err_solve_dense(sr.solve_wilson_eo)
    assert err > 1e-3


def test_mutation_swapped_masses_in_multi_are_caught():
    dims = (2, 2, 2, 2)
    U = li.random_gauge(dims, 381)
    a = li.gaussian_spinor(dims, 382)
    c = li.gaussian_spinor(dims, 383)
    out = oracle.dslash_multi(U, np.stack([a, c]), [0.4, 0.1][::-1])
    M = oracle.dense_matrix(U, 0.4)
    assert rel(out[0].ravel(), M @ a.ravel()) > 1e-2
