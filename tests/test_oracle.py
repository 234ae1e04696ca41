"""Pins for the CPU oracle: closed forms, invariants and brute force.

None of these checks re-types the oracle's formula. Each one is something the
mathematics of the Wilson-Dirac operator (Sec. II-A, eq. (1) of the paper, in
the (4+m) - H/2 normalisation) fixes independently, and the mutation tests at
the end show that plausible mistakes in the oracle (a flipped gamma, U where
U^dag belongs, a shift in the wrong direction, a dropped factor) fail at least
one of them.
"""

import os

import numpy as np
import pytest

import lattice_inputs as li
import oracle
import oracle.wilson_ref as wr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def inner(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


# ---------------------------------------------------------------- pin helpers
# Each returns a relative error that is ~1e-15 for a correct operator.

def err_free_field(dslash_fn, dims=(6, 4, 8, 4), m=0.1, n=(1, 3, 2, 1), seed=7):
    """Plane wave on unit links: D e^{ipx} chi = e^{ipx}[m + sum(1-cos p) + i sum g sin p] chi."""
    X, Y, Z, T = dims
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    chi = li.complex_gaussian(np.random.default_rng(seed), (4, 3))
    psi = phase[..., None, None] * chi
    M = (m + sum(1 - np.cos(pm) for pm in p)) * np.eye(4) + 1j * sum(
        oracle.GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    expect = phase[..., None, None] * (M @ chi)
    return rel(dslash_fn(li.unit_gauge(dims), psi, m), expect)


def err_gamma5_hermiticity(dslash_fn, dims=(4, 2, 6, 4), m=0.3, seed=11):
    """<phi, D psi> = <g5 D g5 phi, psi> for any gauge field."""
    U = li.random_gauge(dims, seed)
    phi = li.gaussian_spinor(dims, seed + 1)
    psi = li.gaussian_spinor(dims, seed + 2)
    g5 = oracle.gamma5_apply
    lhs = inner(phi, dslash_fn(U, psi, m))
    rhs = inner(g5(dslash_fn(U, g5(phi), m)), psi)
    return abs(lhs - rhs) / abs(lhs)


def gauge_transform(U, omega):
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        om_fwd = oracle.shift(omega, mu, +1)
        out[..., mu, :, :] = omega @ U[..., mu, :, :] @ np.conj(np.swapaxes(om_fwd, -1, -2))
    return out


def err_gauge_covariance(dslash_fn, dims=(4, 6, 2, 4), m=0.2, seed=21):
    """D[U^Omega](Omega psi) = Omega (D[U] psi) for a random SU(3) transform."""
    U = li.random_gauge(dims, seed)
    psi = li.gaussian_spinor(dims, seed + 1)
    omega = li.random_su3_field(dims, seed + 2)
    rot = lambda f: np.einsum("...ab,...sb->...sa", omega, f)  # noqa: E731
    return rel(dslash_fn(gauge_transform(U, omega), rot(psi), m), rot(dslash_fn(U, psi, m)))


def err_point_source(dslash_fn, dims=(5, 4, 6, 3), x0=(1, 3, 0, 2)):
    """Compare with the hand-derived values in tests/golden."""
    rows = np.loadtxt(os.path.join(GOLDEN, "point_source_unit_gauge.txt"))
    X, Y, Z, T = dims
    psi = np.zeros((T, Z, Y, X, 4, 3), dtype=np.complex128)
    psi[x0[3], x0[2], x0[1], x0[0], 0, 0] = 1.0
    expect = np.zeros_like(psi)
    for dx, dy, dz, dt, s, c, re, im in rows:
        x = (x0[0] + int(dx)) % X
        y = (x0[1] + int(dy)) % Y
        z = (x0[2] + int(dz)) % Z
        t = (x0[3] + int(dt)) % T
        expect[t, z, y, x, int(s), int(c)] += re + 1j * im
    return float(np.abs(dslash_fn(li.unit_gauge(dims), psi, 0.1) - expect).max())


# ------------------------------------------------------------ basis and inputs

def test_gamma_basis_clifford_and_chiral():
    G = oracle.GAMMA
    for mu in range(4):
        assert np.allclose(G[mu], G[mu].conj().T, atol=0)          # Hermitian
        for nu in range(4):
            anti = G[mu] @ G[nu] + G[nu] @ G[mu]
            assert np.allclose(anti, 2 * (mu == nu) * np.eye(4), atol=0)
        assert np.allclose(oracle.GAMMA5 @ G[mu], -G[mu] @ oracle.GAMMA5, atol=0)
    # DeGrand-Rossi is a chiral basis: gamma5 = g1 g2 g3 g4 = diag(1, 1, -1, -1).
    assert np.array_equal(oracle.GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))


@pytest.mark.parametrize("kind", ["random", "near_unity"])
def test_generated_links_are_su3(kind):
    dims = (4, 4, 2, 3)
    U = li.random_gauge(dims, 5) if kind == "random" else li.near_unity_gauge(dims, 5, 0.3)
    Ud = np.conj(np.swapaxes(U, -1, -2))
    assert np.abs(U @ Ud - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    if kind == "near_unity":
        dist = np.linalg.norm(U - np.eye(3), axis=(-2, -1))
        assert 0.05 < dist.mean() < 1.0 and dist.max() < 2.5


def test_generator_reproducible_and_gaussian():
    dims = (8, 8, 4, 4)
    a = li.gaussian_spinor(dims, 123)
    assert np.array_equal(a, li.gaussian_spinor(dims, 123))
    assert not np.array_equal(a, li.gaussian_spinor(dims, 124))
    v = np.concatenate([a.real.ravel(), a.imag.ravel()])
    assert abs(v.mean()) < 0.03 and abs(v.var() - 1) < 0.05


def test_flop_convention():
    assert oracle.flops_per_site() == 1320


# --------------------------------------------------------- pins of the operator

def test_free_field_plane_wave():
    assert err_free_field(oracle.dslash) < 1e-14
    assert err_free_field(oracle.dslash, dims=(4, 4, 4, 8), n=(0, 1, 3, 5), m=-0.3) < 1e-14


def test_free_field_special_modes():
    m = 0.37
    chi = li.complex_gaussian(np.random.default_rng(3), (4, 3))
    dims = (4, 2, 6, 8)
    X, Y, Z, T = dims
    const = np.broadcast_to(chi, (T, Z, Y, X, 4, 3)).copy()
    assert rel(oracle.dslash(li.unit_gauge(dims), const, m), m * const) < 1e-14
    t, z, y, x = np.meshgrid(*(np.arange(n) for n in (T, Z, Y, X)), indexing="ij")
    sign = ((-1.0) ** (x + y + z + t))[..., None, None]
    pi_mode = sign * const
    assert rel(oracle.dslash(li.unit_gauge(dims), pi_mode, m), (m + 8) * pi_mode) < 1e-14


def test_point_source_golden():
    assert err_point_source(oracle.dslash) < 1e-15


def test_point_source_extent_two_double_hop():
    # On an extent-2 direction x0+mu = x0-mu: both hops land there, -1/2[(1-g)+(1+g)]e = -e.
    dims = (2, 2, 2, 2)
    psi = np.zeros((2, 2, 2, 2, 4, 3), dtype=np.complex128)
    psi[0, 0, 0, 0, 1, 2] = 1.0
    out = oracle.dslash(li.unit_gauge(dims), psi, 0.0)
    for mu in range(4):
        idx = [0, 0, 0, 0]
        idx[3 - mu] = 1
        site = out[tuple(idx)]
        expect = np.zeros((4, 3), dtype=complex)
        expect[1, 2] = -1.0
        assert np.abs(site - expect).max() < 1e-15


def test_gamma5_hermiticity():
    assert err_gamma5_hermiticity(oracle.dslash) < 1e-14


def test_adjoint_is_adjoint():
    dims = (4, 2, 2, 6)
    U = li.random_gauge(dims, 31)
    phi = li.gaussian_spinor(dims, 32)
    psi = li.gaussian_spinor(dims, 33)
    lhs = inner(phi, oracle.dslash(U, psi, 0.15))
    rhs = inner(oracle.dslash_dagger(U, phi, 0.15), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14


def test_gauge_covariance():
    assert err_gauge_covariance(oracle.dslash) < 1e-14


def test_translation_covariance():
    dims = (4, 6, 2, 4)
    U = li.random_gauge(dims, 41)
    psi = li.gaussian_spinor(dims, 42)
    shift = (1, 2, 1, 3)
    roll = lambda f: np.roll(f, shift=(shift[3], shift[2], shift[1], shift[0]),  # noqa: E731
                             axis=(0, 1, 2, 3))
    assert rel(oracle.dslash(roll(U), roll(psi), 0.1), roll(oracle.dslash(U, psi, 0.1))) < 1e-15


def test_mass_shift_and_linearity():
    dims = (2, 4, 4, 2)
    U = li.random_gauge(dims, 51)
    a = li.gaussian_spinor(dims, 52)
    b = li.gaussian_spinor(dims, 53)
    d1 = oracle.dslash(U, a, 0.7) - oracle.dslash(U, a, -0.2)
    assert rel(d1, 0.9 * a) < 1e-14
    ca, cb = 0.3 - 1.1j, -2.0 + 0.5j
    lhs = oracle.dslash(U, ca * a + cb * b, 0.1)
    assert rel(lhs, ca * oracle.dslash(U, a, 0.1) + cb * oracle.dslash(U, b, 0.1)) < 1e-14


def test_paper_equation_one():
    """eq. (1)'s hopping term D_h = gamma5 H gamma5 = 2(4+m) - 2 gamma5 D gamma5."""
    dims = (4, 2, 6, 4)
    U = li.random_gauge(dims, 61)
    psi = li.gaussian_spinor(dims, 62)
    m = 0.1
    g5 = oracle.gamma5_apply
    rhs = 2 * (4 + m) * psi - 2 * g5(oracle.dslash(U, g5(psi), m))
    assert rel(oracle.hopping_paper(U, psi), rhs) < 1e-14
    # m = -4 isolates the pure hopping term -H/2
    assert rel(oracle.hopping_paper(U, psi), -2 * g5(oracle.dslash(U, g5(psi), -4.0))) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (3, 2, 1, 2), (1, 3, 2, 2)])
def test_dense_matrix_brute_force(dims):
    U = li.random_gauge(dims, 71)
    psi = li.gaussian_spinor(dims, 72)
    M = oracle.dense_matrix(U, 0.1)
    assert rel(M @ psi.ravel(), oracle.dslash(U, psi, 0.1).ravel()) < 1e-14
    assert rel(M.conj().T @ psi.ravel(), oracle.dslash_dagger(U, psi, 0.1).ravel()) < 1e-14
    G5 = np.kron(np.eye(li.volume(dims)), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.abs(G5 @ M @ G5 - M.conj().T).max() < 1e-14


@pytest.mark.slow
def test_dense_matrix_brute_force_4444():
    dims = (4, 4, 4, 4)
    U = li.random_gauge(dims, li.seed_gauge(1))
    psi = li.gaussian_spinor(dims, li.seed_spinor(1))
    M = oracle.dense_matrix(U, 0.1)
    assert rel(M @ psi.ravel(), oracle.dslash(U, psi, 0.1).ravel()) < 1e-14


def test_dslash_sites_matches_whole_lattice():
    dims = (5, 3, 4, 6)
    U = li.random_gauge(dims, 81)
    psi = li.gaussian_spinor(dims, 82)
    full = oracle.dslash(U, psi, 0.25).reshape(-1, 4, 3)
    sites = np.random.default_rng(0).choice(li.volume(dims), 50, replace=False)
    assert np.abs(oracle.dslash_sites(U, psi, 0.25, sites) - full[sites]).max() < 1e-14


def test_cg_normal_matches_dense_solve():
    dims = (2, 2, 2, 2)
    U = li.near_unity_gauge(dims, 91, 0.3)
    b = li.gaussian_spinor(dims, 92)
    m = 0.05
    x, iters, res = oracle.cg_normal(U, m, b, tol=1e-12)
    M = oracle.dense_matrix(U, m)
    x_ref = np.linalg.solve(M.conj().T @ M, b.ravel())
    assert res <= 1e-12 and iters > 0
    assert rel(x.ravel(), x_ref) < 1e-9


# ----------------------------------------------------- the pins catch mistakes

def _flip_gamma(monkeypatch, mu):
    g = oracle.GAMMA.copy()
    g[mu] = -g[mu]
    monkeypatch.setattr(wr, "GAMMA", g)


@pytest.mark.parametrize("mu", range(4))
def test_mutation_flipped_gamma_is_caught(monkeypatch, mu):
    _flip_gamma(monkeypatch, mu)
    assert err_free_field(wr.dslash, n=(1, 1, 1, 1)) > 1e-2
    assert err_point_source(wr.dslash) > 0.5


def test_mutation_link_not_daggered_is_caught(monkeypatch):
    monkeypatch.setattr(wr, "_colour_dag", wr._colour)
    assert err_gamma5_hermiticity(wr.dslash) > 1e-2
    assert err_gauge_covariance(wr.dslash) > 1e-2


def test_mutation_transposed_link_is_caught():
    transposed = lambda U, psi, m: oracle.dslash(np.swapaxes(U, -1, -2), psi, m)  # noqa: E731
    assert err_gauge_covariance(transposed) > 1e-2


def test_mutation_shift_direction_is_caught(monkeypatch):
    monkeypatch.setattr(wr, "shift", lambda f, mu, step, a=0: np.roll(f, step, axis=a + 3 - mu))
    assert err_gauge_covariance(wr.dslash) > 1e-2
    assert err_free_field(wr.dslash) > 1e-2


def test_mutation_dropped_half_and_direction_is_caught():
    no_half = lambda U, psi, m: 2 * oracle.dslash(U, psi, m) - (4 + m) * psi  # noqa: E731
    assert err_free_field(no_half) > 1e-2

    def no_t(U, psi, m):
        V = U.copy()
        V[..., 3, :, :] = 0
        return oracle.dslash(V, psi, m)
    assert err_free_field(no_t) > 1e-2
    assert err_point_source(no_t) > 0.4
