"""FP64 reference Wilson-Dirac operator (test infrastructure only).

Paper: Meyer et al., "SVE-enabling Lattice QCD Codes", Sec. II-A, eq. (1).

Eq. (1) defines the Wilson hopping term acting on a quark field psi^{ia}_x
(spin i = 1..4, colour a = 1..3, site x) with SU(3) links U_{x,mu} and the
constant Dirac matrices gamma_mu:

    D_h psi(x) = sum_mu { U_{x,mu} (1+gamma_mu) psi(x+mu)
                          + U^dag_{x-mu,mu} (1-gamma_mu) psi(x-mu) }.

The operator this library computes is the Wilson-Dirac operator with bare
mass m in the (4+m) normalisation and the opposite gamma sign convention,

    D psi(x) = (4+m) psi(x)
               - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
                              + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ].

Since gamma5 (1 -/+ gamma_mu) gamma5 = 1 +/- gamma_mu, the two are related
exactly by  D_h = 2(4+m) - 2 gamma5 D gamma5  (checked in the tests through
``hopping_paper``). The paper names no gamma basis; the DeGrand-Rossi basis is
used. Boundaries are periodic in all four directions. mu = 0,1,2,3 is
x,y,z,t, and x is the fastest site index.

Layout: psi[T][Z][Y][X][spin][colour], U[T][Z][Y][X][mu][row][col], complex128.
"""

from __future__ import annotations

import numpy as np

# DeGrand-Rossi Dirac matrices gamma_1..gamma_4 (x, y, z, t); Hermitian and
# anticommuting, with gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).
_I = 1j
GAMMA = np.array([
    [[0, 0, 0, _I], [0, 0, _I, 0], [0, -_I, 0, 0], [-_I, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, _I, 0], [0, 0, 0, -_I], [-_I, 0, 0, 0], [0, _I, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)

# gamma5 as the product of the four Dirac matrices (not typed in by hand).
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

_ONE4 = np.eye(4, dtype=np.complex128)


def flops_per_site() -> int:
    """Conventional flop count of the hopping term per site.

    Per direction and hop: the 4->2 spin projection (6 complex adds = 12),
    two 3x3 complex matrix-vector products (2 x 66 = 132); then 24 flops to add
    each of the 8 contributions after the first into the 4x3 accumulator:
    8*12 + 8*132 + 7*24 = 1320. The mass term and epilogue are not counted.
    """
    return 8 * 12 + 8 * 132 + 7 * 24


def _axis(mu: int, site_axis0: int) -> int:
    """Array axis of direction mu: site axes are (t, z, y, x)."""
    return site_axis0 + 3 - mu


def shift(field: np.ndarray, mu: int, step: int, site_axis0: int = 0) -> np.ndarray:
    """field evaluated at x + step*mu_hat, periodic (np.roll by -step)."""
    return np.roll(field, -step, axis=_axis(mu, site_axis0))


def _colour(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)_{s a} = sum_b U_{a b} psi_{s b} at every site."""
    return np.einsum("...ab,...sb->...sa", U, psi)


def _colour_dag(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U^dag psi)_{s a} = sum_b conj(U_{b a}) psi_{s b} at every site."""
    return np.einsum("...ba,...sb->...sa", np.conj(U), psi)


def _spin(G: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(G psi)_{s a} = sum_t G_{s t} psi_{t a} at every site."""
    return np.einsum("st,...ta->...sa", G, psi)


def gamma5_apply(psi: np.ndarray) -> np.ndarray:
    """gamma5 acting on the spin index of a spinor field."""
    return _spin(GAMMA5, psi)


def dslash(U: np.ndarray, psi: np.ndarray, m: float) -> np.ndarray:
    """Wilson-Dirac operator D psi on the whole periodic lattice (module doc).

    The full 4x4 spin matrices (1 -/+ gamma_mu) are applied; no spin
    projection, no reordering, FP64 throughout.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    acc = np.zeros_like(psi)
    for mu in range(4):
        U_mu = U[..., mu, :, :]
        psi_fwd = shift(psi, mu, +1)          # psi(x + mu)
        psi_bwd = shift(psi, mu, -1)          # psi(x - mu)
        U_bwd = shift(U_mu, mu, -1)           # U_mu(x - mu)
        acc += _spin(_ONE4 - GAMMA[mu], _colour(U_mu, psi_fwd))
        acc += _spin(_ONE4 + GAMMA[mu], _colour_dag(U_bwd, psi_bwd))
    return (4.0 + m) * psi - 0.5 * acc


def dslash_dagger(U: np.ndarray, psi: np.ndarray, m: float) -> np.ndarray:
    """The adjoint D^dag psi, from the adjoint of each hop of ``dslash``.

    The forward hop (1-gamma_mu) U_mu(x) psi(x+mu) has as adjoint, seen from
    the output site, (1-gamma_mu) U_mu(x-mu)^dag psi(x-mu) (gamma_mu is
    Hermitian); the backward hop likewise turns into (1+gamma_mu) U_mu(x)
    psi(x+mu). So D^dag is D with the sign of every gamma_mu flipped.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    acc = np.zeros_like(psi)
    for mu in range(4):
        U_mu = U[..., mu, :, :]
        acc += _spin(_ONE4 + GAMMA[mu], _colour(U_mu, shift(psi, mu, +1)))
        acc += _spin(_ONE4 - GAMMA[mu],
                     _colour_dag(shift(U_mu, mu, -1), shift(psi, mu, -1)))
    return (4.0 + m) * psi - 0.5 * acc


def dslash_multi(U: np.ndarray, psis: np.ndarray, masses) -> np.ndarray:
    """D(m_k) psi_k for a stack of right-hand sides psis[k]."""
    return np.stack([dslash(U, p, float(mk)) for p, mk in zip(psis, masses)])


def hopping_paper(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """The hopping term D_h of eq. (1), written as the paper states it:
    U_{x,mu}(1+gamma_mu) psi(x+mu) + U^dag_{x-mu,mu}(1-gamma_mu) psi(x-mu)."""
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)
    for mu in range(4):
        U_mu = U[..., mu, :, :]
        out += _colour(U_mu, _spin(_ONE4 + GAMMA[mu], shift(psi, mu, +1)))
        out += _colour_dag(shift(U_mu, mu, -1),
                           _spin(_ONE4 - GAMMA[mu], shift(psi, mu, -1)))
    return out


def site_index(dims, x, y, z, t):
    """Canonical site index, x fastest: x + X(y + Y(z + Z t))."""
    X, Y, Z, _ = dims
    return x + X * (y + Y * (z + Z * t))


def site_coords(dims, s):
    """Inverse of ``site_index``: (x, y, z, t)."""
    X, Y, Z, _ = dims
    s = np.asarray(s)
    return s % X, (s // X) % Y, (s // (X * Y)) % Z, s // (X * Y * Z)


def dslash_sites(U: np.ndarray, psi: np.ndarray, m: float, sites) -> np.ndarray:
    """D psi at the listed canonical sites only (same definition as ``dslash``).

    For lattices too large to apply the whole operator in a test: each output
    site is computed from its 8 neighbours by explicit periodic coordinates.
    Returns an array of shape (len(sites), 4, 3).
    """
    T, Z, Y, X = psi.shape[:4]
    dims = (X, Y, Z, T)
    ext = (X, Y, Z, T)
    sites = np.asarray(sites, dtype=np.int64)
    c = list(site_coords(dims, sites))
    psi_f = psi.reshape(-1, 4, 3)
    U_f = U.reshape(-1, 4, 3, 3)
    acc = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for mu in range(4):
        cf = list(c)
        cf[mu] = (c[mu] + 1) % ext[mu]
        cb = list(c)
        cb[mu] = (c[mu] - 1) % ext[mu]
        sf = site_index(dims, *cf)
        sb = site_index(dims, *cb)
        acc += _spin(_ONE4 - GAMMA[mu], _colour(U_f[sites, mu], psi_f[sf]))
        acc += _spin(_ONE4 + GAMMA[mu], _colour_dag(U_f[sb, mu], psi_f[sb]))
    return (4.0 + m) * psi_f[sites] - 0.5 * acc


def dense_matrix(U: np.ndarray, m: float) -> np.ndarray:
    """The operator as a dense 12V x 12V matrix, built entry by entry.

    Row/column index I(site, s, a) = 12*site + 3*s + a. Entries are added
    (never assigned) so that on extent-2 directions, where x+mu = x-mu, both
    hops contribute. Pure Python loops: tiny lattices only.
    """
    T, Z, Y, X = U.shape[:4]
    dims = (X, Y, Z, T)
    ext = (X, Y, Z, T)
    V = X * Y * Z * T
    Uf = U.reshape(V, 4, 3, 3)
    M = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for site in range(V):
        coords = [int(v) for v in site_coords(dims, site)]
        for k in range(12):
            M[12 * site + k, 12 * site + k] += 4.0 + m
        for mu in range(4):
            fwd = list(coords)
            fwd[mu] = (coords[mu] + 1) % ext[mu]
            bwd = list(coords)
            bwd[mu] = (coords[mu] - 1) % ext[mu]
            sf = int(site_index(dims, *fwd))
            sb = int(site_index(dims, *bwd))
            Pm = _ONE4 - GAMMA[mu]
            Pp = _ONE4 + GAMMA[mu]
            for s in range(4):
                for t in range(4):
                    for a in range(3):
                        for b in range(3):
                            M[12 * site + 3 * s + a, 12 * sf + 3 * t + b] += (
                                -0.5 * Pm[s, t] * Uf[site, mu, a, b])
                            M[12 * site + 3 * s + a, 12 * sb + 3 * t + b] += (
                                -0.5 * Pp[s, t] * np.conj(Uf[sb, mu, b, a]))
    return M
