"""Even-odd (red-black) preconditioning on the GPU against the oracle, through
the C ABI: the parity split of spinors, the odd-site Schur complement
S = (4+m) - H_oe H_eo / (4(4+m)) (dslash_apply_eo), and the solves of D x = b
(cg_solve_wilson) with full-lattice and even-odd gauge fields.

Operator tolerances as for dslash (relative 2-norm over the field against the
FP64 oracle): 1e-13 FP64, 1e-6 FP32, 2e-3 FP16 storage. Every solution is
checked by the oracle recomputing |b - D x| / |b| in FP64 on the CPU.
"""

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import oracle.solve_ref as sr
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

from gpu_util import PRECS, TOL, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


SHAPES = [
    (2, 2, 2, 2),      # every extent 2: both hops of a direction land on one site
    (4, 4, 4, 4),      # 128 half sites: one partial workgroup
    (6, 4, 2, 8),      # 192 half sites, X/2 = 3
    (12, 10, 6, 14),   # 5040 half sites: many workgroups and a ragged tail
    (16, 8, 8, 8),     # 4096 half sites: 16 workgroups, XCD-contiguous order
    (32, 32, 16, 12),  # 98304 half sites
]


def schur_gpu(U, psis, masses, prec, c12=False, flags=0):
    nrhs = len(masses)
    g = DeviceGauge(U, prec, c12, eo=True)
    src = g.pack_eo(psis if nrhs > 1 else psis[0], 1, nrhs=nrhs)
    dst = g.half_spinor(nrhs)
    tmp = g.half_spinor(nrhs)
    w.dslash_apply_eo(g.handle, masses, nrhs, src, dst, tmp, prec, flags)
    out = g.unpack_eo(dst, 1, nrhs=nrhs)
    return out if nrhs > 1 else out[None]


def test_eo_spinor_split_roundtrip():
    dims = (6, 4, 2, 8)
    psi = li.gaussian_spinors(dims, [501, 502])
    g = DeviceGauge(li.unit_gauge(dims), w.WD_FP64, eo=True)
    def restrict(fields, p):
        return np.stack([sr.restrict(f, p) for f in fields])
    for p in (0, 1):
        back = g.unpack_eo(g.pack_eo(psi, p), p, nrhs=2)
        assert np.array_equal(back, restrict(psi, p))
    g32 = DeviceGauge(li.unit_gauge(dims), w.WD_FP32, eo=True)
    back = g32.unpack_eo(g32.pack_eo(psi, 1), 1, nrhs=2)
    assert np.array_equal(back, restrict(psi.astype(np.complex64).astype(np.complex128), 1))


@pytest.mark.parametrize("c12", [False, True], ids=["full", "c12"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_schur_parity(dims, prec, c12):
    print(f"case schur dims={dims} prec={prec} c12={c12}", flush=True)
    U = li.random_gauge(dims, li.seed_gauge(1))
    masses = [0.1, -0.3, 0.05]
    psis = li.gaussian_spinors(dims, [li.seed_spinor(1, k) for k in range(3)])
    out = schur_gpu(U, psis, masses, PRECS[prec], c12)
    for k, m in enumerate(masses):
        assert rel(out[k], sr.schur_odd(U, m, psis[k])) <= TOL[PRECS[prec]], k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_schur_gamma5_flag_near_unity(prec):
    dims = (8, 6, 4, 4)
    U = li.near_unity_gauge(dims, 511, 0.3)
    psi = li.gaussian_spinor(dims, 512)
    out = schur_gpu(U, psi[None], [0.05], PRECS[prec], True, w.WD_FLAG_GAMMA5)
    assert rel(out[0], oracle.gamma5_apply(sr.schur_odd(U, 0.05, psi))) <= TOL[PRECS[prec]]


def test_schur_dense_block_elimination_2222():
    """S on the GPU equals M_oo - M_oe M_ee^-1 M_eo of the brute-force matrix."""
    from test_oracle_solve import dense_schur
    dims = (2, 2, 2, 2)
    U = li.random_gauge(dims, 521)
    psi = li.gaussian_spinor(dims, 522)
    S, o = dense_schur(U, 0.13)
    out = schur_gpu(U, psi[None], [0.13], w.WD_FP64)[0].ravel()
    assert rel(out[o], S @ psi.ravel()[o]) <= 1e-13


def test_schur_free_field_closed_form_on_gpu():
    """Unit links, odd-site plane wave: the closed form of the oracle's pin."""
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
    out = schur_gpu(li.unit_gauge(dims), psi[None], [m], w.WD_FP64)[0]
    assert rel(out, np.where(odd, phase * (sym @ chi), 0)) <= 1e-13


# ------------------------------------------------------------------ solves

INNER = {"fp64": w.WD_FP64, "fp32": w.WD_FP32, "fp16": w.WD_FP16}


def wilson_solve(U, masses, bs, inner, eo, tol=1e-10, check_every=4, max_iter=20000, x0=None,
                 c12=False):
    nrhs = len(masses)
    ghi = DeviceGauge(U, w.WD_FP64, c12, eo=eo)
    glo = DeviceGauge(U, inner, c12, eo=eo) if inner != w.WD_FP64 else None
    b = ghi.pack(bs, nrhs=nrhs)
    x = ghi.pack(x0, nrhs=nrhs) if x0 is not None else ghi.spinor(nrhs)
    ws = torch.empty(w.wilson_workspace_bytes(ghi.dims, nrhs, inner, eo), dtype=torch.uint8,
                     device="cuda")
    params = dict(tol=tol, max_iter=max_iter, inner=inner, delta=0.1, check_every=check_every,
                  x0_given=int(x0 is not None), use_graph=0)
    rc, stats = w.cg_solve_wilson(ghi.handle, glo.handle if glo else None, masses, nrhs, b, x,
                                  params, ws)
    xs = ghi.unpack(x, nrhs=nrhs)
    return rc, (xs if nrhs > 1 else xs[None]), stats


@pytest.mark.parametrize("eo", [False, True], ids=["plain", "eo"])
@pytest.mark.parametrize("inner", ["fp64", "fp32", "fp16"])
def test_wilson_solve_dense_2222(inner, eo):
    dims = (2, 2, 2, 2)
    U = li.near_unity_gauge(dims, 311, 0.3)
    b = li.gaussian_spinor(dims, 312)
    m = 0.05
    rc, xs, st = wilson_solve(U, [m], b[None], INNER[inner], eo, tol=1e-12)
    assert rc == w.WD_OK, st
    M = oracle.dense_matrix(U, m)
    x_ref = np.linalg.solve(M, b.ravel())
    assert sr.wilson_residual(U, m, b, xs[0]) <= 1e-12
    assert rel(xs[0].ravel(), x_ref) <= np.linalg.cond(M) * 1e-12
    assert abs(st[0]["true_rel_residual"] - sr.wilson_residual(U, m, b, xs[0])) <= 1e-14


@pytest.mark.parametrize("eo", [False, True], ids=["plain", "eo"])
@pytest.mark.parametrize("inner", ["fp64", "fp32", "fp16"])
def test_wilson_solve_matches_oracle(inner, eo):
    dims = (8, 4, 4, 6)
    U = li.near_unity_gauge(dims, 4001, 0.3)
    bs = li.gaussian_spinors(dims, [4100, 4101])
    masses = [0.05, 0.3]
    print(f"case wilson solve dims={dims} inner={inner} eo={eo}", flush=True)
    rc, xs, st = wilson_solve(U, masses, bs, INNER[inner], eo)
    assert rc == w.WD_OK, st
    for k, m in enumerate(masses):
        res = sr.wilson_residual(U, m, bs[k], xs[k])
        assert res <= 1e-10, (k, res)
        assert abs(res - st[k]["true_rel_residual"]) <= 1e-3 * res + 1e-15
        x_ref, _, _ = sr.solve_wilson_eo(U, m, bs[k], tol=1e-12)
        assert rel(xs[k], x_ref) <= 1e-7
        print(k, st[k])


def test_eo_needs_fewer_iterations_and_batches_bitwise():
    dims = (8, 8, 4, 4)
    U = li.near_unity_gauge(dims, 531, 0.3)
    bs = li.gaussian_spinors(dims, [532, 533, 534])
    masses = [0.05, 0.2, 0.5]
    rc, xs, st = wilson_solve(U, masses, bs, w.WD_FP32, True)
    assert rc == w.WD_OK, st
    rc_p, _, st_p = wilson_solve(U, masses, bs, w.WD_FP32, False)
    assert rc_p == w.WD_OK, st_p
    for k in range(3):
        assert st[k]["iters"] < st_p[k]["iters"]
        rc1, x1, st1 = wilson_solve(U, [masses[k]], bs[k][None], w.WD_FP32, True)
        assert rc1 == w.WD_OK
        assert np.array_equal(x1[0], xs[k]) and st1[0]["iters"] == st[k]["iters"]


def test_wilson_solve_24_4_even_odd_fp16():
    """The solver configuration: 24^4, m = 0.05, near-unity links, tol 1e-10."""
    dims = (24, 24, 24, 24)
    U = li.near_unity_gauge(dims, li.seed_gauge(4), 0.3)
    b = li.gaussian_spinor(dims, li.seed_spinor(4))
    m = 0.05
    print("case wilson solve 24^4 eo fp16", flush=True)
    rc, xs, st = wilson_solve(U, [m], b[None], w.WD_FP16, True, check_every=8)
    assert rc == w.WD_OK, st
    res = sr.wilson_residual(U, m, b, xs[0])
    assert res <= 1e-10
    print(st[0], res)


def test_wilson_start_vector_and_c12():
    dims = (8, 4, 4, 4)
    U = li.near_unity_gauge(dims, 541, 0.3)
    b = li.gaussian_spinor(dims, 542)
    x_ref, _, _ = sr.solve_wilson_eo(U, 0.1, b, tol=1e-12)
    x0 = x_ref + 1e-6 * li.gaussian_spinor(dims, 543)
    rc, xs, st = wilson_solve(U, [0.1], b[None], w.WD_FP64, True, x0=x0[None], c12=True)
    assert rc == w.WD_OK, st
    assert sr.wilson_residual(U, 0.1, b, xs[0]) <= 1e-10
    rc2, _, st2 = wilson_solve(U, [0.1], b[None], w.WD_FP64, True, c12=True)
    assert st[0]["iters"] < st2[0]["iters"]  # the start vector was used


def _code(fn, *a, **k):
    with pytest.raises(w.WilsonError) as e:
        fn(*a, **k)
    return e.value.code


def test_eo_error_paths():
    dims = (4, 4, 4, 4)
    U = li.random_gauge(dims, 551)
    geo = DeviceGauge(U, w.WD_FP64, eo=True)
    gfull = DeviceGauge(U, w.WD_FP64)
    a, b, t = geo.half_spinor(), geo.half_spinor(), geo.half_spinor()
    fa, fb = gfull.spinor(), gfull.spinor()
    # layouts are not interchangeable
    assert _code(w.dslash_apply, geo.handle, 0.1, fa, fb, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply_eo, gfull.handle, [0.1], 1, a, b, t, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    # aliasing, mass -4, odd extents
    assert _code(w.dslash_apply_eo, geo.handle, [0.1], 1, a, a, t, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply_eo, geo.handle, [-4.0], 1, a, b, t, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    assert w.wd_gauge_eo_bytes((4, 4, 3, 4), w.WD_FP64) == 0
    Uo = torch.zeros((4, 3, 4, 4, 4, 3, 3), dtype=torch.complex128, device="cuda")
    buf = torch.empty(w.wd_gauge_eo_bytes(dims, w.WD_FP64), dtype=torch.uint8, device="cuda")
    assert _code(w.wd_gauge_import_eo, (4, 4, 3, 4), Uo, w.WD_FP64, 0, buf) == w.WD_ERR_SHAPE
    # the normal-equation solver wants a full-lattice handle
    ws = torch.empty(w.cg_workspace_bytes(dims, 1, w.WD_FP64), dtype=torch.uint8, device="cuda")
    params = dict(tol=1e-10, max_iter=100, inner=w.WD_FP64, delta=0.1, check_every=4, x0_given=0,
                  use_graph=0)
    assert _code(w.cg_solve_normal, geo.handle, None, [0.1], 1, fa, fb, params, ws) == w.WD_ERR_INVALID_ARG
