"""GPU parity of dslash_apply against the FP64 oracle, through the C ABI.

Tolerances (relative 2-norm over the whole field, against the FP64 oracle on
the original FP64 inputs): 1e-13 in FP64, 1e-6 in FP32. Lattices span one
tile, several tiles, ragged tails, extents 1 and 2, and the 32^3x64 production
size (every site) in the launch configuration the benchmark times.
"""

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

from gpu_util import PRECS, TOL, HipMem, gpu_dslash, rel

pytestmark = pytest.mark.gpu

SHAPES = [
    (4, 4, 4, 4),      # 256 sites: one tile
    (2, 2, 2, 2),      # extent 2: both hops land on the same neighbour
    (6, 4, 2, 4),      # 192 sites: one partial tile
    (5, 3, 7, 4),      # 420 sites: ragged tail
    (1, 2, 3, 4),      # extent 1: the site is its own neighbour
    (16, 8, 8, 8),     # 8192 sites = 32 tiles: XCD-grouped tile order
    (12, 10, 6, 14),   # 10080 sites: many tiles + ragged tail
    (32, 32, 16, 11),  # t-marching, 3 steps per workgroup, ragged last t block
    (24, 24, 4, 8),    # t-marching, 24-wide rows (3 waves), 3 y tiles per plane
    (64, 2, 2, 3),     # t-marching, extent-2 y and z
    (64, 1, 1, 1),     # t-marching, one site thick in y, z and t: every y/z/t hop lands on itself
    (128, 1, 2, 2),    # t-marching, two-step march with extent-1 y
    (96, 2, 1, 5),     # t-marching, extent-1 z, odd T
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


@pytest.mark.parametrize("c12", [False, True], ids=["full", "c12"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_parity_random_su3(dims, prec, c12):
    print(f"case dims={dims} prec={prec} c12={c12}", flush=True)
    U = li.random_gauge(dims, li.seed_gauge(1))
    psi = li.gaussian_spinor(dims, li.seed_spinor(1))
    ref = oracle.dslash(U, psi, 0.1)
    out = gpu_dslash(U, psi, 0.1, PRECS[prec], c12)
    assert rel(out, ref) <= TOL[PRECS[prec]]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_parity_near_unity_links(prec):
    dims = (8, 6, 4, 6)
    U = li.near_unity_gauge(dims, li.seed_gauge(3), 0.3)
    psi = li.gaussian_spinor(dims, li.seed_spinor(3))
    out = gpu_dslash(U, psi, 0.1, PRECS[prec], True)
    assert rel(out, oracle.dslash(U, psi, 0.1)) <= TOL[PRECS[prec]]


def test_dense_matrix_2222():
    dims = (2, 2, 2, 2)
    U = li.random_gauge(dims, 17)
    psi = li.gaussian_spinor(dims, 18)
    M = oracle.dense_matrix(U, 0.1)
    out = gpu_dslash(U, psi, 0.1)
    assert rel(out.ravel(), M @ psi.ravel()) <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gamma5_flag(prec):
    dims = (4, 6, 2, 4)
    U = li.random_gauge(dims, 23)
    psi = li.gaussian_spinor(dims, 24)
    out = gpu_dslash(U, psi, 0.3, PRECS[prec], flags=w.WD_FLAG_GAMMA5)
    ref = oracle.gamma5_apply(oracle.dslash(U, psi, 0.3))
    assert rel(out, ref) <= TOL[PRECS[prec]]


def test_paper_equation_one_on_gpu():
    """eq. (1)'s hopping term = -2 gamma5 [D(m=-4)] gamma5, with D from the GPU."""
    dims = (4, 4, 2, 6)
    U = li.random_gauge(dims, 29)
    psi = li.gaussian_spinor(dims, 30)
    g5 = oracle.gamma5_apply
    hop = -2.0 * g5(gpu_dslash(U, g5(psi), -4.0))
    assert rel(hop, oracle.hopping_paper(U, psi)) <= 1e-13


def test_free_field_closed_form_on_gpu():
    dims = (6, 4, 8, 4)
    X, Y, Z, T = dims
    n = (1, 3, 2, 1)
    m = 0.1
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    t, z, y, x = np.meshgrid(*(np.arange(k) for k in (T, Z, Y, X)), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    chi = li.complex_gaussian(np.random.default_rng(5), (4, 3))
    psi = phase[..., None, None] * chi
    M = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(
        oracle.GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    out = gpu_dslash(li.unit_gauge(dims), psi, m)
    assert rel(out, phase[..., None, None] * (M @ chi)) <= 1e-13


def test_gamma5_hermiticity_on_gpu():
    dims = (4, 2, 6, 4)
    U = li.random_gauge(dims, 11)
    phi = li.gaussian_spinor(dims, 12)
    psi = li.gaussian_spinor(dims, 13)
    g = DeviceGauge(U, w.WD_FP64)
    g5 = oracle.gamma5_apply
    lhs = np.vdot(phi, gpu_dslash(U, psi, 0.3, gauge=g))
    rhs = np.vdot(g5(gpu_dslash(U, g5(phi), 0.3, gauge=g)), psi)
    assert abs(lhs - rhs) / abs(lhs) <= 1e-13


def test_gauge_covariance_on_gpu():
    from test_oracle import gauge_transform
    dims = (4, 6, 2, 4)
    U = li.random_gauge(dims, 21)
    psi = li.gaussian_spinor(dims, 22)
    om = li.random_su3_field(dims, 23)
    rot = lambda f: np.einsum("...ab,...sb->...sa", om, f)  # noqa: E731
    lhs = gpu_dslash(gauge_transform(U, om), rot(psi), 0.2)
    assert rel(lhs, rot(gpu_dslash(U, psi, 0.2))) <= 1e-13


@pytest.fixture(scope="module")
def production():
    """32^3 x 64 (2,097,152 sites) inputs of the benchmark and the oracle's
    result over the whole field (computed once for the module)."""
    dims = (32, 32, 32, 64)
    U = li.random_gauge(dims, li.seed_gauge(2))
    psi = li.gaussian_spinor(dims, li.seed_spinor(2))
    print("case production: oracle over the whole 32^3x64 field", flush=True)
    return dims, U, psi, oracle.dslash(U, psi, 0.1)


@pytest.mark.parametrize("c12", [False, True], ids=["full", "c12"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_production_lattice_full_field(production, prec, c12):
    """Every site of 32^3 x 64 against the oracle, in the launch the benchmark
    times: the key is tuned first (the tuner keeps only choices whose output
    is bit-identical to the default launch's), then applied."""
    dims, U, psi, ref = production
    print(f"case production dims={dims} prec={prec} c12={c12}", flush=True)
    g = DeviceGauge(U, PRECS[prec], c12)
    src = g.pack(psi)
    dst = g.spinor()
    scratch = g.spinor()
    tuned = w.wd_tune_dslash(g.handle, 1, src, dst, scratch, reps=2)
    assert tuned["eligible"] >= 1
    assert w.wd_tune_lookup(dims, g.prec, c12, 1) is not None
    w.dslash_apply(g.handle, 0.1, src, dst, g.prec)
    out = g.unpack(dst)
    assert rel(out, ref) <= TOL[PRECS[prec]]
    # every site: its largest error against its largest component (FP16 storage
    # rounds each input site to 11 bits of its own largest component)
    site_err = np.abs(out - ref).max(axis=(-2, -1)) / np.abs(ref).max(axis=(-2, -1))
    assert float(site_err.max()) <= (10 if prec == "fp16" else 1e3) * TOL[PRECS[prec]]
    # the second application is bitwise identical (no atomics, fixed order)
    dst2 = g.spinor()
    w.dslash_apply(g.handle, 0.1, src, dst2, g.prec)
    torch.cuda.synchronize()
    assert torch.equal(dst, dst2)


def test_links_beyond_4_gib():
    """48^3 x 72 in FP64 (7,962,624 sites): the packed links take 4.59 GB, more
    than 32-bit buffer offsets reach, so the operator must read them through
    plain pointers. Sampled sites, among them the last ones (whose t links lie
    beyond 4 GiB in the packed field), against the oracle."""
    dims = (48, 48, 48, 72)
    assert w.wd_gauge_bytes(dims, w.WD_FP64, 0) > 1 << 32
    print(f"case dims={dims} fp64: links beyond 4 GiB", flush=True)
    U = li.random_gauge(dims, li.seed_gauge(5))
    psi = li.gaussian_spinor(dims, li.seed_spinor(5))
    g = DeviceGauge(U, w.WD_FP64)
    src = g.pack(psi)
    dst = g.spinor()
    w.dslash_apply(g.handle, 0.1, src, dst, w.WD_FP64)
    out = g.unpack(dst).reshape(-1, 4, 3)
    V = li.volume(dims)
    rng = np.random.default_rng(55)
    sites = np.concatenate([rng.choice(V, 2000, replace=False), np.arange(64), V - 1 - np.arange(64)])
    assert rel(out[sites], oracle.dslash_sites(U, psi, 0.1, sites)) <= TOL[w.WD_FP64]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pack_roundtrip_exact(prec):
    dims = (5, 3, 7, 4)
    psi = li.gaussian_spinors(dims, [1, 2, 3])
    g = DeviceGauge(li.unit_gauge(dims), PRECS[prec])
    back = g.unpack(g.pack(psi), nrhs=3)
    expect = psi if prec == "fp64" else psi.astype(np.complex64).astype(np.complex128)
    assert np.array_equal(back, expect)


def test_empty_nrhs_is_noop():
    dims = (4, 4, 4, 4)
    g = DeviceGauge(li.unit_gauge(dims), w.WD_FP64)
    buf = g.spinor(1)
    assert w.wd_spinor_import(g.handle, buf, w.WD_FP64, 0, buf) == w.WD_OK


# ------------------------------------------------------------- error paths

def _code(fn, *a, **k):
    with pytest.raises(w.WilsonError) as e:
        fn(*a, **k)
    return e.value.code


def test_error_paths():
    dims = (4, 4, 4, 4)
    g = DeviceGauge(li.random_gauge(dims, 1), w.WD_FP64)
    a = g.spinor()
    b = g.spinor()
    host = torch.empty_like(a, device="cpu")
    assert _code(w.dslash_apply, g.handle, 0.1, host, b, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply, g.handle, 0.1, a, a, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply, g.handle, 0.1, a, b, w.WD_FP32) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply, g.handle, 0.1, a, b, w.WD_FP16) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply, g.handle, 0.1, a, b, 5) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply, g.handle, 0.1, a, b, w.WD_FP64, flags=4) == w.WD_ERR_INVALID_ARG
    assert _code(w.dslash_apply, None, 0.1, a, b, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    # a buffer that ends before the field does
    need = w.wd_spinor_bytes(dims, w.WD_FP64, 1)
    small = HipMem(need // 2)
    try:
        assert _code(w.dslash_apply, g.handle, 0.1, a, small.value, w.WD_FP64) == w.WD_ERR_INVALID_ARG
    finally:
        small.free()
    Ud = torch.zeros((4, 4, 4, 4, 4, 3, 3), dtype=torch.complex128, device="cuda")
    buf = torch.empty(w.wd_gauge_bytes(dims, w.WD_FP64), dtype=torch.uint8, device="cuda")
    assert _code(w.wd_gauge_import, (4, 4, 0, 4), Ud, w.WD_FP64, 0, buf) == w.WD_ERR_SHAPE
    assert _code(w.wd_gauge_import, dims, Ud, w.WD_FP64, 0, buf,
                 dst_bytes=buf.numel() - 1) == w.WD_ERR_INVALID_ARG
    assert _code(w.wd_gauge_import, dims, Ud.cpu(), w.WD_FP64, 0, buf) == w.WD_ERR_INVALID_ARG
    assert _code(w.wd_gauge_import, dims, Ud, 7, 0, buf) == w.WD_ERR_INVALID_ARG
    assert w.wd_gauge_release(None) == w.WD_OK
