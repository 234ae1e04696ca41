"""FP16 storage (binary16 fields, FP32 arithmetic) against the FP64 oracle.

Two bars for every result:
  * against the oracle on the original FP64 inputs: relative 2-norm <= 2e-3;
  * against the oracle on the inputs as the FP16 format holds them (links and
    spinors rounded the way the format prescribes, emulated here in numpy):
    every component within half a binary16 step of its site's largest
    component (the rounding of the stored result), plus an FP32 arithmetic
    slack proportional to the field's largest component (where a site's
    result cancels, its FP32 error is set by its inputs, not by the result).
The second bar shows that the only error beyond FP32 arithmetic is the
rounding of inputs and output to the storage format.
"""

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

from gpu_util import TOL, rel

pytestmark = pytest.mark.gpu

HALF_STEP = 2.0 ** -12   # half a binary16 step on [0.5, 1), relative to the site scale
ARITH = 4e-6             # FP32 arithmetic slack, relative to the field's largest component


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


def _q16(a):
    """FP64 reals rounded once to the nearest binary16 (ties to even)."""
    return a.astype(np.float16).astype(np.float64)


def half_links(U, c12):
    """Links as the FP16 format holds them; with c12 the third row is rebuilt
    from the stored first two as conj(r0 x r1)."""
    Uq = _q16(U.real) + 1j * _q16(U.imag)
    if c12:
        Uq[..., 2, :] = np.conj(np.cross(Uq[..., 0, :], Uq[..., 1, :]))
    return Uq


def half_spinor(psi):
    """Spinor sites as the FP16 format holds them: the 24 reals of a site (in
    binary32) divided by their largest modulus, rounded to binary16, and
    multiplied back, all in binary32."""
    v = np.stack([psi.real, psi.imag], -1).astype(np.float32)
    flat = v.reshape(v.shape[:-3] + (24,))
    m = np.abs(flat).max(-1, keepdims=True)
    # a subnormal site scale is handled with both operands times 2^64 (exact), so
    # its reciprocal does not overflow: the q of unbounded exponents
    k = np.where((m > 0) & (m < np.float32(2.0 ** -126)), np.float32(2.0 ** 64), np.float32(1.0))
    inv = np.zeros_like(m)
    np.divide(np.float32(1.0), m * k, out=inv, where=m > 0)
    q = ((flat * k) * inv).astype(np.float16)
    deq = (q.astype(np.float32) * m).astype(np.float64).reshape(v.shape)
    return deq[..., 0] + 1j * deq[..., 1]


def site_scale(f):
    """Largest modulus of the 24 reals of every site (shape of the site axes)."""
    return np.maximum(np.abs(f.real), np.abs(f.imag)).max(axis=(-2, -1))


def check_rounding_bound(out, ref, arith=ARITH):
    """Every component of out within half a binary16 step of its site scale of
    ref, plus arith times the largest component of ref."""
    scale = site_scale(ref)
    bound = HALF_STEP * 1.001 * scale + arith * float(scale.max())
    err = np.maximum(np.abs((out - ref).real), np.abs((out - ref).imag)).max(axis=(-2, -1))
    ratio = err / np.maximum(bound, 1e-300)
    i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    assert ratio[i] <= 1.0, (f"component error {ratio[i]:.3f} x the binary16 rounding bound at site "
                             f"{i}: error {err[i]:.3e}, site scale {scale[i]:.3e}")


def test_fp16_pack_matches_format():
    dims = (5, 3, 7, 4)  # ragged: 420 sites in 7 blocks of 64
    psi = li.gaussian_spinors(dims, [11, 12])
    psi[0, 0, 0, 0, 1] = 0.0                      # an all-zero site
    psi[1, 1, 2, 1, 3] *= 1e-30                   # a site of tiny values: the scale keeps them
    psi[1, 2, 3, 2, 4, 2, 1] = 1e6                # one entry far above the rest
    g = DeviceGauge(li.unit_gauge(dims), w.WD_FP16)
    back = g.unpack(g.pack(psi, nrhs=2), nrhs=2)
    assert np.array_equal(back, half_spinor(psi))
    assert np.all(back[0, 0, 0, 0, 1] == 0)
    # the format rounds each component to within half a step of its site scale
    check_rounding_bound(back, psi, arith=0.0)


def test_fp16_subnormal_site_scale():
    """A site whose largest component is FP32-subnormal (below 2^-126): its
    reciprocal scale would overflow, so the format scales it by 2^64 first. The
    stored site, the operator's output next to it and a field that is zero
    except for that site must all stay finite and match the oracle."""
    dims = (16, 8, 4, 4)  # t-marching tiles
    U = li.random_gauge(dims, 391)
    psi = li.gaussian_spinor(dims, 392)
    tiny = 1e-39 * li.gaussian_spinor(dims, 393)[1, 2, 3, 4]
    assert np.abs(np.stack([tiny.real, tiny.imag])).max() < 2.0 ** -126
    psi[1, 2, 3, 4] = tiny
    alone = np.zeros_like(psi)
    alone[1, 2, 3, 4] = tiny
    g = DeviceGauge(U, w.WD_FP16)
    for field in (psi, alone):
        src = g.pack(field)
        back = g.unpack(src)
        assert np.all(np.isfinite(back))
        assert np.array_equal(back, half_spinor(field))
        assert rel(back[1, 2, 3, 4], tiny) < 1e-3
        dst = g.spinor()
        w.dslash_apply(g.handle, 0.1, src, dst, w.WD_FP16)
        out = g.unpack(dst)
        assert np.all(np.isfinite(out))
        assert rel(out, oracle.dslash(U, field, 0.1)) <= TOL[w.WD_FP16]


SHAPES = [
    (4, 4, 4, 4),      # one tile, site kernel
    (5, 3, 7, 4),      # ragged tail
    (2, 2, 2, 2),      # extent 2
    (12, 10, 6, 14),   # many tiles + ragged tail
    (32, 32, 16, 11),  # t-marching, ragged last t block
    (24, 24, 4, 8),    # t-marching, 3 y tiles per plane
    (64, 1, 1, 1),     # t-marching, extent 1 in y, z and t
]


@pytest.mark.parametrize("c12", [False, True], ids=["full", "c12"])
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_fp16_parity(dims, c12):
    print(f"case fp16 dims={dims} c12={c12}", flush=True)
    U = li.random_gauge(dims, li.seed_gauge(1))
    psi = li.gaussian_spinor(dims, li.seed_spinor(1))
    g = DeviceGauge(U, w.WD_FP16, c12)
    dst = g.spinor()
    w.dslash_apply(g.handle, 0.1, g.pack(psi), dst, w.WD_FP16)
    out = g.unpack(dst)
    assert rel(out, oracle.dslash(U, psi, 0.1)) <= TOL[w.WD_FP16]
    check_rounding_bound(out, oracle.dslash(half_links(U, c12), half_spinor(psi), 0.1))


def test_fp16_gamma5_near_unity():
    dims = (16, 16, 4, 8)  # t-marching
    U = li.near_unity_gauge(dims, li.seed_gauge(3), 0.3)
    psi = li.gaussian_spinor(dims, li.seed_spinor(3))
    g = DeviceGauge(U, w.WD_FP16, True)
    dst = g.spinor()
    w.dslash_apply(g.handle, 0.05, g.pack(psi), dst, w.WD_FP16, w.WD_FLAG_GAMMA5)
    out = g.unpack(dst)
    ref = oracle.gamma5_apply(oracle.dslash(U, psi, 0.05))
    assert rel(out, ref) <= TOL[w.WD_FP16]
    check_rounding_bound(out, oracle.gamma5_apply(
        oracle.dslash(half_links(U, True), half_spinor(psi), 0.05)))


def test_fp16_production_lattice_sampled():
    """32^3 x 64, full links, FP16 storage: sampled sites against the oracle on
    the original inputs and on the stored inputs, and a bitwise rerun."""
    dims = (32, 32, 32, 64)
    print(f"case fp16 production dims={dims}", flush=True)
    U = li.random_gauge(dims, li.seed_gauge(2))
    psi = li.gaussian_spinor(dims, li.seed_spinor(2))
    g = DeviceGauge(U, w.WD_FP16)
    src = g.pack(psi)
    dst = g.spinor()
    w.dslash_apply(g.handle, 0.1, src, dst, w.WD_FP16)
    out = g.unpack(dst).reshape(-1, 4, 3)
    rng = np.random.default_rng(98)
    sites = np.concatenate([rng.choice(li.volume(dims), 3000, replace=False),
                            np.arange(32), li.volume(dims) - 1 - np.arange(32)])
    assert rel(out[sites], oracle.dslash_sites(U, psi, 0.1, sites)) <= TOL[w.WD_FP16]
    ref_q = oracle.dslash_sites(half_links(U, False), half_spinor(psi), 0.1, sites)
    check_rounding_bound(out[sites], ref_q)
    dst2 = g.spinor()
    w.dslash_apply(g.handle, 0.1, src, dst2, w.WD_FP16)
    torch.cuda.synchronize()
    assert torch.equal(dst, dst2)
