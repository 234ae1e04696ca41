"""Fused multi-right-hand-side dslash against the oracle (per right-hand side)
and against separate single-right-hand-side launches (bit for bit)."""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

from gpu_util import PRECS, TOL, HipMem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


SHAPES = [(4, 4, 4, 4), (5, 3, 7, 4), (32, 32, 16, 11), (24, 24, 4, 8), (16, 8, 8, 8), (64, 1, 2, 1)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_multi_matches_oracle_and_single(dims, prec):
    nrhs = 5
    print(f"case multi dims={dims} prec={prec}", flush=True)
    U = li.random_gauge(dims, 301)
    psis = li.gaussian_spinors(dims, [310 + k for k in range(nrhs)])
    masses = [0.1, -0.3, 0.5, 0.05, 1.0]
    g = DeviceGauge(U, PRECS[prec])
    src = g.pack(psis, nrhs=nrhs)
    dst = g.spinor(nrhs)
    w.dslash_apply_multi(g.handle, masses, nrhs, src, dst, g.prec)
    out = g.unpack(dst, nrhs=nrhs)
    for k in range(nrhs):
        assert rel(out[k], oracle.dslash(U, psis[k], masses[k])) <= TOL[PRECS[prec]]
    # the same fields one at a time give the same bits
    one = g.spinor(1)
    res = g.spinor(1)
    for k in range(nrhs):
        w.wd_spinor_import(g.handle, torch.from_numpy(psis[k]).cuda(), g.prec, 1, one)
        w.dslash_apply(g.handle, masses[k], one, res, g.prec)
        assert np.array_equal(g.unpack(res), out[k])


def test_multi_gamma5_and_limits():
    dims = (16, 8, 8, 8)
    U = li.random_gauge(dims, 5)
    psis = li.gaussian_spinors(dims, list(range(16)))
    masses = list(np.linspace(-0.5, 0.5, 16))
    g = DeviceGauge(U, w.WD_FP32)
    src = g.pack(psis, nrhs=16)
    dst = g.spinor(16)
    w.dslash_apply_multi(g.handle, masses, 16, src, dst, g.prec, flags=w.WD_FLAG_GAMMA5)
    out = g.unpack(dst, nrhs=16)
    for k in (0, 7, 15):
        ref = oracle.gamma5_apply(oracle.dslash(U, psis[k], masses[k]))
        assert rel(out[k], ref) <= TOL[w.WD_FP32]
    assert w.dslash_apply_multi(g.handle, [], 0, src, dst, g.prec) == w.WD_OK
    with pytest.raises(w.WilsonError) as e:
        w.dslash_apply_multi(g.handle, [0.1] * 17, 17, src, dst, g.prec)
    assert e.value.code == w.WD_ERR_UNSUPPORTED
    with pytest.raises(w.WilsonError) as e:
        w.dslash_apply_multi(g.handle, [0.1, float("nan")], 2, src, dst, g.prec)
    assert e.value.code == w.WD_ERR_INVALID_ARG
    small = HipMem(w.wd_spinor_bytes(dims, w.WD_FP32, 2))  # an exact allocation for 2 fields
    try:
        with pytest.raises(w.WilsonError) as e:
            w.dslash_apply_multi(g.handle, [0.1] * 16, 16, src, small.value, g.prec)
        assert e.value.code == w.WD_ERR_INVALID_ARG
    finally:
        small.free()


@pytest.fixture(scope="module")
def twelve_rhs():
    """24^3 x 48 with 12 Gaussian right-hand sides on near-unity links, and the
    oracle's result for every field (computed once, in threads)."""
    dims = (24, 24, 24, 48)
    nrhs = 12
    U = li.near_unity_gauge(dims, li.seed_gauge(3), 0.3)
    psis = li.gaussian_spinors(dims, [li.seed_spinor(3, k) for k in range(nrhs)])
    masses = [0.1 + 0.02 * k for k in range(nrhs)]
    print("case multi 24^3x48 x12: oracle over every field", flush=True)
    with ThreadPoolExecutor(4) as ex:
        refs = list(ex.map(lambda k: oracle.dslash(U, psis[k], masses[k]), range(nrhs)))
    return dims, U, psis, masses, refs


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp64"])
def test_multi_24_3_48_twelve_rhs_full_field(twelve_rhs, prec):
    """24^3 x 48, 12 right-hand sides with their own masses, near-unity links:
    every site of every field against the oracle, in the tuned launch."""
    dims, U, psis, masses, refs = twelve_rhs
    nrhs = len(masses)
    print(f"case multi 24^3x48 x12 {prec}", flush=True)
    g = DeviceGauge(U, PRECS[prec])
    src = g.pack(psis, nrhs=nrhs)
    dst = g.spinor(nrhs)
    scratch = g.spinor(nrhs)
    w.wd_tune_dslash(g.handle, nrhs, src, dst, scratch, reps=2)
    w.dslash_apply_multi(g.handle, masses, nrhs, src, dst, g.prec)
    out = g.unpack(dst, nrhs=nrhs)
    for k in range(nrhs):
        assert rel(out[k], refs[k]) <= TOL[PRECS[prec]], k
    # several right-hand sides share a workgroup here: still the bits of single launches
    one = g.spinor(1)
    res = g.spinor(1)
    for k in (0, 5, 11):
        w.wd_spinor_import(g.handle, torch.from_numpy(psis[k]).cuda(), g.prec, 1, one)
        w.dslash_apply(g.handle, masses[k], one, res, g.prec)
        assert np.array_equal(g.unpack(res), out[k])
