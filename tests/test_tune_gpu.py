"""The autotuner on the GPU: every candidate reproduces the default launch bit
for bit, the kept choice is registered and used, and results do not change."""

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

from gpu_util import PRECS, TOL, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


@pytest.fixture(autouse=True)
def _clean():
    w.wd_tune_reset()
    yield
    w.wd_tune_reset()


@pytest.mark.parametrize("prec,nrhs,c12", [("fp64", 1, False), ("fp32", 4, False), ("fp16", 2, True)])
def test_tuning_keeps_bits_and_registers_choice(prec, nrhs, c12):
    dims = (16, 16, 8, 16)
    print(f"case tune dims={dims} prec={prec} nrhs={nrhs} c12={c12}", flush=True)
    U = li.random_gauge(dims, 41)
    psis = li.gaussian_spinors(dims, [42 + k for k in range(nrhs)])
    g = DeviceGauge(U, PRECS[prec], c12)
    src = g.pack(psis, nrhs=nrhs)
    masses = [0.1] * nrhs
    before = g.spinor(nrhs)
    w.dslash_apply_multi(g.handle, masses, nrhs, src, before, g.prec)
    out, ref = g.spinor(nrhs), g.spinor(nrhs)
    res = w.wd_tune_dslash(g.handle, nrhs, src, out, ref, reps=5)
    print(res)
    assert res["candidates"] >= 4
    assert res["eligible"] == res["candidates"]  # tuned knobs never change a bit
    assert 0 < res["best_us"] <= res["default_us"]
    assert w.wd_tune_lookup(dims, g.prec, c12, nrhs) == (res["tb"], res["gw"], res["group"], res["rb"])
    after = g.spinor(nrhs)
    w.dslash_apply_multi(g.handle, masses, nrhs, src, after, g.prec)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    got = g.unpack(after, nrhs=nrhs)
    got = got if nrhs > 1 else got[None]
    for k in range(nrhs):
        assert rel(got[k], oracle.dslash(U, psis[k], 0.1)) <= TOL[PRECS[prec]]


def test_tuning_site_kernel_lattice_and_errors():
    dims = (260, 2, 2, 2)  # x rows longer than a workgroup: one site per lane, nothing to tune
    g = DeviceGauge(li.unit_gauge(dims), w.WD_FP32)
    a, b, c = g.spinor(), g.spinor(), g.spinor()
    res = w.wd_tune_dslash(g.handle, 1, a, b, c, reps=2)
    assert res["candidates"] == 0
    assert w.wd_tune_lookup(dims, w.WD_FP32, 0, 1) is None
    with pytest.raises(w.WilsonError) as e:
        w.wd_tune_dslash(g.handle, 1, a, a, c)
    assert e.value.code == w.WD_ERR_INVALID_ARG
    with pytest.raises(w.WilsonError) as e:
        w.wd_tune_dslash(g.handle, 1, a, b, c, reps=0)
    assert e.value.code == w.WD_ERR_INVALID_ARG
    with pytest.raises(w.WilsonError) as e:
        w.wd_tune_dslash(g.handle, 17, a, b, c)
    assert e.value.code == w.WD_ERR_UNSUPPORTED


@pytest.mark.parametrize("prec,c12,nrhs,line", [
    ("fp32", False, 4, "16 16 8 16 1 0 4 4 1 0 2"),   # two right-hand sides per lane, 2 lane pairs
    ("fp16", True, 2, "16 16 8 16 2 1 2 16 1 8 2"),   # FP16 storage, 12-real links, XCD runs of 8
])
def test_loaded_choice_two_rhs_per_lane_keeps_bits(tmp_path, prec, c12, nrhs, line):
    dims = (16, 16, 8, 16)
    U = li.near_unity_gauge(dims, 51, 0.3)
    psis = li.gaussian_spinors(dims, [52 + k for k in range(nrhs)])
    masses = [0.05 + 0.1 * k for k in range(nrhs)]
    g = DeviceGauge(U, PRECS[prec], c12)
    src = g.pack(psis, nrhs=nrhs)
    default = g.spinor(nrhs)
    w.dslash_apply_multi(g.handle, masses, nrhs, src, default, g.prec, flags=w.WD_FLAG_GAMMA5)
    f = tmp_path / "tune.txt"
    f.write_text("# wilson dslash launch tuning v2: X Y Z T prec c12 nrhs tb gw group rb\n" + line + "\n")
    w.wd_tune_load(str(f))
    assert w.wd_tune_lookup(dims, g.prec, c12, nrhs)[3] == 2
    tuned = g.spinor(nrhs)
    w.dslash_apply_multi(g.handle, masses, nrhs, src, tuned, g.prec, flags=w.WD_FLAG_GAMMA5)
    torch.cuda.synchronize()
    assert torch.equal(default, tuned)
    got = g.unpack(tuned, nrhs=nrhs)
    for k in range(nrhs):
        ref = oracle.gamma5_apply(oracle.dslash(U, psis[k], masses[k]))
        assert rel(got[k], ref) <= TOL[PRECS[prec]]
