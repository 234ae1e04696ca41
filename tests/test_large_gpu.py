"""A 64^4 lattice (16.8 million sites): byte offsets of the packed fields
pass 2^32 (the FP64 links take 9.7 GB). Inputs are generated on the device;
each sampled output site is checked against the oracle applied to the 3^4
block of sites around it (its eight hops stay inside the block, so the
block's own periodicity never enters)."""

import numpy as np
import pytest
import torch

import lattice_inputs.device as dev
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

from gpu_util import TOL, rel

pytestmark = pytest.mark.gpu

DIMS = (64, 64, 64, 64)


@pytest.fixture(scope="module")
def fields():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    print(f"case large dims={DIMS}: generating on the device", flush=True)
    U = dev.random_gauge(DIMS, 7001)
    psi = dev.gaussian_spinor(DIMS, 7100)
    yield U, psi
    del U, psi
    torch.cuda.empty_cache()


def sample_sites(V, rng):
    return np.concatenate([[0, 1, V // 2, V - 2, V - 1], rng.choice(V, 40, replace=False)])


def block(field, site):
    """The 3^4 block of sites around `site` (periodic in the whole lattice),
    ordered [t][z][y][x], as a host array."""
    X, Y, Z, T = DIMS
    x, y, z, t = site % X, (site // X) % Y, (site // (X * Y)) % Z, site // (X * Y * Z)
    d = torch.arange(-1, 2, device=field.device)
    tt, zz, yy, xx = torch.meshgrid((t + d) % T, (z + d) % Z, (y + d) % Y, (x + d) % X, indexing="ij")
    idx = ((tt * Z + zz) * Y + yy) * X + xx
    flat = field.reshape((-1,) + tuple(field.shape[4:]))
    return flat[idx.reshape(-1)].reshape((3, 3, 3, 3) + tuple(field.shape[4:])).cpu().numpy()


@pytest.mark.parametrize("prec", [w.WD_FP64, w.WD_FP16], ids=["fp64", "fp16"])
def test_large_lattice_sampled(fields, prec):
    U, psi = fields
    V = DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3]
    print(f"case large dims={DIMS} prec={prec}", flush=True)
    g = DeviceGauge(U, prec)
    src = g.pack(psi)
    dst = g.spinor()
    w.dslash_apply(g.handle, 0.1, src, dst, prec)
    out = torch.empty_like(psi)
    w.wd_spinor_export(g.handle, dst, prec, 1, out)
    torch.cuda.synchronize()
    sites = sample_sites(V, np.random.default_rng(17))
    got = out.reshape(-1, 4, 3)[torch.as_tensor(sites, device=out.device)].cpu().numpy()
    ref = np.stack([oracle.dslash(block(U, s), block(psi, s), 0.1)[1, 1, 1, 1] for s in sites])
    assert rel(got, ref) <= TOL[prec]
    del g, src, dst, out
