"""cg_solve_normal_noalloc (static device workspace, no allocation) against
cg_solve_normal with a caller workspace, through the C ABI: the two give the
same solution bits and statistics, on two calls in a row, the second with a
smaller input; limits and unsupported options are errors, not faults."""

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


def _params(inner, **kw):
    p = dict(tol=1e-10, max_iter=20000, inner=inner, delta=0.1, check_every=4, x0_given=0,
             use_graph=0)
    p.update(kw)
    return p


def _both(dims, masses, inner, seed):
    """Solves the same system with both entry points; returns the two packed
    solutions, their stats and the canonical inputs."""
    nrhs = len(masses)
    U = li.near_unity_gauge(dims, seed, 0.3)
    bs = li.gaussian_spinors(dims, [seed + 1 + k for k in range(nrhs)])
    ghi = DeviceGauge(U, w.WD_FP64)
    glo = DeviceGauge(U, inner) if inner != w.WD_FP64 else None
    b = ghi.pack(bs, nrhs=nrhs)
    ws = torch.empty(w.cg_workspace_bytes(dims, nrhs, inner), dtype=torch.uint8, device="cuda")
    x_ref = ghi.spinor(nrhs)
    rc, st_ref = w.cg_solve_normal(ghi.handle, glo.handle if glo else None, masses, nrhs, b, x_ref,
                                   _params(inner), ws)
    assert rc == w.WD_OK, st_ref
    x = ghi.spinor(nrhs)
    x.fill_(0xA5)  # garbage: the solver must not read x without x0_given
    rc, st = w.cg_solve_normal_noalloc(ghi.handle, glo.handle if glo else None, masses, nrhs, b, x,
                                       _params(inner))
    assert rc == w.WD_OK, st
    torch.cuda.synchronize()
    return x_ref, x, st_ref, st, U, bs, ghi


def _check(dims, masses, inner, seed):
    print(f"case noalloc dims={dims} nrhs={len(masses)} inner={inner}", flush=True)
    x_ref, x, st_ref, st, U, bs, ghi = _both(dims, masses, inner, seed)
    # every lattice site bit for bit (the padding sites of a packed field, which
    # no reduction reads, carry whatever the buffers held)
    xs = ghi.unpack(x, nrhs=len(masses))
    assert np.array_equal(xs, ghi.unpack(x_ref, nrhs=len(masses)))
    for a, b in zip(st, st_ref):
        assert (a["iters"], a["reliable_updates"], a["true_rel_residual"]) == (
            b["iters"], b["reliable_updates"], b["true_rel_residual"])
    xs = xs if len(masses) > 1 else xs[None]
    for k, m in enumerate(masses):
        r = bs[k] - oracle.normal_op(U, m, xs[k])
        assert np.linalg.norm(r) / np.linalg.norm(bs[k]) <= 1e-10


def test_noalloc_two_calls_second_smaller():
    # first call: 8^4 with 3 right-hand sides, FP16-storage inner iterations
    _check((8, 8, 8, 8), [0.05, 0.2, 0.5], w.WD_FP16, 8101)
    # second call, on the same static workspace: a smaller lattice, one
    # right-hand side, plain FP64 (other offsets into the array, stale contents)
    _check((4, 4, 4, 4), [0.1], w.WD_FP64, 8201)


def test_noalloc_mixed_fp32_after_others():
    _check((8, 4, 4, 8), [0.07, 0.3], w.WD_FP32, 8301)


def test_noalloc_limits():
    dims = (4, 4, 4, 4)
    U = li.near_unity_gauge(dims, 8401, 0.3)
    g = DeviceGauge(U, w.WD_FP64)
    b = g.pack(li.gaussian_spinor(dims, 8402))
    x = g.spinor()
    with pytest.raises(w.WilsonError) as e:
        w.cg_solve_normal_noalloc(g.handle, None, [0.1], 1, b, x, _params(w.WD_FP64, use_graph=1))
    assert e.value.code == w.WD_ERR_UNSUPPORTED
    # a solve whose workspace exceeds the static array is refused before any launch
    big = (32, 32, 32, 32)
    assert w.cg_workspace_bytes(big, 1, w.WD_FP64) > 64 << 20
    Ub = torch.zeros((32, 32, 32, 32, 4, 3, 3), dtype=torch.complex128, device="cuda")
    Ub[..., 0, 0] = Ub[..., 1, 1] = Ub[..., 2, 2] = 1
    gb = DeviceGauge(Ub, w.WD_FP64)
    bb = gb.spinor()
    bb.zero_()
    xb = gb.spinor()
    with pytest.raises(w.WilsonError) as e:
        w.cg_solve_normal_noalloc(gb.handle, None, [0.1], 1, bb, xb, _params(w.WD_FP64))
    assert e.value.code == w.WD_ERR_NOMEM
    assert "workspace" in w.wd_last_error()
