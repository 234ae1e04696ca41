"""Request server (continuous batching of CG solves) on the GPU.

Each finished solve is checked by the oracle (true residual recomputed in FP64
on the CPU); a request solved in a mix gives bit for bit the x it gets alone;
the arena is never exceeded, and a small arena makes requests wait.
"""

import time

import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge, to_device

pytestmark = pytest.mark.gpu

DEADLINE_S = 90.0


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


class Lattice:
    def __init__(self, dims, seed):
        self.dims = dims
        self.U = li.near_unity_gauge(dims, seed, 0.3)
        self.Ud = to_device(self.U)
        self.packer = DeviceGauge(self.Ud, w.WD_FP64)  # only to pack / unpack spinors


def wait_all(srv, tickets):
    """Polls until every ticket is final; returns {ticket: (status, result)}."""
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < DEADLINE_S, f"requests still pending: {set(tickets) - set(out)}"
        for t in tickets:
            if t in out:
                continue
            rc, res = w.cg_poll(srv, t)
            if rc != w.WD_PENDING:
                out[t] = (rc, res)
        time.sleep(0.002)
    return out


def true_rel_residual(U, m, b, x):
    r = b - oracle.normal_op(U, m, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def make_server(arena_bytes, **kw):
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = w.wd_server_create(arena, kw.pop("inner", w.WD_FP32), **kw)
    return srv, arena


@pytest.mark.parametrize("inner", ["fp32", "fp16"])
def test_server_mix_alone_equals_mix_and_residuals(inner):
    lats = [Lattice((8, 8, 8, 8), 501), Lattice((16, 8, 8, 4), 502)]
    rng = np.random.default_rng(5000)
    reqs = []  # (lattice index, masses, b canonical [nrhs,...])
    for i in range(8):
        li_ = int(rng.integers(0, 2))
        nrhs = int(rng.integers(1, 4))
        masses = list(rng.uniform(0.05, 0.5, nrhs))
        b = li.gaussian_spinors(lats[li_].dims, [6000 + 10 * i + k for k in range(nrhs)])
        reqs.append((li_, masses, b))

    def run(subset):
        srv, arena = make_server(1 << 30, inner={"fp32": w.WD_FP32, "fp16": w.WD_FP16}[inner],
                                 check_every=4, max_rhs_per_group=8, n_streams=4)
        try:
            gids = [w.wd_server_add_gauge(srv, L.dims, L.Ud) for L in lats]
            bufs, tickets = {}, []
            for i in subset:
                li_, masses, b = reqs[i]
                L = lats[li_]
                bd = L.packer.pack(b, nrhs=len(masses))
                xd = L.packer.spinor(len(masses))
                t = w.cg_submit(srv, gids[li_], masses, bd, xd, tol=1e-10)
                bufs[t] = (i, bd, xd)
                tickets.append(t)
            done = wait_all(srv, tickets)
            info = w.wd_server_info(srv)
            assert info["arena_peak"] <= arena.numel() and info["unfinished"] == 0
            xs = {}
            for t in tickets:
                i, bd, xd = bufs[t]
                rc, res = done[t]
                assert rc == w.WD_OK, res
                nrhs = len(reqs[i][1])
                x = lats[reqs[i][0]].packer.unpack(xd, nrhs=nrhs)
                xs[i] = (x if nrhs > 1 else x[None], res)
            return xs
        finally:
            w.wd_server_destroy(srv)

    mix = run(range(len(reqs)))
    for i, (li_, masses, b) in enumerate(reqs):
        x, res = mix[i]
        for k, m in enumerate(masses):
            assert res["stats"][k]["status"] == w.WD_OK
            assert true_rel_residual(lats[li_].U, m, b[k], x[k]) <= 1e-10
        assert res["t_done"] >= res["t_start"] >= res["t_submit"]
    for i in (0, 3, 7):
        alone = run([i])
        assert np.array_equal(alone[i][0], mix[i][0]), f"request {i} differs alone vs in the mix"


def test_server_small_arena_queues_and_fp64_inner():
    L = Lattice((8, 8, 8, 8), 601)
    V = li.volume(L.dims)
    # room for the gauge field and one group of 2 slots only
    gauge = w.wd_gauge_bytes(L.dims, w.WD_FP64, 0)
    group = 2 * w.wd_spinor_bytes(L.dims, w.WD_FP64, 2) + w.cg_workspace_bytes(L.dims, 2, w.WD_FP64)
    arena_bytes = gauge + group + 64 * 1024
    srv, arena = make_server(arena_bytes, inner=w.WD_FP64, check_every=2, max_rhs_per_group=2,
                             n_streams=2)
    try:
        gid = w.wd_server_add_gauge(srv, L.dims, L.Ud)
        tickets, data = [], {}
        for i in range(5):
            b = li.gaussian_spinors(L.dims, [700 + 2 * i, 701 + 2 * i])
            bd, xd = L.packer.pack(b, nrhs=2), L.packer.spinor(2)
            t = w.cg_submit(srv, gid, [0.1, 0.3], bd, xd)
            tickets.append(t)
            data[t] = (b, bd, xd)
        done = wait_all(srv, tickets)
        starts = sorted(done[t][1]["t_start"] for t in tickets)
        ends = sorted(done[t][1]["t_done"] for t in tickets)
        # one group at a time: each request starts after an earlier one ended
        assert all(starts[k + 1] >= ends[k] - 1e-3 for k in range(len(tickets) - 1))
        info = w.wd_server_info(srv)
        assert info["arena_peak"] <= arena_bytes
        for t in tickets:
            b, bd, xd = data[t]
            assert done[t][0] == w.WD_OK
            x = L.packer.unpack(xd, nrhs=2)
            assert true_rel_residual(L.U, 0.3, b[1], x[1]) <= 1e-10
        assert V > 0
    finally:
        w.wd_server_destroy(srv)


def test_server_errors_and_cancel():
    L = Lattice((8, 8, 8, 8), 801)
    srv, arena = make_server(256 << 20, check_every=4, max_rhs_per_group=4)
    try:
        gid = w.wd_server_add_gauge(srv, L.dims, L.Ud)
        b = L.packer.pack(li.gaussian_spinor(L.dims, 1))
        x = L.packer.spinor(1)
        with pytest.raises(w.WilsonError) as e:
            w.cg_submit(srv, gid + 99, [0.1], b, x)
        assert e.value.code == w.WD_ERR_INVALID_ARG
        with pytest.raises(w.WilsonError) as e:
            w.cg_submit(srv, gid, [0.1] * 5, b, x)
        assert e.value.code == w.WD_ERR_UNSUPPORTED
        with pytest.raises(w.WilsonError) as e:
            w.cg_submit(srv, gid, [0.1], b, b)
        assert e.value.code == w.WD_ERR_INVALID_ARG
        with pytest.raises(w.WilsonError) as e:
            w.cg_poll(srv, 12345)
        assert e.value.code == w.WD_ERR_UNKNOWN_TICKET
        # not converged within max_iter
        t = w.cg_submit(srv, gid, [0.05], b, x, max_iter=4)
        rc, res = wait_all(srv, [t])[t]
        assert rc == w.WD_ERR_NOT_CONVERGED and res["stats"][0]["iters"] == 4
        # a ticket is reported once
        with pytest.raises(w.WilsonError):
            w.cg_poll(srv, t)
        # many queued requests, then destroy: every one ends OK or CANCELLED
        bs = [L.packer.pack(li.gaussian_spinor(L.dims, 10 + i)) for i in range(6)]
        xs = [L.packer.spinor(1) for _ in range(6)]
        for i in range(6):
            w.cg_submit(srv, gid, [0.05], bs[i], xs[i])
    finally:
        w.wd_server_destroy(srv)
    torch.cuda.synchronize()


def test_server_rejects_group_that_cannot_fit():
    L = Lattice((8, 8, 8, 8), 901)
    gauge = w.wd_gauge_bytes(L.dims, w.WD_FP64, 0) + w.wd_gauge_bytes(L.dims, w.WD_FP32, 0)
    srv, arena = make_server(gauge + (1 << 20), check_every=4, max_rhs_per_group=4)
    try:
        gid = w.wd_server_add_gauge(srv, L.dims, L.Ud)
        b = L.packer.pack(li.gaussian_spinor(L.dims, 1))
        x = L.packer.spinor(1)
        with pytest.raises(w.WilsonError) as e:
            w.cg_submit(srv, gid, [0.1], b, x)
        assert e.value.code == w.WD_ERR_NOMEM
    finally:
        w.wd_server_destroy(srv)


@pytest.mark.parametrize("evict", [False, True])
def test_server_evicts_least_recently_used_idle_gauge(evict):
    dims = (8, 8, 8, 8)
    lats = [Lattice(dims, 1101 + i) for i in range(4)]
    gauge = w.wd_gauge_bytes(dims, w.WD_FP64, 0) + w.wd_gauge_bytes(dims, w.WD_FP16, 0)
    group = 2 * w.wd_spinor_bytes(dims, w.WD_FP64, 1) + w.cg_workspace_bytes(dims, 1, w.WD_FP16)
    assert group > gauge
    arena_bytes = 2 * gauge + group + (64 << 10)
    srv, arena = make_server(arena_bytes, inner=w.WD_FP16, check_every=4, max_rhs_per_group=1,
                             n_streams=1, evict_idle_gauges=evict)
    try:
        a = w.wd_server_add_gauge(srv, dims, lats[0].Ud)
        b = w.wd_server_add_gauge(srv, dims, lats[1].Ud)
        src = li.gaussian_spinor(dims, 77)
        bd, x = lats[0].packer.pack(src), lats[0].packer.spinor(1)
        t = w.cg_submit(srv, a, [0.2], bd, x)            # a becomes the most recently used
        assert wait_all(srv, [t])[t][0] == w.WD_OK
        t0 = time.time()
        while w.wd_server_info(srv)["arena_in_use"] > 2 * gauge:   # its group is freed
            assert time.time() - t0 < DEADLINE_S
            time.sleep(0.005)
        c = w.wd_server_add_gauge(srv, dims, lats[2].Ud)  # fits where the group was
        assert w.wd_server_info(srv)["evictions"] == 0
        if not evict:
            with pytest.raises(w.WilsonError) as e:
                w.wd_server_add_gauge(srv, dims, lats[3].Ud)
            assert e.value.code == w.WD_ERR_NOMEM
            return
        d = w.wd_server_add_gauge(srv, dims, lats[3].Ud)  # evicts b, the least recently used
        info = w.wd_server_info(srv)
        assert info["evictions"] == 1 and info["gauges"] == 3
        with pytest.raises(w.WilsonError) as e:
            w.cg_submit(srv, b, [0.2], bd, x)
        assert e.value.code == w.WD_ERR_INVALID_ARG
        w.wd_server_remove_gauge(srv, c)                  # room for a group beside a and d
        src_d = li.gaussian_spinor(dims, 78)
        bd_d, x_d = lats[3].packer.pack(src_d), lats[3].packer.spinor(1)
        t = w.cg_submit(srv, d, [0.2], bd_d, x_d)
        assert wait_all(srv, [t])[t][0] == w.WD_OK
        assert true_rel_residual(lats[3].U, 0.2, src_d, lats[3].packer.unpack(x_d)) <= 1e-10
    finally:
        w.wd_server_destroy(srv)


def test_server_opens_a_smaller_group_when_a_full_one_does_not_fit():
    dims = (8, 8, 8, 8)
    lats = [Lattice(dims, 1201), Lattice(dims, 1202)]
    inner = w.WD_FP32
    gauge = w.wd_gauge_bytes(dims, w.WD_FP64, 0) + w.wd_gauge_bytes(dims, inner, 0)

    def group(S):
        return 2 * w.wd_spinor_bytes(dims, w.WD_FP64, S) + w.cg_workspace_bytes(dims, S, inner)

    # two gauge fields, one group of 4 slots and one of 1 (not 2)
    arena_bytes = 2 * gauge + group(4) + group(1) + (64 << 10)
    assert group(1) + (64 << 10) < group(2)
    b_big = li.gaussian_spinors(dims, [1300 + k for k in range(4)])
    b_one = li.gaussian_spinor(dims, 1310)

    def run(with_big):
        srv, arena = make_server(arena_bytes, inner=inner, check_every=4, max_rhs_per_group=4,
                                 n_streams=2)
        try:
            ga = w.wd_server_add_gauge(srv, dims, lats[0].Ud)
            gb = w.wd_server_add_gauge(srv, dims, lats[1].Ud)
            tickets = []
            if with_big:
                bd_big, x_big = lats[0].packer.pack(b_big, nrhs=4), lats[0].packer.spinor(4)
                tickets.append(w.cg_submit(srv, ga, [0.05, 0.1, 0.2, 0.3], bd_big, x_big, tol=1e-10))
            bd_one, x_one = lats[1].packer.pack(b_one), lats[1].packer.spinor(1)
            tickets.append(w.cg_submit(srv, gb, [0.07], bd_one, x_one, tol=1e-10))
            done = wait_all(srv, tickets)
            assert all(done[t][0] == w.WD_OK for t in tickets)
            assert w.wd_server_info(srv)["arena_peak"] <= arena_bytes
            res = {t: done[t][1] for t in tickets}
            return res, tickets, lats[1].packer.unpack(x_one)
        finally:
            w.wd_server_destroy(srv)

    res, (t_big, t_one), x = run(True)
    # the 1-RHS request runs beside the 4-RHS one instead of waiting for its memory
    assert res[t_one]["t_start"] < res[t_big]["t_done"]
    assert true_rel_residual(lats[1].U, 0.07, b_one, x) <= 1e-10
    _, _, x_alone = run(False)
    assert np.array_equal(x, x_alone)
