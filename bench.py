"""Benchmark of the Wilson-Dirac operator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp64|fp32|fp16] [--c12]

A step is one application of dslash_apply (D = (4+m) - H/2, periodic, m = 0.1)
to a Gaussian spinor with random SU(3) links on the 32^3 x 64 lattice
(2,097,152 sites), inputs already packed in HBM. Prints one JSON line with
GFlop/s (1320 flop/site), the HBM roofline fraction on compulsory bytes, a
sampled parity check against the CPU oracle, and the oracle's own time on the
host as the CPU baseline.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "dslash GFlop/s & % HBM peak; mixed-prec CG solves/s, p50/p99 latency"
FLOPS_PER_SITE = 1320
HBM_PEAK_GBS = 8000.0
# FP32 vector rate without packed FP32 instructions, which the build disables
# (157.3 TFLOP/s with them); the arithmetic of the FP32 and FP16-storage paths
FP32_VECTOR_PEAK_GFLOPS = 78600.0
DIMS = (32, 32, 32, 64)
CONFIG_INDEX = 2          # seeds of the production-lattice configuration

# Bytes per site of a packed spinor and of one packed link (full or 12-real).
SPINOR_BYTES = {"fp64": 192, "fp32": 96, "fp16": 52}   # FP16: 24 binary16 + FP32 scale
REAL_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}


# Compulsory HBM bytes per site: 4 links + spinor in + spinor out.
def compulsory_bytes(prec: str, c12: bool) -> int:
    return REAL_BYTES[prec] * 4 * (12 if c12 else 18) + 2 * SPINOR_BYTES[prec]


# HBM traffic of the dslash kernel measured with rocprofv3 --pmc (FETCH_SIZE,
# WRITE_SIZE), scaled by the same counters on a plain copy of known size; valid
# only for the kernel sources it was measured on (hash below) and the launch
# timed, else null.
TRAFFIC = {
    # FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (copy-calibrated KiB per dispatch), measured for
    # the kernel code hashed below, per launch "tb,gw,group,rb" the bytes belong to
    "wilson_dslash_32x32x32x64_fp64": {"source_sha": "f8e8833d29f40acb", "launches": {
        "32,1,32,1": 2211276800}},  # 883,117 / 393,216
    "wilson_dslash_32x32x32x64_fp64_c12": {"source_sha": "f8e8833d29f40acb", "launches": {
        "32,1,32,1": 1778633728}},  # 671,843 / 393,261
    "wilson_dslash_32x32x32x64_fp32": {"source_sha": "f8e8833d29f40acb", "launches": {
        "16,1,64,1": 1115131904}},  # 446,191 / 196,614
    "wilson_dslash_32x32x32x64_fp16": {"source_sha": "f8e8833d29f40acb", "launches": {
        "4,1,256,1": 618565632}},   # 248,786 / 106,496
}
KERNEL_SOURCES = ["paper_1901_07294_amd/csrc/dslash.hip", "paper_1901_07294_amd/csrc/stencil.h",
                  "paper_1901_07294_amd/csrc/fields.h", "paper_1901_07294_amd/csrc/cplx.h"]


def strip_comments(src: str) -> str:
    """C++ source text without its comments (string and character literals
    kept), trailing blanks and empty lines: the code a compiler sees."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash() -> str:
    """Hash of the dslash kernels' code (comments excluded, so that editing
    one does not orphan counters taken on the same code)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            h.update(strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", choices=["fp64", "fp32", "fp16"], default="fp64")
    ap.add_argument("--c12", action="store_true", help="12-real link compression")
    ap.add_argument("--dims", type=str, default=",".join(map(str, DIMS)))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests in the serving measurement (capacity and each load level)")
    ap.add_argument("--tuning", type=str, default=None,
                    help="TB,GW,GROUP,RB: time the operator with this launch instead of the "
                         "autotuner's choice (profiling runs pin it)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the secondary precision/compression measurements")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-RHS measurement")
    ap.add_argument("--no-cg", action="store_true", help="skip the CG solves/s measurement")
    ap.add_argument("--no-cg-multi", action="store_true", help="skip the 12-RHS CG measurement")
    ap.add_argument("--no-wilson", action="store_true", help="skip the D x = b (even-odd) measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch choices (skip the autotuner)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain device copy of known size (PMC calibration)")
    return ap.parse_args(argv)


def copy_calibration(torch, nbytes=1 << 30, reps=5):
    """Plain device-to-device copy of nbytes, for counter calibration and the
    achievable-bandwidth ceiling. Returns GB/s (read + write bytes)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return 2 * nbytes / t / 1e9


def stream_triad(torch, nbytes=1 << 30, reps=10):
    """STREAM triad a = b + s c on FP64 arrays of nbytes each (torch's own
    elementwise kernel): the achievable-bandwidth ceiling of a plain stream.
    Returns GB/s (two reads + one write)."""
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    torch.add(b, c, alpha=3.0, out=a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(b, c, alpha=3.0, out=a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return 3 * n * 8 / t / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


TUNE = True  # set from --no-tune


def tune(torch, w, g, nrhs, src):
    """Runs the library's autotuner for g's lattice and nrhs (outside any timed
    region); later launches of that key use its choice."""
    if not TUNE:
        return None
    out, ref = g.spinor(nrhs), g.spinor(nrhs)
    res = w.wd_tune_dslash(g.handle, nrhs, src, out, ref, reps=5)
    del out, ref
    return {k: (round(v, 2) if isinstance(v, float) else v) for k, v in res.items()}


def force_tuning(w, dims, prec_id, c12, spec):
    """Registers the launch `spec` = "tb,gw,group,rb" for the single-field
    operator on `dims` (through a one-line tuning file) instead of running the
    autotuner, so that separate profiling runs time the same launch."""
    tb, gw, group, rb = (int(v) for v in spec.split(","))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tuning.txt")
        w.wd_tune_save(path)  # the header and whatever is registered already
        with open(path, "a") as f:
            f.write(f"{dims[0]} {dims[1]} {dims[2]} {dims[3]} {prec_id} {int(c12)} 1 {tb} {gw} {group} {rb}\n")
        w.wd_tune_load(path)
    return {"forced": True, "tb": tb, "gw": gw, "group": group, "rb": rb}


def time_applies(torch, w, g, src, dst, mass, steps, warmup):
    for _ in range(warmup):
        w.dslash_apply(g.handle, mass, src, dst, g.prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        w.dslash_apply(g.handle, mass, src, dst, g.prec)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per apply


def bench_latency(torch, w, li, DeviceGauge, oracle, n=1000):
    """The smallest configuration, 4^4 FP64 with random SU(3) links: launch
    latency of one dslash_apply (median of n individually timed launches) and
    its parity against the oracle. Cache-resident; not a bandwidth figure."""
    dims = (4, 4, 4, 4)
    U = li.random_gauge(dims, li.seed_gauge(1))
    psi = li.gaussian_spinor(dims, li.seed_spinor(1))
    g = DeviceGauge(U, w.WD_FP64)
    src, dst = g.pack(psi), g.spinor()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for _ in range(20):
        w.dslash_apply(g.handle, 0.1, src, dst, g.prec)
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        w.dslash_apply(g.handle, 0.1, src, dst, g.prec)
        b.record()
    torch.cuda.synchronize()
    us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    ref = oracle.dslash(U, psi, 0.1)
    err = float(np.linalg.norm(g.unpack(dst) - ref) / np.linalg.norm(ref))
    return {"workload": "wilson_dslash_4x4x4x4_fp64", "launches": n,
            "median_us": round(float(np.median(us)), 2), "p10_us": round(float(np.percentile(us, 10)), 2),
            "p90_us": round(float(np.percentile(us, 90)), 2), "parity_rel_err": err,
            "parity_ok": err <= 1e-13}


def multi_roof(nrhs: int, bytes_per_site: int, gflops: float) -> dict:
    """The roof of a fused multi-right-hand-side launch: the smaller of the HBM
    peak times its arithmetic intensity (nrhs x 1320 flop per bytes_per_site)
    and the FP32 vector peak, and the fraction of it that gflops reaches."""
    by_hbm = HBM_PEAK_GBS * nrhs * FLOPS_PER_SITE / bytes_per_site
    bound, roof = ("alu", FP32_VECTOR_PEAK_GFLOPS) if FP32_VECTOR_PEAK_GFLOPS < by_hbm else ("hbm", by_hbm)
    return {"bound": bound, "roof_gflops": round(roof, 1), "frac": round(gflops / roof, 4)}


def bench_multi(torch, w, li, DeviceGauge, prec="fp32", steps=50, warmup=5, inputs=None):
    """12 right-hand sides on 24^3 x 48, near-unity links, FP32 or FP16 storage:
    one fused launch against 12 single launches."""
    dims, nrhs = (24, 24, 24, 48), 12
    V = li.volume(dims)
    if inputs is None:
        inputs = (li.near_unity_gauge(dims, li.seed_gauge(3), 0.3),
                  li.gaussian_spinors(dims, [li.seed_spinor(3, k) for k in range(nrhs)]))
    U, psis = inputs
    masses = [0.1] * nrhs
    g = DeviceGauge(U, {"fp32": w.WD_FP32, "fp16": w.WD_FP16}[prec])
    src = g.pack(psis, nrhs=nrhs)
    dst = g.spinor(nrhs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    tuned = tune(torch, w, g, nrhs, src)
    fused = timed(lambda: w.dslash_apply_multi(g.handle, masses, nrhs, src, dst, g.prec))
    one = g.spinor(1)
    res = g.spinor(1)
    w.wd_spinor_import(g.handle, torch.from_numpy(psis[0]).cuda(), g.prec, 1, one)
    tune(torch, w, g, 1, one)
    single = timed(lambda: w.dslash_apply(g.handle, 0.1, one, res, g.prec)) * nrhs
    comp = REAL_BYTES[prec] * 4 * 18 + nrhs * 2 * SPINOR_BYTES[prec]  # links once + 12 x (in + out)
    # parity of the fused launch's output against the oracle on sampled sites of every field
    import oracle
    outs = g.unpack(dst, nrhs=nrhs).reshape(nrhs, -1, 4, 3)
    sites = np.random.default_rng(8).choice(V, 256, replace=False)
    err = 0.0
    for k in range(nrhs):
        ref = oracle.dslash_sites(U, psis[k], masses[k], sites)
        err = max(err, float(np.linalg.norm(outs[k][sites] - ref) / np.linalg.norm(ref)))
    tol = {"fp32": 1e-6, "fp16": 2e-3}[prec]
    gflops = nrhs * FLOPS_PER_SITE * V / (fused / 1e3) / 1e9
    return {"workload": "wilson_dslash_multi_24x24x24x48_x12", "prec": prec, "links": "full",
            "parity": {"max_rel_err": err, "tol": tol, "sites_per_field": 256, "ok": err <= tol},
            "gauge": "near-unity eps=0.3", "ms_per_apply": round(fused, 4),
            "gflops": round(gflops, 1),
            "pct_hbm_peak": round(100 * comp * V / (fused / 1e3) / 1e9 / HBM_PEAK_GBS, 2),
            "roof": multi_roof(nrhs, comp, gflops),
            "ms_12_single_applies": round(single, 4), "speedup_vs_single": round(single / fused, 3),
            "tuning": tuned}


def bench_cg(torch, w, li, DeviceGauge, reps=5, cpu=True):
    """Solves of D^dag D x = b on 24^4, m = 0.05, near-unity links, to a true
    residual of 1e-10: plain FP64 CG against FP32 or FP16-storage inner
    iterations with FP64 reliable updates, eager and with chunks of iterations
    replayed as HIP graphs; and the same eager/graph pair on an 8^4 lattice,
    where launch overhead dominates. Every solution is checked outside the
    timed region by the oracle: its true residual |b - D^dag D x| / |b|
    recomputed in FP64 on the CPU, and its distance from the FP64 solve's x."""
    import oracle
    m = 0.05
    x_fp64 = {}

    def setup(dims):
        U = li.near_unity_gauge(dims, li.seed_gauge(4), 0.3)
        b = li.gaussian_spinor(dims, li.seed_spinor(4))
        ghi = DeviceGauge(U, w.WD_FP64)
        glo = {w.WD_FP64: ghi, w.WD_FP32: DeviceGauge(U, w.WD_FP32),
               w.WD_FP16: DeviceGauge(U, w.WD_FP16)}
        return ghi, glo, ghi.pack(b), ghi.spinor(1), b, U

    x_eager = {}

    def check(dims, lat, inner, use_graph):
        ghi, _, _, x, b, U = lat
        xs = ghi.unpack(x)
        if use_graph and (dims, inner) in x_eager:  # graph replay: the eager solve's bits
            return {"same_x_as_eager": bool(np.array_equal(xs, x_eager[(dims, inner)]))}
        x_eager[(dims, inner)] = xs
        r = b - oracle.normal_op(U, m, xs)
        out = {"oracle_true_rel_residual": float(np.linalg.norm(r) / np.linalg.norm(b))}
        if inner == w.WD_FP64:
            x_fp64[dims] = xs
        elif dims in x_fp64:
            ref = x_fp64[dims]
            out["rel_diff_vs_fp64_solution"] = float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))
        return out

    def run(dims, lat, inner, use_graph, delta=0.1):
        ghi, glo, bd, x, b, _ = lat
        for g in {id(ghi): ghi, id(glo[inner]): glo[inner]}.values():
            tune(torch, w, g, 1, g.pack(b))
        ws = torch.empty(w.cg_workspace_bytes(dims, 1, inner), dtype=torch.uint8, device="cuda")
        params = dict(tol=1e-10, max_iter=20000, inner=inner, delta=delta, check_every=8, x0_given=0,
                      use_graph=use_graph)
        gl = glo[inner].handle
        w.cg_solve_normal(ghi.handle, gl, [m], 1, bd, x, params, ws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rc, st = w.cg_solve_normal(ghi.handle, gl, [m], 1, bd, x, params, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        return {"status": rc, "solves_per_s": round(1.0 / dt, 2), "ms_per_solve": round(dt * 1e3, 3),
                "iters": st[0]["iters"], "reliable_updates": st[0]["reliable_updates"],
                "true_rel_residual": st[0]["true_rel_residual"], **check(dims, lat, inner, use_graph)}

    dims = (24, 24, 24, 24)
    lat = setup(dims)
    out = {"workload": "cg_normal_24x24x24x24_m0.05", "tol": 1e-10, "gauge": "near-unity eps=0.3",
           "check_every": 8, "delta": 0.1}
    if cpu:
        # the oracle's CG (FP64 numpy, one core) timed over 5 iterations and
        # extrapolated to the GPU FP64 solver's iteration count
        U = li.near_unity_gauge(dims, li.seed_gauge(4), 0.3)
        b = li.gaussian_spinor(dims, li.seed_spinor(4))
        t0 = time.perf_counter()
        oracle.normal_op(U, m, b)
        t_op = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.cg_normal(U, m, b, tol=1e-10, max_iter=5)
        t5 = time.perf_counter() - t0
        out["cpu_oracle"] = {"kind": "oracle", "cores": 1, "label": "extrapolated",
                             "s_per_iteration": round((t5 - t_op) / 5, 3), "s_setup": round(t_op, 3)}
        del U, b
    for name, inner, graph in (("fp64", w.WD_FP64, 0), ("mixed_fp32", w.WD_FP32, 0),
                               ("mixed_fp16", w.WD_FP16, 0), ("fp64_graph", w.WD_FP64, 1),
                               ("mixed_fp32_graph", w.WD_FP32, 1), ("mixed_fp16_graph", w.WD_FP16, 1)):
        out[name] = run(dims, lat, inner, graph)
    # the same FP16-storage solve with reliable updates at every drop by 20 (delta
    # 0.05) instead of 10: the same iterations, fewer FP64 recomputes here
    out["mixed_fp16_delta_0.05"] = {"delta": 0.05, **run(dims, lat, w.WD_FP16, 0, delta=0.05)}
    if "cpu_oracle" in out:
        c = out["cpu_oracle"]
        c["iterations"] = out["fp64"]["iters"]
        c["s_per_solve"] = round(c["s_setup"] + c["iterations"] * c["s_per_iteration"], 1)
        c["solves_per_s"] = round(1.0 / c["s_per_solve"], 5)
    base = out["fp64"]["ms_per_solve"]
    for name in ("mixed_fp32", "mixed_fp16", "fp64_graph", "mixed_fp32_graph", "mixed_fp16_graph",
                 "mixed_fp16_delta_0.05"):
        out[name]["speedup_vs_fp64"] = round(base / out[name]["ms_per_solve"], 3)
    del lat
    small = (8, 8, 8, 8)
    lat = setup(small)
    out["small_8x8x8x8"] = {name: run(small, lat, inner, graph) for name, inner, graph in
                            (("mixed_fp32", w.WD_FP32, 0), ("mixed_fp32_graph", w.WD_FP32, 1))}
    return out


def bench_cg_multi(torch, w, li, DeviceGauge, nrhs=12, reps=3, single_fp64_ms=None):
    """One cg_solve_normal call on 12 right-hand sides of 24^4 (m = 0.05,
    near-unity links, tol 1e-10): plain FP64 CG against FP32 and FP16-storage
    inner iterations with FP64 reliable updates, in right-hand-side solves per
    second, and against 12 separate single-right-hand-side FP64 solves. The
    oracle recomputes |b - D^dag D x| / |b| of the first and last right-hand
    side of every batch outside the timed region."""
    import oracle
    dims, m = (24, 24, 24, 24), 0.05
    U = li.near_unity_gauge(dims, li.seed_gauge(4), 0.3)
    bs = li.gaussian_spinors(dims, [li.seed_spinor(4, k) for k in range(nrhs)])
    ghi = DeviceGauge(U, w.WD_FP64)
    glo = {w.WD_FP64: ghi, w.WD_FP32: DeviceGauge(U, w.WD_FP32), w.WD_FP16: DeviceGauge(U, w.WD_FP16)}
    b = ghi.pack(bs, nrhs=nrhs)
    x = ghi.spinor(nrhs)
    out = {"workload": f"cg_normal_24x24x24x24_m0.05_x{nrhs}", "tol": 1e-10, "nrhs": nrhs,
           "gauge": "near-unity eps=0.3", "check_every": 8}
    for name, inner in (("fp64", w.WD_FP64), ("mixed_fp32", w.WD_FP32), ("mixed_fp16", w.WD_FP16)):
        for g in {id(ghi): ghi, id(glo[inner]): glo[inner]}.values():
            tune(torch, w, g, nrhs, g.pack(bs, nrhs=nrhs))
        ws = torch.empty(w.cg_workspace_bytes(dims, nrhs, inner), dtype=torch.uint8, device="cuda")
        params = dict(tol=1e-10, max_iter=20000, inner=inner, delta=0.1, check_every=8, x0_given=0,
                      use_graph=0)
        gl = glo[inner].handle
        w.cg_solve_normal(ghi.handle, gl, [m] * nrhs, nrhs, b, x, params, ws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rc, st = w.cg_solve_normal(ghi.handle, gl, [m] * nrhs, nrhs, b, x, params, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        xs = ghi.unpack(x, nrhs=nrhs)
        res = []
        for k in (0, nrhs - 1):
            r = bs[k] - oracle.normal_op(U, m, xs[k])
            res.append(float(np.linalg.norm(r) / np.linalg.norm(bs[k])))
        out[name] = {"status": rc, "ms_per_batch": round(dt * 1e3, 2),
                     "rhs_solves_per_s": round(nrhs / dt, 2),
                     "iters_max": max(s["iters"] for s in st),
                     "reliable_updates_max": max(s["reliable_updates"] for s in st),
                     "true_rel_residual_max": max(s["true_rel_residual"] for s in st),
                     "oracle_true_rel_residual_sample": res}
        del ws
        print(f"[bench] cg x{nrhs} {name}: {out[name]['rhs_solves_per_s']} RHS solves/s",
              file=sys.stderr, flush=True)
    base = out["fp64"]["rhs_solves_per_s"]
    for name in ("mixed_fp32", "mixed_fp16"):
        out[name]["speedup_vs_fp64_batch"] = round(out[name]["rhs_solves_per_s"] / base, 3)
    if single_fp64_ms:
        out["single_fp64_rhs_solves_per_s"] = round(1e3 / single_fp64_ms, 2)
        for name in ("fp64", "mixed_fp32", "mixed_fp16"):
            out[name]["speedup_vs_single_fp64"] = round(out[name]["rhs_solves_per_s"] * single_fp64_ms / 1e3, 3)
    return out


def bench_wilson(torch, w, li, DeviceGauge, reps=3):
    """Solves of D x = b itself on 24^4 (m = 0.05, near-unity links) to
    |b - D x| / |b| <= 1e-10: the normal equations D^dag D x = D^dag b against
    even-odd preconditioning (CG on the odd-site Schur complement), FP64 and
    FP16-storage inner iterations. The oracle recomputes |b - D x| / |b| of
    every solution outside the timed region."""
    import oracle.solve_ref as sr
    dims, m = (24, 24, 24, 24), 0.05
    U = li.near_unity_gauge(dims, li.seed_gauge(4), 0.3)
    bh = li.gaussian_spinor(dims, li.seed_spinor(4))
    out = {"workload": "wilson_solve_24x24x24x24_m0.05", "tol": 1e-10, "gauge": "near-unity eps=0.3",
           "check_every": 8}
    for eo in (False, True):
        ghi = DeviceGauge(U, w.WD_FP64, eo=eo)
        b = ghi.pack(bh)
        x = ghi.spinor()
        for iname, inner in (("fp64", w.WD_FP64), ("mixed_fp16", w.WD_FP16)):
            glo = DeviceGauge(U, inner, eo=eo) if inner != w.WD_FP64 else ghi
            if not eo:
                for g in {id(ghi): ghi, id(glo): glo}.values():
                    tune(torch, w, g, 1, g.pack(bh))
            ws = torch.empty(w.wilson_workspace_bytes(dims, 1, inner, eo), dtype=torch.uint8,
                             device="cuda")
            params = dict(tol=1e-10, max_iter=20000, inner=inner, delta=0.1, check_every=8,
                          x0_given=0, use_graph=0)
            w.cg_solve_wilson(ghi.handle, glo.handle, [m], 1, b, x, params, ws)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                rc, st = w.cg_solve_wilson(ghi.handle, glo.handle, [m], 1, b, x, params, ws)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            res = sr.wilson_residual(U, m, bh, ghi.unpack(x))
            name = f"{'eo' if eo else 'normal'}_{iname}"
            out[name] = {"status": rc, "solves_per_s": round(1.0 / dt, 2), "ms_per_solve": round(dt * 1e3, 3),
                         "iters": st[0]["iters"], "reliable_updates": st[0]["reliable_updates"],
                         "true_rel_residual": st[0]["true_rel_residual"],
                         "oracle_wilson_rel_residual": res}
            print(f"[bench] wilson {name}: {out[name]['solves_per_s']} solves/s, "
                  f"{st[0]['iters']} iterations", file=sys.stderr, flush=True)
            del ws
    for iname in ("fp64", "mixed_fp16"):
        out[f"eo_{iname}"]["speedup_vs_normal"] = round(
            out[f"normal_{iname}"]["ms_per_solve"] / out[f"eo_{iname}"]["ms_per_solve"], 3)
    out["eo_mixed_fp16"]["speedup_vs_normal_fp64"] = round(
        out["normal_fp64"]["ms_per_solve"] / out["eo_mixed_fp16"]["ms_per_solve"], 3)
    return out


def bench_serve(torch, w, li, DeviceGauge, n_req=80, loads=(0.5, 0.8, 0.95), seed=5000, arena_gib=128):
    """Request server under Poisson streams of CG solves (tol 1e-10, FP16-storage
    inner iterations with FP64 reliable updates) on a resident pool of two
    near-unity gauge fields per lattice size (8^4, 16^4, 24^3x48, 32^3x64);
    1..12 right-hand sides per request, masses uniform in [0.05, 0.5], in an
    arena of `arena_gib` GiB (gauge fields and solve groups). One list of
    `n_req` requests is drawn once: capacity is its makespan with up to 80
    queued at a time (all of them at the default 80), then the same requests
    arrive as a Poisson stream (one
    pattern of gaps, scaled) at each of `loads` times that rate, so the levels
    differ only in load. A second server with a small arena forces requests to
    queue."""
    import oracle
    from paper_1901_07294_amd.buffers import to_device
    sizes = [(8, 8, 8, 8), (16, 16, 16, 16), (24, 24, 24, 48), (32, 32, 32, 64)]
    nrhs_max = 12
    rng = np.random.default_rng(seed)

    def make_pool(srv, size_list, configs):
        lat = []
        for i, d in enumerate(size_list):
            for j in range(configs):
                U = li.near_unity_gauge(d, 5100 + configs * i + j, 0.3)
                Ud = to_device(U)
                gid = w.wd_server_add_gauge(srv, d, Ud)
                packer = DeviceGauge(Ud, w.WD_FP64)
                del Ud
                base = [li.gaussian_spinor(d, 5200 + 10 * i + k) for k in range(4)]
                bs = np.stack([base[k % 4] for k in range(nrhs_max)])
                pool = packer.pack(bs, nrhs=nrhs_max)   # shared, read-only right-hand sides
                del bs
                # the oracle checks results of 8^4 and 16^4 requests, and one of 24^3x48
                checked = d[0] * d[1] * d[2] * d[3] <= 24 ** 3 * 48
                lat.append({"dims": d, "U": U if checked else None, "gid": gid, "packer": packer,
                            "pool": pool, "base": base if checked else None})
        return lat

    def draw(lat, max_rhs):
        i = int(rng.integers(0, len(lat)))
        nrhs = int(rng.integers(1, max_rhs + 1))
        return i, list(rng.uniform(0.05, 0.5, nrhs))

    def run_stream(srv, lat, reqs, arrivals, max_live=80, keep=12, keep_mid=0, max_live_bytes=96 << 30):
        """Submits reqs[k] = (pool index, masses) at arrivals[k] (s; None = as
        soon as fewer than max_live requests are in flight); returns
        {ticket: (rc, res, (pool index, masses, x or None))}, the makespan and
        how many submissions waited for client memory. The solutions' buffers
        (the client's) in flight stay under max_live_bytes: a submission that
        would pass it waits for earlier requests to finish. Solutions are kept
        for the first `keep` finished 8^4 / 16^4 requests and the first
        `keep_mid` 24^3 x 48 ones (the oracle's sample); the others' buffers
        are released."""
        live, done = {}, {}
        kept = {"small": 0, "mid": 0}
        held = [0]

        def live_bytes():
            return sum(v[2].numel() for v in live.values())

        def poll():
            for t in list(live):
                rc, res = w.cg_poll(srv, t)
                if rc != w.WD_PENDING:
                    i, m, x = live.pop(t)
                    kind = None
                    if lat[i]["U"] is not None:
                        kind = "small" if li.volume(lat[i]["dims"]) <= 16 ** 4 else "mid"
                    if kind is not None and kept[kind] < (keep if kind == "small" else keep_mid):
                        kept[kind] += 1
                    else:
                        x = None
                    done[t] = (rc, res, (i, m, x))

        t0 = time.time()
        for j, ((i, m), a) in enumerate(zip(reqs, arrivals)):
            if j and j % 100 == 0:
                print(f"[bench] serving: {j} of {len(reqs)} submitted", file=sys.stderr, flush=True)
            while (a is not None and time.time() - t0 < a) or (a is None and len(live) >= max_live):
                poll()
                time.sleep(0.0005)
            need = w.wd_spinor_bytes(lat[i]["dims"], w.WD_FP64, len(m))
            if live and live_bytes() + need > max_live_bytes:
                held[0] += 1
                while live and live_bytes() + need > max_live_bytes:
                    poll()
                    time.sleep(0.0005)
            x = lat[i]["packer"].spinor(len(m))
            t = w.cg_submit(srv, lat[i]["gid"], m, lat[i]["pool"], x, tol=1e-10)
            live[t] = (i, m, x)
        deadline = time.time() + 120
        note = time.time() + 30
        while live:
            assert time.time() < deadline, f"serving measurement timed out ({len(live)} requests left)"
            if time.time() > note:
                print(f"[bench] serving: {len(live)} requests still running", file=sys.stderr, flush=True)
                note += 30
            poll()
            time.sleep(0.0005)
        return done, time.time() - t0, held[0]

    def worst_residual(lat, done, limit=12, mid=False):
        """Largest true residual the oracle recomputes over a sample of at most
        `limit` right-hand sides of the kept 8^4 and 16^4 solutions (smallest
        lattice first); with mid, the true residual of the first right-hand
        side of the kept 24^3 x 48 solution instead."""
        worst, checked = 0.0, 0
        kept = [v for v in done.values() if v[2][2] is not None and
                (li.volume(lat[v[2][0]]["dims"]) > 16 ** 4) == mid]
        kept.sort(key=lambda v: li.volume(lat[v[2][0]]["dims"]))
        for rc, res, (i, m, x) in kept:
            if checked >= (1 if mid else limit):
                break
            L = lat[i]
            xs = L["packer"].unpack(x, nrhs=len(m))
            xs = xs if len(m) > 1 else xs[None]
            for k in range(min(len(m), (1 if mid else limit) - checked)):
                b = L["base"][k % 4]
                r = b - oracle.normal_op(L["U"], m[k], xs[k])
                worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(b)))
                checked += 1
        return worst if checked or not mid else None

    def pct(v, q):
        return round(float(np.percentile(v, q)) * 1e3, 2)

    out = {"workload": "cg_requests_8^4_16^4_24^3x48_32^3x64_poisson", "inner": "fp16+fp64_reliable",
           "tol": 1e-10, "gauge_pool": "2 near-unity configs per size (seeds 5100..5107)",
           "arena_gib": arena_gib}
    torch.cuda.empty_cache()
    arena = torch.empty(arena_gib << 30, dtype=torch.uint8, device="cuda")
    srv = w.wd_server_create(arena, w.WD_FP16, check_every=8, delta=0.1,
                             max_rhs_per_group=nrhs_max, n_streams=4)
    try:
        lat = make_pool(srv, sizes, 2)
        reqs = [draw(lat, nrhs_max) for _ in range(n_req)]
        gaps = rng.exponential(1.0, n_req)  # unit-rate Poisson gaps, scaled per level
        nrhs_total = sum(len(m) for _, m in reqs)
        done, makespan, held = run_stream(srv, lat, reqs, [None] * n_req, keep_mid=1)
        capacity = n_req / makespan
        print(f"[bench] serving capacity {capacity:.2f} req/s", file=sys.stderr, flush=True)
        out["requests"] = n_req
        out["rhs_per_request_mean"] = round(nrhs_total / n_req, 2)
        out["capacity_req_per_s"] = round(capacity, 3)
        out["capacity_rhs_solves_per_s"] = round(nrhs_total / makespan, 2)
        out["capacity_submissions_held_for_client_memory"] = held
        out["levels"] = []
        worst = worst_residual(lat, done)
        # one 24^3 x 48 right-hand side, recomputed in full by the oracle (~5 s)
        out["oracle_true_rel_residual_24x24x24x48"] = worst_residual(lat, done, mid=True)
        for load in loads:
            arrivals = list(np.cumsum(gaps / (load * capacity)))
            done, wall, held = run_stream(srv, lat, reqs, arrivals)
            lat_s = np.array([res["t_done"] - res["t_submit"] for rc, res, _ in done.values()])
            wait_s = np.array([res["t_start"] - res["t_submit"] for rc, res, _ in done.values()])
            out["levels"].append({
                "offered_load": load, "requests": n_req, "latency_samples": int(len(lat_s)),
                "ok": int(sum(rc == w.WD_OK for rc, _, _ in done.values())),
                "req_per_s": round(n_req / wall, 3), "rhs_solves_per_s": round(nrhs_total / wall, 2),
                "p50_ms": pct(lat_s, 50), "p90_ms": pct(lat_s, 90), "p99_ms": pct(lat_s, 99),
                "queue_wait_p50_ms": pct(wait_s, 50), "queue_wait_p99_ms": pct(wait_s, 99),
                "submissions_held_for_client_memory": held})
            worst = max(worst, worst_residual(lat, done))
            lv = out["levels"][-1]
            print(f"[bench] serving load {load}: p50 {lv['p50_ms']} ms, p99 {lv['p99_ms']} ms",
                  file=sys.stderr, flush=True)
        out["max_true_rel_residual_oracle_sample"] = worst  # 12 RHS of 8^4 / 16^4 requests per run
        out["arena_peak_gb"] = round(w.wd_server_info(srv)["arena_peak"] / 1e9, 2)
    finally:
        w.wd_server_destroy(srv)
        del arena
    # a small arena: the two smallest sizes, room for the gauge fields and one group
    small_sizes = sizes[:2]
    per_group = (2 * w.wd_spinor_bytes(small_sizes[1], w.WD_FP64, 4) +
                 w.cg_workspace_bytes(small_sizes[1], 4, w.WD_FP16))
    gauges = sum(2 * (w.wd_gauge_bytes(d, w.WD_FP64, 0) + w.wd_gauge_bytes(d, w.WD_FP16, 0) + 512)
                 for d in small_sizes)
    arena_bytes = gauges + per_group + (1 << 20)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = w.wd_server_create(arena, w.WD_FP16, check_every=8, delta=0.1, max_rhs_per_group=4,
                             n_streams=2)
    try:
        lat = make_pool(srv, small_sizes, 2)
        done, wall, _ = run_stream(srv, lat, [draw(lat, 4) for _ in range(16)], [None] * 16)
        wait_s = np.array([res["t_start"] - res["t_submit"] for rc, res, _ in done.values()])
        info = w.wd_server_info(srv)
        out["small_arena"] = {
            "arena_mb": round(arena_bytes / 1e6, 1), "requests": 16,
            "ok": int(sum(rc == w.WD_OK for rc, _, _ in done.values())),
            "arena_peak_mb": round(info["arena_peak"] / 1e6, 1),
            "queue_wait_p50_ms": pct(wait_s, 50), "queue_wait_max_ms": pct(wait_s, 100),
            "max_true_rel_residual": worst_residual(lat, done)}
    finally:
        w.wd_server_destroy(srv)
    return out


def main(argv=None):
    args = parse(argv)
    global TUNE
    TUNE = not args.no_tune
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path is a single-GPU whole-lattice operator)", file=sys.stderr)
        return 2

    import torch
    import lattice_inputs as li
    import paper_1901_07294_amd.wilson as w
    from paper_1901_07294_amd.buffers import DeviceGauge

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)

    if args.copy_calib:
        gbs = copy_calibration(torch)
        print(json.dumps({"copy_calibration_bytes": 1 << 30, "copy_gbs": round(gbs, 1)}))
        return 0

    dims = tuple(int(v) for v in args.dims.split(","))
    V = li.volume(dims)
    mass = 0.1
    prec_id = {"fp64": w.WD_FP64, "fp32": w.WD_FP32, "fp16": w.WD_FP16}
    print(f"[bench] generating inputs dims={dims}", file=sys.stderr, flush=True)
    t0 = time.time()
    U = li.random_gauge(dims, li.seed_gauge(CONFIG_INDEX))
    psi = li.gaussian_spinor(dims, li.seed_spinor(CONFIG_INDEX))
    print(f"[bench] inputs ready in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    Ud = torch.from_numpy(U).to("cuda")
    psid = torch.from_numpy(psi).to("cuda")

    def measure(prec: str, c12: bool, steps: int, warmup: int):
        g = DeviceGauge(Ud, prec_id[prec], c12)
        src = g.spinor()
        dst = g.spinor()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        w.wd_spinor_import(g.handle, psid, g.prec, 1, src)
        e1.record()
        torch.cuda.synchronize()
        pack_ms = e0.elapsed_time(e1)
        if args.tuning and (prec, c12) == (args.prec, args.c12):
            tuned = force_tuning(w, dims, prec_id[prec], c12, args.tuning)
        else:
            tuned = tune(torch, w, g, 1, src)
        ms = time_applies(torch, w, g, src, dst, mass, steps, warmup)
        return g, src, dst, ms, pack_ms, tuned

    print(f"[bench] timing {args.prec} c12={args.c12}", file=sys.stderr, flush=True)
    g, src, dst, ms, pack_ms, tuned = measure(args.prec, args.c12, args.steps, args.warmup)
    t_s = ms / 1e3
    gflops = FLOPS_PER_SITE * V / t_s / 1e9
    cbytes = compulsory_bytes(args.prec, args.c12)
    achieved = cbytes * V / t_s / 1e9

    # parity on sampled sites (outside the timed region)
    import oracle
    out = g.unpack(dst).reshape(-1, 4, 3)
    rng = np.random.default_rng(7)
    sites = rng.choice(V, min(V, 2048), replace=False)
    ref = oracle.dslash_sites(U, psi, mass, sites)
    parity = float(np.linalg.norm(out[sites] - ref) / np.linalg.norm(ref))
    tol = {"fp64": 1e-13, "fp32": 1e-6, "fp16": 2e-3}[args.prec]
    del g, src, dst

    variants = {}
    if not args.no_variants:
        for p, c in (("fp64", False), ("fp64", True), ("fp32", False), ("fp32", True),
                     ("fp16", False), ("fp16", True)):
            if (p, c) == (args.prec, args.c12):
                continue
            # the median of three timed batches of the headline's step count
            gv, sv, dv, msv, _, tv = measure(p, c, args.steps, max(20, args.warmup))
            batches = sorted([msv] + [time_applies(torch, w, gv, sv, dv, mass, args.steps, 5) for _ in range(2)])
            msv = batches[1]
            outv = gv.unpack(dv).reshape(-1, 4, 3)
            errv = float(np.linalg.norm(outv[sites[:512]] - ref[:512]) / np.linalg.norm(ref[:512]))
            tolv = {"fp64": 1e-13, "fp32": 1e-6, "fp16": 2e-3}[p]
            variants[f"{p}{'_c12' if c else ''}"] = {
                "ms_per_apply": round(msv, 5), "batches_ms": [round(b, 5) for b in batches],
                "applies_per_batch": args.steps, "tuning": tv,
                "parity": {"rel_err": errv, "tol": tolv, "sites": 512, "ok": errv <= tolv},
                "gflops": round(FLOPS_PER_SITE * V / (msv / 1e3) / 1e9, 1),
                "pct_hbm_peak": round(100 * compulsory_bytes(p, c) * V / (msv / 1e3) / 1e9
                                      / HBM_PEAK_GBS, 2)}
            del gv, sv, dv
    copy_gbs = copy_calibration(torch)
    triad_gbs = stream_triad(torch)
    del Ud, psid
    multi = None
    if not args.no_multi:
        print("[bench] multi-RHS 24^3x48 x12", file=sys.stderr, flush=True)
        mdims = (24, 24, 24, 48)
        minputs = (li.near_unity_gauge(mdims, li.seed_gauge(3), 0.3),
                   li.gaussian_spinors(mdims, [li.seed_spinor(3, k) for k in range(12)]))
        multi = {p: bench_multi(torch, w, li, DeviceGauge, p, inputs=minputs) for p in ("fp32", "fp16")}
        del minputs
    cg = None
    if not args.no_cg:
        print("[bench] CG 24^4", file=sys.stderr, flush=True)
        cg = bench_cg(torch, w, li, DeviceGauge, cpu=not args.no_cpu_baseline)
    cg_multi = None
    if not args.no_cg_multi:
        print("[bench] CG 24^4 x12", file=sys.stderr, flush=True)
        cg_multi = bench_cg_multi(torch, w, li, DeviceGauge,
                                  single_fp64_ms=cg["fp64"]["ms_per_solve"] if cg else None)
    wilson = None
    if not args.no_wilson:
        print("[bench] D x = b 24^4, normal equations and even-odd", file=sys.stderr, flush=True)
        wilson = bench_wilson(torch, w, li, DeviceGauge)
    print("[bench] latency 4^4", file=sys.stderr, flush=True)
    latency = bench_latency(torch, w, li, DeviceGauge, oracle)

    workload = "wilson_dslash_" + "x".join(map(str, dims))
    key = f"{workload}_{args.prec}{'_c12' if args.c12 else ''}"
    traffic = None
    rec = TRAFFIC.get(key)
    launch = ",".join(str(tuned[k]) for k in ("tb", "gw", "group", "rb")) if tuned else None
    if rec and rec["source_sha"] == kernel_source_hash() and launch in rec["launches"]:
        traffic = rec["launches"][launch]

    serve = None
    if not args.no_serve:
        print("[bench] request server", file=sys.stderr, flush=True)
        serve = bench_serve(torch, w, li, DeviceGauge, n_req=args.serve_requests)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle (one full application)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        oracle.dslash(U, psi, mass)
        tc = time.perf_counter() - t0
        cpu = {"value": round(FLOPS_PER_SITE * V / tc / 1e9, 4), "unit": "GFlop/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one full FP64 application on the {'x'.join(map(str, dims))} lattice "
                         f"({tc:.1f} s, numpy, single thread, {os.cpu_count()} host cores visible, "
                         f"{cpu_model()})"}

    line = {
        "metric": METRIC,
        "value": round(gflops, 1),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32",  # FP16 storage computes in FP32
        "data": "synthetic (seeded random SU(3) links, Gaussian spinor)",
        "config": {"workload": workload, "dims": list(dims), "prec": args.prec,
                   "links": "12-real" if args.c12 else "full", "mass": mass,
                   "gauge": "random SU(3)", "boundary": "periodic"},
        "pct_hbm_peak": round(100 * achieved / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": cbytes * V},
        "parity": {"rel_err": parity, "tol": tol, "sites": int(len(sites)), "ok": parity <= tol},
        "pack_ms": round(pack_ms, 4),
        "tuning": tuned,
        "torch_copy_gbs": round(copy_gbs, 1),
        "stream_triad_gbs": round(triad_gbs, 1),
        "variants": variants,
        "latency_4x4x4x4": latency,
        "multi_rhs": multi,
        "cg": cg,
        "cg_multi_rhs": cg_multi,
        "wilson_solve": wilson,
        "serve": serve,
        "kernel_source_sha": kernel_source_hash(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0 if parity <= tol else 3


if __name__ == "__main__":
    sys.exit(main())
