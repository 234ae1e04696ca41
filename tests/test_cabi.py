"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/*.h declares, and answers size queries (no GPU work)."""

import glob
import os
import re

import pytest

import paper_1901_07294_amd.wilson as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        names.update(re.findall(r"^WD_API\s+[^;(]*?\b(\w+)\s*\(", text, flags=re.M))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(w.LIB_PATH):
        pytest.fail(f"{w.LIB_PATH} missing: run python -m paper_1901_07294_amd.build")
    return w._L()


def test_header_declares_entry_points():
    names = declared_symbols()
    assert {"wd_abi_version", "wd_last_error", "wd_gauge_import", "dslash_apply"} <= names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing
    assert set(w.SIGNATURES) == declared_symbols()


def test_exports_only_the_abi():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", w.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported == declared_symbols()


def test_version_and_sizes(lib):
    assert w.wd_abi_version() == 4
    d = (32, 32, 32, 64)
    V = 32 ** 3 * 64
    assert w.wd_spinor_bytes(d, w.WD_FP64, 1) == 192 * V
    assert w.wd_spinor_bytes(d, w.WD_FP32, 3) == 3 * 96 * V
    assert w.wd_gauge_bytes(d, w.WD_FP64, 0) == 576 * V
    assert w.wd_gauge_bytes(d, w.WD_FP64, 1) == 384 * V
    assert w.wd_gauge_bytes(d, w.WD_FP32, 0) == 288 * V
    assert w.wd_gauge_bytes(d, w.WD_FP32, 1) == 192 * V
    # FP16 storage: 24 binary16 + one FP32 scale per spinor site; unscaled links
    assert w.wd_spinor_bytes(d, w.WD_FP16, 12) == 12 * 52 * V
    assert w.wd_gauge_bytes(d, w.WD_FP16, 0) == 144 * V
    assert w.wd_gauge_bytes(d, w.WD_FP16, 1) == 96 * V
    # padding to whole blocks of 2048 sites
    assert w.wd_spinor_bytes((5, 3, 7, 4), w.WD_FP16, 1) == 2048 * 52
    assert w.wd_spinor_bytes((16, 16, 16, 9), w.WD_FP64, 2) == 2 * 36864 * 192
    assert w.wd_spinor_bytes((17, 16, 16, 9), w.WD_FP64, 1) == 40960 * 192


def test_size_queries_reject_bad_arguments(lib):
    assert w.wd_spinor_bytes((4, 4, 0, 4), w.WD_FP64, 1) == 0
    assert "extent" in w.wd_last_error()
    assert w.wd_spinor_bytes((4, 4, 4, 4), w.WD_FP64, -1) == 0
    assert w.wd_spinor_bytes((4, 4, 4, 4), 9, 1) == 0
    assert w.wd_gauge_bytes((4096, 4096, 4096, 4096), w.WD_FP64, 0) == 0
    assert w.wd_spinor_bytes((1, 1, 1, 1), w.WD_FP64, 0) == 0
