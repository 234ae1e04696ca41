"""The autotuner's cache file: load, save, lookup and validation (host only).

A loaded choice drives kernel launches, so every line is checked against its
lattice (bounds, lanes, LDS) and a file with any invalid line is rejected
whole.
"""

import pytest

import paper_1901_07294_amd.wilson as w

HEADER = "# wilson dslash launch tuning v2: X Y Z T prec c12 nrhs tb gw group rb\n"
PROD = (32, 32, 32, 64)


@pytest.fixture(autouse=True)
def _clean():
    w.wd_tune_reset()
    yield
    w.wd_tune_reset()


def write(path, lines, header=HEADER):
    path.write_text(header + "".join(line + "\n" for line in lines))
    return str(path)


def test_load_lookup_save_roundtrip(tmp_path):
    assert w.wd_tune_lookup(PROD, w.WD_FP64, 0, 1) is None
    f = write(tmp_path / "a.txt", ["32 32 32 64 0 0 1 16 1 0 1",
                                   "24 24 24 48 1 0 12 48 4 27 1",
                                   "24 24 24 48 2 1 12 12 1 0 2"])
    assert w.wd_tune_load(f) == w.WD_OK
    assert w.wd_tune_lookup(PROD, w.WD_FP64, 0, 1) == (16, 1, 0, 1)
    assert w.wd_tune_lookup(PROD, w.WD_FP64, 1, 1) is None   # other link format
    assert w.wd_tune_lookup(PROD, w.WD_FP64, 0, 2) is None   # other nrhs
    assert w.wd_tune_lookup((24, 24, 24, 48), w.WD_FP32, 0, 12) == (48, 4, 27, 1)
    g = tmp_path / "b.txt"
    assert w.wd_tune_save(str(g)) == w.WD_OK
    w.wd_tune_reset()
    assert w.wd_tune_lookup(PROD, w.WD_FP64, 0, 1) is None
    assert w.wd_tune_load(str(g)) == w.WD_OK
    assert w.wd_tune_lookup((24, 24, 24, 48), w.WD_FP16, 1, 12) == (12, 1, 0, 2)
    assert g.read_text().splitlines()[0] == HEADER.strip()


@pytest.mark.parametrize("line,why", [
    ("32 32 32 64 0 0 1 0 1 0 1", "no t steps"),
    ("32 32 32 64 0 0 1 65 1 0 1", "more t steps than T"),
    ("32 32 32 64 0 0 2 16 2 0 1", "two FP64 tiles do not fit the LDS"),
    ("24 24 24 48 1 0 12 8 5 0 1", "gw does not divide nrhs"),
    ("24 24 24 48 1 0 12 8 12 0 1", "12 x 192 lanes exceed a workgroup"),
    ("24 24 24 48 1 0 17 8 1 0 1", "nrhs above 16"),
    ("32 32 32 64 3 0 1 16 1 0 1", "unknown precision"),
    ("32 32 32 64 0 2 1 16 1 0 1", "bad link format"),
    ("32 32 32 64 0 0 1 16 1 -1 1", "negative XCD run"),
    ("300 2 2 2 0 0 1 1 1 0 1", "x rows longer than a workgroup: no t-marching kernel"),
    ("32 32 0 64 0 0 1 16 1 0 1", "zero extent"),
    ("32 32 32 64 0 0 1 16 1", "nine fields"),
    ("32 32 32 64 0 0 1 16 1 0 1 7", "twelve fields"),
    ("32 32 32 64 0 0 2 16 1 0 2", "two right-hand sides per lane need FP32 arithmetic"),
    ("24 24 24 48 1 0 12 8 2 0 2", "two per lane with two lane groups"),
    ("24 24 24 48 1 0 12 8 1 0 3", "three per lane"),
    ("24 24 24 48 1 0 3 8 1 0 2", "two per lane do not divide three right-hand sides"),
    ("32 32 32 64 0 0 1 sixteen 1 0 1", "not an integer"),
])
def test_invalid_lines_reject_the_whole_file(tmp_path, line, why):
    f = write(tmp_path / "bad.txt", ["32 32 32 64 1 0 1 16 1 0 1", line])
    with pytest.raises(w.WilsonError) as e:
        w.wd_tune_load(f)
    assert e.value.code == w.WD_ERR_INVALID_ARG, why
    assert w.wd_tune_lookup(PROD, w.WD_FP32, 0, 1) is None  # nothing registered


def test_bad_files(tmp_path):
    for body in ("", "no header\n32 32 32 64 0 0 1 16 1 0\n"):
        p = tmp_path / "f.txt"
        p.write_text(body)
        with pytest.raises(w.WilsonError):
            w.wd_tune_load(str(p))
    with pytest.raises(w.WilsonError):
        w.wd_tune_load(str(tmp_path / "missing.txt"))
    p = tmp_path / "long.txt"
    p.write_text(HEADER + "1" * 1000 + "\n")
    with pytest.raises(w.WilsonError):
        w.wd_tune_load(str(p))
    # a header-only file is valid and registers nothing
    assert w.wd_tune_load(write(tmp_path / "h.txt", [])) == w.WD_OK
    assert w.wd_tune_lookup(PROD, w.WD_FP64, 0, 1) is None
