"""bench.py's command-line contract on the CPU: one GPU only, and the traffic
table refers to the kernel sources it was measured on."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_defaults_and_tuning_option():
    a = bench.parse([])
    assert a.gpus == 1 and a.steps > 0 and a.warmup >= 0 and a.prec == "fp64" and a.tuning is None
    assert bench.parse(["--tuning", "32,1,32,1"]).tuning == "32,1,32,1"


def test_traffic_table_entries_name_launches_and_byte_counts():
    for key, rec in bench.TRAFFIC.items():
        assert key.startswith("wilson_dslash_")
        assert len(rec["source_sha"]) == 16
        for launch, nbytes in rec["launches"].items():
            assert len(launch.split(",")) == 4 and nbytes > 0
    # the FP64 entry exceeds the compulsory 960 B/site (reads are never below compulsory)
    v = 32 * 32 * 32 * 64
    for nbytes in bench.TRAFFIC["wilson_dslash_32x32x32x64_fp64"]["launches"].values():
        assert nbytes >= 960 * v


def test_source_hash_ignores_comments_but_not_code():
    src = ('int a = 1; // note "x"\n'
           '/* block\n   comment */ int b = \'/\';\n'
           'const char* s = "// kept \\" /* kept */";\n'
           '\n'
           'int c;   \n')
    stripped = bench.strip_comments(src)
    assert stripped == ('int a = 1;\n'
                        '  int b = \'/\';\n'
                        'const char* s = "// kept \\" /* kept */";\n'
                        'int c;')
    # a comment edit (even one that adds lines) leaves the code, a code edit does not
    assert bench.strip_comments(src.replace("// note", "// another\n// note")) == stripped
    assert bench.strip_comments(src.replace("int c;", "int d;")) != stripped


def test_multi_rhs_roof_is_the_smaller_of_hbm_and_alu():
    # FP32, 12 fields: links once (288 B) + 12 x (in + out) (96 B each) = 2592 B per site;
    # 8 TB/s x 12 x 1320 / 2592 = 48.9 TFLOP/s, below the 78.6 TFLOP/s vector peak
    r = bench.multi_roof(12, 2592, 19201.7)
    assert r["bound"] == "hbm" and abs(r["roof_gflops"] - 8000 * 12 * 1320 / 2592) < 0.1
    assert abs(r["frac"] - 19201.7 / (8000 * 12 * 1320 / 2592)) < 1e-4
    # FP16 storage: 144 + 12 x 2 x 52 = 1392 B per site would allow 91 TFLOP/s: ALU-bound
    r = bench.multi_roof(12, 1392, 26032.7)
    assert r["bound"] == "alu" and r["roof_gflops"] == bench.FP32_VECTOR_PEAK_GFLOPS
    assert abs(r["frac"] - 26032.7 / 78600.0) < 1e-4
