"""The arithmetic behind the committed rocprofv3 summaries and bench.py's
`roofline.traffic`, on synthetic rocprofv3 output (no GPU): counter
averaging over the last dispatches, scaling by the calibration copy, the
kernel-source hash that invalidates stale summaries, and the kernel
statistics reader."""
import argparse
import csv
import json
import os

import pytest

import bench
from paper_1110_0899_amd import profiling


def write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, kern, name, val in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": kern, "Counter_Name": name,
                        "Counter_Value": val})
    return d


def test_counter_summary_arithmetic(tmp_path):
    k = "void wolff::team_kernel<256, 2>(wolff::Rep*)"
    # dispatch ids out of order: the reader sorts them before taking the last n
    fetch = write_counters(str(tmp_path / "f"), [(7, k, "FETCH_SIZE", 300.0), (3, k, "FETCH_SIZE", 100.0),
                                                  (5, k, "FETCH_SIZE", 200.0),
                                                  (9, "other_kernel", "FETCH_SIZE", 1e9)])
    write = write_counters(str(tmp_path / "w"), [(3, k, "WRITE_SIZE", 50.0), (5, k, "WRITE_SIZE", 60.0),
                                                  (7, k, "WRITE_SIZE", 70.0)])
    # the calibration copy moves 1 GiB each way; FETCH_SIZE reads half of it
    cf = write_counters(str(tmp_path / "cf"), [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0)])
    cw = write_counters(str(tmp_path / "cw"), [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)])
    out = str(tmp_path / "summary.json")
    a = argparse.Namespace(kernel="team_kernel", workload="2d", fetch=fetch, write=write,
                           copy_fetch=cf, copy_write=cw, out=out, command="cmd", last=2, added=1000.0)
    profiling.counters(a)
    d = json.load(open(out))
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert d["dispatches"] == 2
    assert d["fetch_kib_per_dispatch_raw"] == 250.0 and d["write_kib_per_dispatch_raw"] == 65.0
    fetch_b, write_b = 250.0 * 1024 * 2.0, 65.0 * 1024
    assert d["hbm_bytes_per_launch"] == pytest.approx(fetch_b + write_b, rel=1e-12)
    assert d["added_spins_per_launch"] == 500.0
    assert d["hbm_bytes_per_added_spin"] == pytest.approx((fetch_b + write_b) / 500.0, rel=1e-12)
    assert d["kernel_source_sha"] == profiling.kernel_source_sha()


def test_stale_summary_is_ignored(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = {"kernel_source_sha": profiling.kernel_source_sha(), "hbm_bytes_per_launch": 123.0,
            "hbm_bytes_per_added_spin": 2.5}
    (prof / "counters_k_w.json").write_text(json.dumps(good))
    (prof / "counters_k_old.json").write_text(json.dumps(dict(good, kernel_source_sha="0" * 16)))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # bytes per added spin of the counter run, times this run's spins per launch
    assert bench.counter_traffic("k", "w", 1000.0) == 2500.0
    assert bench.counter_traffic("k", "old", 1000.0) is None
    assert bench.counter_traffic("k", "missing", 1000.0) is None


def test_source_hash_covers_device_code_only():
    # the hash follows the device sources; the host library is not part of it
    assert "wolff_lib.hip" not in profiling.DEVICE_SOURCES
    csrc = os.path.join(os.path.dirname(profiling.__file__), "csrc")
    assert all(os.path.exists(os.path.join(csrc, n)) for n in profiling.DEVICE_SOURCES)
    assert {"wolff_kernels.hip", "wolff_device.h"} <= set(profiling.DEVICE_SOURCES)
    # every file the kernels include (directly or through a hashed header) is hashed
    for n in profiling.DEVICE_SOURCES:
        with open(os.path.join(csrc, n)) as f:
            for line in f:
                if line.startswith('#include "'):
                    inc = line.split('"')[1]
                    if os.path.exists(os.path.join(csrc, inc)):
                        assert inc in profiling.DEVICE_SOURCES, (n, inc)


def test_kernel_stats_reader(tmp_path):
    d = tmp_path / "stats"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow(["void wolff::team_kernel<256, 2>(wolff::Rep*)", 4, 4000.0, 1000.0, 90.0])
        w.writerow(["__amd_rocclr_copyBuffer", 2, 20.0, 10.0, 10.0])
    rows = profiling.kernel_stats(str(d))
    assert rows[0] == ("void wolff::team_kernel<256, 2>(wolff::Rep*)", 4, 4.0, 1.0, 90.0)
    out = tmp_path / "s.md"
    profiling.write_stats(str(d), str(out), "cmd --x", note="a note")
    text = out.read_text()
    assert "    cmd --x" in text and "a note" in text
    assert "| `void wolff::team_kernel<256, 2>` | 4 | 4.0 | 1.000 | 90.00 |" in text
    assert text.strip().endswith(profiling.kernel_source_sha())


def test_pmc_table_sums_the_last_dispatches(tmp_path):
    # one --pmc run with two counters: the table averages each counter over
    # the kernel's last n dispatches (sorted by id) and divides the sum by
    # the added spins; other kernels' rows are left out
    k = "void wolff::lds_kernel<512, 2, true>(wolff::LdsArgs, unsigned int)"
    d = write_counters(str(tmp_path / "sq"), [
        (4, k, "SQ_INSTS_VALU", 40.0), (2, k, "SQ_INSTS_VALU", 20.0), (6, k, "SQ_INSTS_VALU", 60.0),
        (2, k, "SQ_INSTS_LDS", 2.0), (4, k, "SQ_INSTS_LDS", 4.0), (6, k, "SQ_INSTS_LDS", 6.0),
        (5, "wolff::init_kernel", "SQ_INSTS_VALU", 1e9)])
    out = str(tmp_path / "sq.md")
    a = argparse.Namespace(kernel="lds_kernel", dir=d, out=out, command="cmd", last=2, added=10.0,
                           note="")
    profiling.pmc_table(a)
    text = open(out).read()
    assert "`void wolff::lds_kernel<512, 2, true>`" in text
    assert "| `SQ_INSTS_VALU` | 50 | 10 |" in text          # (40 + 60) / 2, (40 + 60) / 10
    assert "| `SQ_INSTS_LDS` | 5 | 1 |" in text
    assert profiling.kernel_source_sha() in text


def test_source_hash_ignores_comments_only():
    # a documentation edit keeps the hash, a change to a token does not
    src = 'int f(int a) { // add one\n  return a + 1; /* sum */ }\nconst char* s = "x // y";\n'
    doc = 'int f(int a)\n{\n    /* adds one */ return a + 1;\n}\nconst char* s = "x // y"; // text\n'
    code = 'int f(int a) { return a + 2; }\nconst char* s = "x // y";\n'
    assert profiling.code_tokens(src) == profiling.code_tokens(doc)
    assert profiling.code_tokens(src) != profiling.code_tokens(code)
    assert '"x // y"' in profiling.code_tokens(src)
    assert profiling.code_tokens("a /* b */ c") == "a c"
    assert profiling.code_tokens("char c = '\\'';") == "char c = '\\'';"
