"""The profile summariser: kernel-name parsing, counter scaling by the copy probe, and the
source hash that gates the traffic bench.py reports (no GPU)."""
import csv
import os

import pytest

from paper_1302_7203_amd import profiling as P


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_short_name():
    assert P.short_name("void k_root<0, 64, true>(ahd::ProbDesc, ahd::Options)") == "k_root<0, 64, true>"
    assert P.short_name("(anonymous namespace)::k_probe_copy(double*, double const*, long)") == "k_probe_copy"


def test_summary_scales_counters_by_the_copy_probe(tmp_path):
    kt, pf, pw = (str(tmp_path / x) for x in ("kt", "pf", "pw"))
    _write(f"{kt}/run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [["void k_vec<0, 2>(ahd::ProbDesc, int)", 2, 60000, 30000],
            ["(anonymous namespace)::k_probe_copy(double*, double const*, long)", 1, 1000, 1000]])
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    copy = "(anonymous namespace)::k_probe_copy(double*, double const*, long)"
    vec = "void k_vec<0, 2>(ahd::ProbDesc, int)"
    _write(f"{pf}/run_counter_collection.csv", hdr, [[copy, "FETCH_SIZE", 512], [vec, "FETCH_SIZE", 10],
                                                     [vec, "FETCH_SIZE", 30]])
    _write(f"{pw}/run_counter_collection.csv", hdr, [[copy, "WRITE_SIZE", 2048], [vec, "WRITE_SIZE", 100]])
    doc = P.summarize(kt, pf, pw, copy_bytes=1 << 20, command="x")
    assert doc["copy_probe"]["fetch_scale"] == pytest.approx(2.0)    # 1 MiB known / 512 KiB counted
    assert doc["copy_probe"]["write_scale"] == pytest.approx(0.5)
    v = doc["kernels"]["k_vec<0, 2>"]
    assert v["avg_us"] == pytest.approx(30.0) and v["fetch_kib"] == pytest.approx(20.0)
    assert v["hbm_bytes"] == pytest.approx(20 * 1024 * 2.0 + 100 * 1024 * 0.5)
    assert doc["source_sha256"] == P.source_hash()
    md = P.markdown(doc, "t")
    assert "k_vec<0, 2>" in md and "scale 2.0000" in md


def test_source_hash_is_stable_and_hex():
    h = P.source_hash()
    assert h == P.source_hash() and len(h) == 64 and int(h, 16) >= 0
