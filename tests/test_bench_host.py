"""Host logic of bench.py (no GPU): the algorithmic byte counts of the
measurement (one 4-byte index and one value per factor entry and sweep,
plus the per-row vector terms), the counter traffic read back from a
committed profile only while it matches the kernel sources, summed over the
launches of a sweep, and the roofline's choice and labels."""
import bench


def test_byte_counts_per_unit():
    # forward: n_off (4 + e) + 20 N (FP64) / 10 N (FP32); backward 28 N / 14 N
    assert bench.fwd_bytes(10, 3, 8) == 10 * 12 + 60
    assert bench.fwd_bytes(10, 3, 4) == 10 * 8 + 30
    assert bench.bwd_bytes(10, 3, 8) == 10 * 12 + 84
    assert bench.bwd_bytes(10, 3, 4) == 10 * 8 + 42
    # elimination: 12 E + 40 n_fill + 20 n_off + 24 N
    assert bench.elim_bytes(5, 7, 11, 13) == 60 + 280 + 220 + 312


def profile(tmp_path, sha, lines):
    p = tmp_path / "traffic.md"
    p.write_text("\n".join(lines + ["", "kernel-sources-sha256: %s" % sha]) + "\n")
    return str(p)


def test_measured_traffic_sums_launches_and_checks_the_sources(tmp_path, monkeypatch):
    sha = bench.kernel_source_hash()
    lines = ["hbm-bytes-per-launch k_ready<double, false, 1>: 100",
             "hbm-bytes-per-launch k_narrow_prep<double>: 20",
             "hbm-bytes-per-launch k_narrow<double, false, 3>: 3"]
    monkeypatch.setitem(bench.TRAFFIC_PROFILES, "w", profile(tmp_path, sha, lines))
    assert bench.measured_traffic("w", "k_ready<double, false, 1>") == 100
    assert bench.measured_traffic("w", ["k_ready<double, false, 1>", "k_narrow_prep<double>",
                                        "k_narrow<double, false, 3>"]) == 123
    # a launch the profile does not list: no figure rather than a partial sum
    assert bench.measured_traffic("w", ["k_ready<double, false, 1>", "k_eliminate"]) is None
    # taken from other kernel sources: not reported
    monkeypatch.setitem(bench.TRAFFIC_PROFILES, "w", profile(tmp_path, "0" * 64, lines))
    assert bench.measured_traffic("w", "k_ready<double, false, 1>") is None
    assert bench.measured_traffic("no such workload", "k_eliminate") is None


def test_roofline_names_the_launches_of_a_sweep():
    info = {"n": 1000, "nnz_off": 9000, "n_input_edges": 3000, "n_fill": 8000, "depth": 50,
            "narrow_levels": 20}
    timing = {"fwd_ms": 1.0, "bwd_ms": 0.9, "elim_ms": 5.0, "applies": 10}
    r = bench.roofline(info, timing, 8, "not profiled")
    assert r["kernel"].startswith("forward sweep")  # 10 x 1.0 ms > 5.0 ms
    assert "k_narrow_prep<double>" in r["kernel"] and "3 launches" in r["kernel"]
    assert r["algorithmic_bytes"] == bench.fwd_bytes(9000, 1000, 8)
    assert abs(r["achieved"] - r["algorithmic_bytes"] / 1e-3 / 1e9) < 0.01
    assert r["traffic"] is None
    names = [o["kernel"] for o in r["others"]]
    assert any(n.startswith("backward sweep") and "k_narrow<double, true, 3>" in n for n in names)
    # no narrow levels: each sweep is its one launch; a long elimination dominates
    info["narrow_levels"] = 0
    timing["elim_ms"] = 50.0
    r = bench.roofline(info, timing, 4, "not profiled")
    assert r["kernel"].startswith("k_eliminate")
    fwd = [o for o in r["others"] if o["kernel"].startswith("forward")][0]
    assert "k_ready<float, false, 1>: 1 launches" in fwd["kernel"]
    assert fwd["algorithmic_bytes"] == bench.fwd_bytes(9000, 1000, 4)
