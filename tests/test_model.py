"""The traffic model behind the roofline figures, pinned to the paper's own
access counts (Section 6.1, Table 2) and to direct counting."""
import json
import os

from paper_1908_06094_amd import model

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table2_access_counts():
    t = json.load(open(os.path.join(HERE, "golden", "table2_access_counts.json")))
    for key in ("without_fusion", "with_fusion"):
        row = t[key]
        got = model.plane_accesses(row["edge_reads"], row["edge_writes"], row["node_reads"], row["node_writes"],
                                   t["n_edges"], t["n_nodes"])
        assert got == row["total"]
    # the fused pattern moves more than 3x fewer words (the paper: "more than a factor 2")
    assert t["without_fusion"]["total"] / t["with_fusion"]["total"] > 3.0


def test_kernel_words():
    assert model.STEP_WORDS == 6
    assert model.donor_kernel_words() == 6
    assert model.pass_kernel_words(False) == 7
    assert model.pass_kernel_words(True) == 10


def test_op_counts_consistent():
    c = model.corrective_pass_ops(True)
    u = model.corrective_pass_ops(False)
    d = model.donor_pass_ops()
    assert c.divisions == 3 * 5 + 2 + 1
    assert u.divisions == 3 * 5 + 1
    assert d.divisions == 1
    s3 = model.step_ops(3, True)
    assert s3.total == d.total + 2 * c.total
    # the peak used for the ALU roofline: 256 CUs x 64 FP64 lanes per clock x 2.4 GHz
    assert abs(model.FP64_VALU_OPS_PEAK - 39.3216e12) < 1e9


def test_traffic_record_matches_kernel_source_and_workload():
    """The counter record under profiles/ is attached to a bench line only for
    the workload it was taken on and while the pass kernel's source is the one
    it was taken on (its recorded hash)."""
    import json
    import os

    import bench
    from paper_1908_06094_amd import profsum

    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "traffic_fused_pass_f64.json")
    rec = json.load(open(path))
    kind = rec.get("kernel_kind", "pass")
    sha = profsum.kernel_source_sha()
    if rec["source_sha256"] == sha:
        assert bench.traffic_record(sha, "f64", "latlon-1024x512x80-wave", kind) == rec["bytes_per_launch"]
    else:   # a stale record (the kernel changed since the counters were taken) is never attached
        assert bench.traffic_record(sha, "f64", "latlon-1024x512x80-wave", kind) is None
    sha = rec["source_sha256"]
    assert bench.traffic_record(sha, "f64", "latlon-256x128x60-solid-body", kind) is None
    assert bench.traffic_record("0" * 64, "f64", "latlon-1024x512x80-wave", kind) is None
    assert bench.traffic_record(sha, "f64", "latlon-1024x512x80-wave", "stage") is None   # another kernel
    # calibrated counter bytes per launch: fetched x copy factor + written, averaged over the matching kernels
    f = rec["copy_calibration"]["fetch_factor"]
    kib = [rec["fetch_kib_per_dispatch"][k] * f + rec["write_kib_per_dispatch"][k] for k in rec["fetch_kib_per_dispatch"]]
    assert abs(sum(kib) / len(kib) * 1024 - rec["bytes_per_launch"]) <= 1e-6 * rec["bytes_per_launch"]


def test_last_launches_mean_skips_warmup(tmp_path):
    """The timed-launch mean of a per-dispatch trace: the last n dispatches of
    the named kernel, whatever order the rows come in."""
    from paper_1908_06094_amd import profsum

    rows = ["\"Kind\",\"Kernel_Name\",\"Start_Timestamp\",\"End_Timestamp\""]
    t = 0
    for n, dur in enumerate([5000, 4000, 1000, 1100, 900, 1000]):       # ns; the first two are warm-up
        rows.append(f"\"KERNEL_DISPATCH\",\"void k_pass<double, true>(Geo)\",{t},{t + dur}")
        rows.append(f"\"KERNEL_DISPATCH\",\"void k_other(Geo)\",{t + dur},{t + dur + 7000}")
        t += dur + 10000
    body = [rows[0]] + rows[1:][::-1]                                   # rows out of order
    (tmp_path / "run_kernel_trace.csv").write_text("\n".join(body) + "\n")
    assert abs(profsum.last_launches_mean(str(tmp_path), "k_pass<double", 4) - 1.0) < 1e-12    # us
    assert abs(profsum.last_launches_mean(str(tmp_path), "k_pass<double", 6) - 13000 / 6 / 1e3) < 1e-12
