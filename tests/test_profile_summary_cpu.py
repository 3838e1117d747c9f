"""Host logic behind the reported HBM traffic: per-dispatch counters from a
rocprofv3 --pmc CSV, scaled by what the same counter reads for a copy of a
known size (synthetic CSVs with known answers)."""
import csv
import json

from paper_1512_02390_amd import profile_summary as ps

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": v})
    return str(path)


def test_traffic_scaling(tmp_path):
    mib = 1 << 20
    copy_bytes = 256 * mib
    # the copy reads half of its bytes in FETCH_SIZE units and all of them in WRITE_SIZE
    cf = _csv(tmp_path / "cf.csv", "FETCH_SIZE", [("fill", 17.0), ("copyBuffer", 128 * 1024.0)])
    cw = _csv(tmp_path / "cw.csv", "WRITE_SIZE", [("copyBuffer", 256 * 1024.0)])
    kern = "void k_fdm2<double, 11>(FdmArgs)"
    f = _csv(tmp_path / "f.csv", "FETCH_SIZE", [(kern, 1000.0), ("other", 5.0), (kern, 3000.0)])
    w = _csv(tmp_path / "w.csv", "WRITE_SIZE", [(kern, 4000.0), (kern, 6000.0)])
    js, md = tmp_path / "t.json", tmp_path / "t.md"
    ps.traffic(f, w, cf, cw, copy_bytes, "k_fdm2<double, 11>", "c2", "hash1", str(js), str(md),
               "cmd a;;cmd b")
    rec = json.load(open(js))
    # fetch: mean 2000 KiB x factor 2; write: mean 5000 KiB x factor 1
    want = 2000 * 1024 * 2.0 + 5000 * 1024 * 1.0
    assert rec["source_hash"] == "hash1"
    assert abs(rec["per_launch"]["c2"] - want) < 1e-6 * want
    d = rec["detail"]["c2"]
    assert d["dispatches"] == [2, 2]
    assert abs(d["copy_factor_fetch"] - 2.0) < 1e-12 and abs(d["copy_factor_write"] - 1.0) < 1e-12
    text = open(md).read()
    assert "cmd a" in text and "cmd b" in text
    # a second key with the same hash is added; a new hash starts a new record
    ps.traffic(f, w, cf, cw, copy_bytes, "k_fdm2<double, 11>", "c3", "hash1", str(js), str(md), "x")
    assert sorted(json.load(open(js))["per_launch"]) == ["c2", "c3"]
    ps.traffic(f, w, cf, cw, copy_bytes, "k_fdm2<double, 11>", "c3", "hash2", str(js), str(md), "x")
    assert sorted(json.load(open(js))["per_launch"]) == ["c3"]


def test_kernel_stats_summary(tmp_path):
    src = tmp_path / "stats.csv"
    with open(src, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow(["k_a", 4, 4000, 1000, 80.0])
        w.writerow(["k_b", 1, 1000, 1000, 20.0])
    dst = tmp_path / "out.md"
    ps.main(str(src), str(dst), "the command")
    text = open(dst).read()
    assert "the command" in text and "`k_a`" in text and "`k_b`" in text
    assert "Total kernel time: 5.0 us" in text


def test_kernel_hash_ignores_comments_and_layout():
    import bench
    files = bench.KERNEL_SOURCES
    base = {f: "int a = 1;\nint b = 2;\n" for f in files}
    commented = dict(base)
    commented["fdm_impl.h"] = "// header\nint a = 1;   /* one */\n\n  int b = 2; // two\n"
    changed = dict(base)
    changed["residual_impl.h"] = "int a = 1;\nint b = 3;\n"
    h = bench.kernel_source_hash(base)
    assert bench.kernel_source_hash(commented) == h
    assert bench.kernel_source_hash(changed) != h
    # the tree's own hash is what the recorded traffic is keyed by
    assert len(bench.kernel_source_hash()) == 16
