"""Host-side helpers of bench.py: the counter summaries read rocprofv3 counter CSVs
(synthetic ones here) and the traffic lookup refuses counters taken on other
kernel sources."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_counter_summary_averages_per_dispatch(tmp_path):
    p = str(tmp_path / "c.csv")
    rows = []
    for d, (valu, salu, wait, cyc) in enumerate([(100, 50, 30, 60), (300, 150, 90, 180)]):
        for name, v in (("SQ_WAVES", 8), ("SQ_INSTS_VALU", valu), ("SQ_INSTS_SALU", salu),
                        ("SQ_WAIT_ANY", wait), ("SQ_WAVE_CYCLES", cyc)):
            rows.append((d, "k_q_dense(DevGraph, int const*)", name, v))
    rows.append((9, "some_other_kernel()", "SQ_WAVES", 1))
    _csv(p, rows)
    out = bench.counter_summary([p]).splitlines()
    assert len(out) == 2  # header + the one timed kernel present
    row = out[1].split()
    assert row[0] == "qh_dense"
    assert float(row[1]) == 8.0 and float(row[2]) == 200.0  # waves, VALU per dispatch
    assert row[-2] == "0.50" and row[-1] == "0.50"  # SALU/VALU, wait fraction


def test_traffic_summary_scales_by_copy(tmp_path):
    f, w, cf, cw = (str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv"))
    _csv(f, [(1, "k_q_dense(DevGraph)", "FETCH_SIZE", 1000.0)])
    _csv(w, [(1, "k_q_dense(DevGraph)", "WRITE_SIZE", 500.0)])
    # the copy reads and writes 1 MiB = 1024 KiB; the counters read half and all of it
    _csv(cf, [(2, "void at::native::direct_copy_kernel_cuda(x)", "FETCH_SIZE", 512.0)])
    _csv(cw, [(2, "void at::native::direct_copy_kernel_cuda(x)", "WRITE_SIZE", 1024.0)])
    text = bench.traffic_summary(f, w, cf, cw, copy_mib=1)
    lines = dict((l.split()[0], l.split()[1:]) for l in text.splitlines() if not l.startswith("kernel"))
    assert lines["source_digest"][0] == bench.source_digest()
    assert abs(float(lines["fetch_scale"][0]) - 2.0) < 1e-9
    k = [l.split() for l in text.splitlines() if l.startswith("kernel qh_dense")][0]
    assert float(k[3]) == 2.0 * 1000.0 * 1024 and float(k[5]) == 500.0 * 1024


def test_traffic_lookup_refuses_other_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_w.txt").write_text("source_digest 0000000000000000\nkernel qh_dense fetch_bytes 1 write_bytes 2\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("w", "qh_dense") is None
    (prof / "traffic_w.txt").write_text(f"source_digest {bench.source_digest()}\n"
                                        "kernel qh_dense fetch_bytes 1 write_bytes 2\n")
    assert bench.traffic_for("w", "qh_dense") == 3
