"""Host-side arithmetic of bench.py that its reported numbers rest on: the
serial FIFO latencies of the served comparison and the HBM-traffic
calibration of the counter summaries (no GPU)."""
import csv
import json
import os

import numpy as np

import bench


def test_fifo_latencies_match_the_waiting_time_formula():
    # independent form: the wait of request i is the largest, over j <= i, of
    # the work arrived in [a_j, a_i) not yet done by a_i (and at least 0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        a = np.cumsum(rng.exponential(1.0, n))
        s = rng.exponential(rng.uniform(0.3, 2.0), n)
        lat, fin = bench.fifo_latencies(a, s)
        for i in range(n):
            wait = max(0.0, max(s[j:i].sum() - (a[i] - a[j]) for j in range(i + 1)))
            assert abs(lat[i] - (wait + s[i])) < 1e-9
        assert abs(fin - (a[-1] + lat[-1])) < 1e-9
    # idle server: no waiting; back-to-back burst: waits add up
    lat, _ = bench.fifo_latencies([0.0, 10.0, 20.0], [1.0, 2.0, 3.0])
    assert lat == [1.0, 2.0, 3.0]
    lat, fin = bench.fifo_latencies([0.0, 0.0, 0.0], [1.0, 2.0, 3.0])
    assert lat == [1.0, 3.0, 6.0] and fin == 6.0


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_pmc_summary_applies_the_copy_calibration(tmp_path, monkeypatch):
    """A 1 GiB copy whose FETCH_SIZE reads 0.5 GiB gives a fetch factor of 2;
    WRITE_SIZE reading it exactly gives 1; the propagation's per-dispatch
    means are scaled by those factors."""
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))  # the summary goes to tmp_path/profiles
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "source-hash")
    kib = 1 << 10
    _counter_csv(tmp_path / "cf.csv", [("copy_kernel", "FETCH_SIZE", (1 << 30) / 2 / kib),
                                       ("small", "FETCH_SIZE", 4.0)])
    _counter_csv(tmp_path / "cw.csv", [("copy_kernel", "WRITE_SIZE", (1 << 30) / kib)])
    _counter_csv(tmp_path / "f.csv", [("imx::k_propagate_pack<false>(...)", "FETCH_SIZE", 1000.0),
                                      ("imx::k_propagate_pack<false>(...)", "FETCH_SIZE", 3000.0),
                                      ("imx::k_fill(...)", "FETCH_SIZE", 9e9)])
    _counter_csv(tmp_path / "w.csv", [("imx::k_propagate_pack<false>(...)", "WRITE_SIZE", 500.0)])

    class A:
        pmc_summary = [str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv")]
        copy_calibration = 1024
        workload = "unit"
        pmc_command = "test"

    bench.pmc_summary(A)
    d = json.load(open(os.path.join(tmp_path, "profiles", "propagate_unit_pmc.json")))
    assert abs(d["copy_calibration"]["fetch_factor"] - 2.0) < 1e-12
    assert abs(d["copy_calibration"]["write_factor"] - 1.0) < 1e-12
    assert d["dispatches"] == [2, 1]
    assert abs(d["fetch_bytes_per_launch"] - 2000.0 * kib * 2.0) < 1e-6
    assert abs(d["write_bytes_per_launch"] - 500.0 * kib) < 1e-6
    assert d["hbm_bytes_per_launch"] == d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert d["kernel_source_hash"] == "source-hash"
