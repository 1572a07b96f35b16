"""Host logic of the measurement: the rocprofv3 summary (calibration of the
HBM counters by a plain copy of known size, per-step kernel groups) on
synthetic rocpd-shaped databases, and the rule that the benchmark reports a
counter record only while the kernel sources still hash to it."""
import json
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1804_07588_amd import profsummary  # noqa: E402


def _db(path, kernels=(), pmc=()):
    os.makedirs(path, exist_ok=True)
    con = sqlite3.connect(os.path.join(path, "run_results.db"))
    con.execute("create table kernels (name text, start integer, end integer)")
    con.execute("create table pmc_events (name text, counter_name text, counter_value real)")
    con.executemany("insert into kernels values (?, ?, ?)", kernels)
    con.executemany("insert into pmc_events values (?, ?, ?)", pmc)
    con.commit()
    con.close()


def test_summary_calibrates_counters_and_groups_launches(tmp_path):
    mib = 64
    true = mib * 2**20
    d = str(tmp_path)
    # kernel trace: two launches of each list variant of k_moments (ns)
    _db(os.path.join(d, "kt"), kernels=[
        ("void fdlbm::k_moments<true, float, float, 3, 5>(...)", 0, 300_000),
        ("void fdlbm::k_moments<true, float, float, 3, 5>(...)", 1_000_000, 1_320_000),
        ("void fdlbm::k_moments<false, float, float, 3, 5>(...)", 400_000, 440_000),
        ("void fdlbm::k_moments<false, float, float, 3, 5>(...)", 1_400_000, 1_440_000),
    ])
    # counters in KiB per dispatch: the copy reads `true` bytes but FETCH_SIZE
    # reports half of them, WRITE_SIZE all of them
    _db(os.path.join(d, "fetch"), pmc=[
        ("k_copy_words(...)", "FETCH_SIZE", true / 2 / 1024),
        ("void fdlbm::k_moments<true, float, float, 3, 5>(...)", "FETCH_SIZE", 1000.0),
        ("void fdlbm::k_moments<false, float, float, 3, 5>(...)", "FETCH_SIZE", 100.0),
    ])
    _db(os.path.join(d, "write"), pmc=[
        ("k_copy_words(...)", "WRITE_SIZE", true / 1024),
        ("void fdlbm::k_moments<true, float, float, 3, 5>(...)", "WRITE_SIZE", 500.0),
        ("void fdlbm::k_moments<false, float, float, 3, 5>(...)", "WRITE_SIZE", 50.0),
    ])
    out_txt, out_json = os.path.join(d, "s.txt"), os.path.join(d, "t.json")
    profsummary.main(["x", d, out_txt, out_json, str(mib), "kt cmd", "pmc cmd"])
    rec = json.load(open(out_json))
    assert rec["factors"] == {"fetch": pytest.approx(2.0), "write": pytest.approx(1.0)}
    g = rec["kernels"]["k_moments"]
    assert g["fetch_bytes"] == pytest.approx((1000.0 + 100.0) * 1024 * 2.0)
    assert g["write_bytes"] == pytest.approx((500.0 + 50.0) * 1024 * 1.0)
    assert g["avg_us"] == pytest.approx(310.0 + 40.0)   # mean durations of both lists, summed
    assert rec["source_sha256"] == profsummary.source_hash()
    assert "k_moments" in open(out_txt).read()


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    import bench
    rec = {"source_sha256": profsummary.source_hash(),
           "kernels": {"k_moments": {"fetch_bytes": 3.0, "write_bytes": 4.0, "avg_us": 1.0}}}
    path = os.path.join(str(tmp_path), "t.json")
    with open(path, "w") as fh:
        json.dump(rec, fh)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", path)
    assert bench.measured_traffic("k_moments") == 7.0
    assert bench.measured_traffic("k_collide") is None
    rec["source_sha256"] = "0" * 64
    with open(path, "w") as fh:
        json.dump(rec, fh)
    assert bench.measured_traffic("k_moments") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", os.path.join(str(tmp_path), "missing.json"))
    assert bench.measured_traffic("k_moments") is None


def test_source_hash_ignores_the_network_sources(tmp_path, monkeypatch):
    """The record covers the lattice-Boltzmann kernels and their C ABI; the
    U-Net's sources and the calibration copy do not enter the hash."""
    csrc = tmp_path / "csrc"
    csrc.mkdir()
    (csrc / "fdlbm_kernels_impl.h").write_text("a")
    (csrc / "unet_kernels.hip").write_text("b")
    monkeypatch.setattr(profsummary, "HERE", str(tmp_path))
    h1 = profsummary.source_hash()
    (csrc / "unet_kernels.hip").write_text("c")
    (csrc / "calib_copy.hip").write_text("d")
    assert profsummary.source_hash() == h1
    (csrc / "fdlbm_kernels_impl.h").write_text("e")
    assert profsummary.source_hash() != h1


def test_bench_refuses_several_gpus():
    """The solver runs on one GPU: more than one exits with a message."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_kernel_algorithmic_bytes_add_up_to_the_step():
    """Each algorithmic byte of a step belongs to exactly one kernel group:
    the collision is credited with its post-collision writes only (its read
    of the streamed copy is overhead of the two-pass step)."""
    import bench
    n_gas, n_links, n_solid, ns, Q = 1362836, 1565578, 734316, 5, 19
    for b in (8, 4, 2):
        total, per = bench.alg_bytes(n_gas, n_links, n_solid, ns, Q, b)
        assert total == n_gas * 2 * Q * ns * b + n_links * 2 * ns * b + n_solid * 2 * b
        assert sum(per.values()) == total
        assert per["k_collide"] == n_gas * Q * ns * b
        assert per["k_moments"] == n_gas * Q * ns * b


def test_run_log_writes_one_json_object_per_line(tmp_path):
    """fdlbm.RunLog: an open line with the metadata, one line per record with
    the step, elapsed seconds, every observable (arrays as lists, non-finite
    values kept) and the caller's extras, and a close line."""
    import json
    import numpy as np
    from paper_1804_07588_amd import fdlbm

    class Fake:
        def __init__(self):
            self.k = 0

        def observe(self):
            self.k += 100
            return {"step": np.int64(self.k), "mass": np.array([1.5, 2.5]), "e_gas": np.float64(3.0),
                    "u_max": float("inf"), "bad": 0}

    path = tmp_path / "run.jsonl"
    log = fdlbm.RunLog(str(path), dict(run="test", n=8))
    sim = Fake()
    log.record(sim, residual={"max": 1e-3}, label="a")
    log.record(sim, residual={"max": 5e-4}, label="a")
    log.close()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [x["event"] for x in lines] == ["open", "step", "step", "close"]
    assert lines[0]["run"] == "test" and lines[0]["n"] == 8
    assert lines[1]["step"] == 100 and lines[2]["step"] == 200
    assert lines[2]["mass"] == [1.5, 2.5] and lines[2]["residual"]["max"] == 5e-4
    assert lines[1]["u_max"] == float("inf") and lines[2]["t"] >= lines[1]["t"] >= 0


def test_steady_state_check_reports_a_failure_in_its_record(monkeypatch):
    """The benchmark line's time-to-steady-state record: the reduced
    configuration (24 beds of 64^3, 20 for training, 150 epochs, 1e-6), and
    a failure of that part ends up in the record instead of losing the
    throughput line."""
    import argparse
    import bench
    seen = {}

    def fake(sub, quiet=False):
        seen.update(n=sub.sur_n, train=sub.sur_train, test=sub.sur_test, epochs=sub.sur_epochs, tol=sub.tol)
        raise RuntimeError("no device")

    monkeypatch.setattr(bench, "surrogate_pipeline", fake)
    rec = bench.steady_state_check(argparse.Namespace(steps=1000))
    assert seen == dict(n=64, train=20, test=4, epochs=150, tol=1e-6)
    assert rec == {"error": "RuntimeError: no device"}
