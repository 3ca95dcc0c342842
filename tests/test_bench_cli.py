"""Host-side checks of bench.py's command line: more than one GPU is refused
with a message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _fake_db(path, counter, rows):
    """A results database with the pmc_events view columns bench.py reads."""
    import sqlite3

    con = sqlite3.connect(path)
    con.execute("create table pmc_events (dispatch_id integer, name text, counter_name text, "
                "counter_value real)")
    con.executemany("insert into pmc_events values (?, ?, ?, ?)",
                    [(i + 1, n, counter, v) for i, (n, v) in enumerate(rows)])
    con.commit()
    con.close()


def test_traffic_table_from_counter_passes(tmp_path, monkeypatch):
    """The per-tuning table maps the k-th pair of aggregation dispatches to the
    k-th tuning, keeps the last frame's counters, scales each counter by the
    1 GiB copies, and the lookup refuses unknown tunings and changed sources."""
    sys.path.insert(0, ROOT)
    import bench

    cand = bench.tuning_candidates()
    assert len(cand) == 72 and len(set(cand)) == 72 and cand[0] == (4, 4, 0, 0, 0)
    agg = "void sf::sgm_tasks_kernel<8, 4, false>(sf::AggView const*)"
    for counter, copy_kib, scale in (("FETCH_SIZE", 524288.0, 1.0), ("WRITE_SIZE", 1048576.0, 2.0)):
        rows = [("__amd_rocclr_copyBuffer", copy_kib)] * 3 + [("__amd_rocclr_copyBuffer", 10.0)]
        for i in range(len(cand)):
            for f in range(bench.SWEEP_FRAMES):
                rows.append(("sf::census_kernel(sf::CensusArgs)", 1.0))
                # the last frame of tuning i reads/writes (i + 1) MiB-ish; earlier frames differ
                last = f == bench.SWEEP_FRAMES - 1
                rows.append((agg, (i + 1) * 1024.0 * scale if last else 999.0))
        _fake_db(str(tmp_path / f"{counter}.db"), counter, rows)
    out = str(tmp_path / "traffic.json")
    bench.write_traffic_table(str(tmp_path / "FETCH_SIZE.db"), str(tmp_path / "WRITE_SIZE.db"), out)
    import json

    with open(out) as f:
        rec = json.load(f)
    assert rec["copy_calibration"]["fetch_factor"] == 2.0
    assert rec["copy_calibration"]["write_factor"] == 1.0
    for i, c in enumerate(cand):
        e = rec["by_tuning"][",".join(map(str, c))]
        # FETCH (i+1) MiB x 2 + WRITE 2 (i+1) MiB x 1 = 4 (i+1) MiB
        assert e["traffic_bytes_per_launch"] == 4 * (i + 1) * (1 << 20)
    monkeypatch.setattr(bench, "TRAFFIC_JSON", out)
    assert bench.measured_traffic("sgm_tasks", (8, 8, 1, 4, 1)) == \
        rec["by_tuning"]["8,8,1,4,1"]["traffic_bytes_per_launch"]
    assert bench.measured_traffic("sgm_tasks", (8, 8, 1, 3, 0)) is None
    assert bench.measured_traffic("sgm_paths", (8, 8, 1, 4, 0)) is None
    rec["sources_sha256"] = "0" * 64
    with open(out, "w") as f:
        json.dump(rec, f)
    assert bench.measured_traffic("sgm_tasks", (8, 8, 1, 4, 1)) is None
