"""Host-side tooling without a GPU: autotuner search space and ranking, rocprofv3 summary
parsing, bench contract on a multi-GPU request."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autotune_candidates_cover_the_space():
    from paper_2005_07547_amd import autotune, psf
    c = list(autotune.candidates())
    assert len(c) == 18
    assert {x["bin_per"] for x in c} == {8, 12, 16}
    assert {x["part_log2"] for x in c} == {10, 11, 12}
    assert {x["flags"] for x in c} == {0, psf.PSF_FLAG_TRANSPOSE_RUNS}
    d = list(autotune.candidates({"insert_mode": [psf.PSF_INSERT_DIRECT], "bin_per": [8]}))
    assert d == [{"insert_mode": psf.PSF_INSERT_DIRECT}]


def test_autotune_keeps_each_candidates_best_round(monkeypatch):
    # candidate A is slow on its first timing (device drift), B steady: two
    # rounds rank A first on its better median, one round would pick B
    from paper_2005_07547_amd import autotune
    seq = {8: [1.2, 1.0], 12: [1.1, 1.1]}

    def fake(table_cfg, params, bufs, warmup, iters):
        return {"ms": seq[params["bin_per"]].pop(0), "dropped": 0}

    monkeypatch.setattr(autotune, "time_config", fake)
    best, res = autotune.tune({}, [], space={"bin_per": [8, 12]})
    assert best == {"bin_per": 8}
    assert [r["ms"] for r in res] == [1.0, 1.1]
    seq.update({8: [1.2], 12: [1.1]})
    best, _ = autotune.tune({}, [], space={"bin_per": [8, 12]}, rounds=1)
    assert best == {"bin_per": 12}


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_by_copy_calibration(tmp_path):
    from paper_2005_07547_amd import profiling
    gib_kib = (1 << 30) / 1024
    _write_counters(tmp_path / "cf", [{"Kernel_Name": "copy", "Counter_Name": "FETCH_SIZE",
                                       "Counter_Value": gib_kib / 2}])
    _write_counters(tmp_path / "cw", [{"Kernel_Name": "copy", "Counter_Name": "WRITE_SIZE",
                                       "Counter_Value": gib_kib}])
    _write_counters(tmp_path / "f", [{"Kernel_Name": "k_bin", "Counter_Name": "FETCH_SIZE", "Counter_Value": 100.0},
                                     {"Kernel_Name": "k_bin", "Counter_Name": "FETCH_SIZE", "Counter_Value": 300.0}])
    _write_counters(tmp_path / "w", [{"Kernel_Name": "k_bin", "Counter_Name": "WRITE_SIZE", "Counter_Value": 50.0}])
    rec = profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"))
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert rec["kernels"]["k_bin"]["bytes"] == (200.0 * 2.0 + 50.0) * 1024
    assert rec["digest"] == profiling.source_digest()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip())["error"]
