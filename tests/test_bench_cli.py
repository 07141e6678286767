"""CPU checks of bench.py's command-line contract: more than one GPU is refused with a
message, and the HBM-traffic summary scales each counter by what it reads for a copy
of known size."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_summary_scales_by_the_copy_probe(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    f, w, cf, cw = (str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv"))
    _counter_csv(f, [("cs::k_region(cs::KCirc)", "FETCH_SIZE", 100.0), ("cs::k_region(cs::KCirc)", "FETCH_SIZE", 300.0),
                     ("other", "FETCH_SIZE", 1e9)])
    _counter_csv(w, [("cs::k_region(cs::KCirc)", "WRITE_SIZE", 50.0)])
    # a 256 MiB copy whose fetch counter reads half of the bytes and write counter all
    _counter_csv(cf, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072.0)])
    _counter_csv(cw, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144.0)])
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "h")
    bench.summarize_pmc(f, w, cf, cw, "k_region", "key", 256)
    d = json.load(open(tmp_path / "profiles" / "hbm_traffic.json"))["key"]
    assert d["fetch_factor"] == 2.0 and d["write_factor"] == 1.0
    assert d["bytes_per_launch"] == int(200 * 1024 * 2 + 50 * 1024)
    assert bench.traffic_from_profiles("h", "key") == d["bytes_per_launch"]
    assert bench.traffic_from_profiles("other-hash", "key") is None
