"""CPU checks of the committed measurement records: the HBM-traffic table that
bench.py reports from belongs to the current kernel source, every entry names a
profile summary that exists, and bench.py's lookup finds the default workload."""
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _table():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        return json.load(f)


def test_traffic_table_matches_kernel_source():
    with open(os.path.join(ROOT, "paper_1506_05094_amd", "csrc", "kernels.hip"), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    assert _table()["kernels_hip_sha256"] == digest, "kernels.hip changed since the counter passes: re-profile"


def test_every_entry_names_an_existing_summary():
    for e in _table()["entries"]:
        assert os.path.exists(os.path.join(ROOT, e["profile"])), e["profile"]
        for k in ("workload", "n", "mode", "tp", "ppb", "skin", "fetch_kib", "write_kib", "fetch_scale",
                  "write_scale"):
            assert k in e, (e["profile"], k)
        assert e["fetch_kib"] > 0 and e["write_kib"] > 0


def test_bench_lookup_finds_the_default_workload():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = bench.hbm_traffic("Kob-Andersen 80:20 NVT", 4096, "persistent", 16, 16, 0.5)
    assert t is not None and 5e8 < t < 7e8
    assert bench.hbm_traffic("Kob-Andersen 80:20 NVT", 4096, "persistent", 16, 16, 0.3) is None
