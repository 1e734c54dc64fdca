"""CPU checks of the committed measurement records: bench.py reports HBM traffic
only from counters of the current kernel source and the same launch shape, every
table entry names a profile summary that exists, and the algorithmic work counts."""
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _table():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        return json.load(f)


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench


def test_traffic_is_reported_only_for_the_profiled_kernel_source():
    with open(os.path.join(ROOT, "paper_1506_05094_amd", "csrc", "kernels.hip"), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    bench = _bench()

    def key(e):
        return (e["workload"], e["n"], e["mode"], e["tp"], e["ppb"], e["skin"], e["list_mode"])

    current = {}
    for e in _table()["entries"]:
        if e["kernels_hip_sha256"] == digest:
            current.setdefault(key(e), 1024.0 * (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"])
                               / e["steps_per_launch"])
    for e in _table()["entries"]:
        # counters of another kernel source are never reported: the lookup gives the
        # current source's entry for the same key, or nothing
        assert bench.hbm_traffic_per_step(*key(e)) == current.get(key(e))


def test_every_entry_names_an_existing_summary():
    for e in _table()["entries"]:
        assert os.path.exists(os.path.join(ROOT, e["profile"])), e["profile"]
        for k in ("workload", "n", "mode", "tp", "ppb", "skin", "fetch_kib", "write_kib", "fetch_scale",
                  "write_scale", "kernels_hip_sha256", "steps_per_launch", "list_mode"):
            assert k in e, (e["profile"], k)
        assert e["fetch_kib"] > 0 and e["write_kib"] > 0


def test_bench_lookup_needs_the_same_shape():
    bench = _bench()
    for e in _table()["entries"]:
        key = (e["workload"], e["n"], e["mode"], e["tp"], e["ppb"], e["skin"], e["list_mode"])
        assert bench.hbm_traffic_per_step(*key[:3], e["tp"] * 128, *key[4:]) is None
        assert bench.hbm_traffic_per_step(*key[:5], e["skin"] + 0.1, key[6]) is None
        assert bench.hbm_traffic_per_step(*key[:6], key[6] + 1) is None


def test_bench_work_counts():
    bench = _bench()
    # force 4 per entry + 40, integrator 96; the whole path adds (170 + 4 L) / k
    assert bench.path_bytes_per_particle_step(100.0, 20.0, False) == 536.0
    assert bench.path_bytes_per_particle_step(100.0, 20.0, True) == 536.0 + 570.0 / 20.0
    assert bench.flops_per_particle_step(100.0, 60.0, "sf") == 2000.0 + 27 * 60.0
    assert bench.flops_per_particle_step(100.0, 60.0, "sp") == 2000.0 + 21 * 60.0
