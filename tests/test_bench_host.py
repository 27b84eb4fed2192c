"""Host logic of bench.py (CPU): the recorded-traffic lookup keys each
kernel's counter record to the sources that define that kernel, and the
multi-GPU request is refused with a message."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree(tmp_path, sources, traffic):
    csrc = tmp_path / "paper_2111_07347_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name, text in sources.items():
        (csrc / name).write_text(text)
    rec = {"workload_config": 2,
           "sources": {n: hashlib.sha256(t.encode()).hexdigest() for n, t in sources.items()},
           "traffic_bytes_per_launch": traffic}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_config2.json").write_text(json.dumps(rec))
    return csrc


def test_recorded_traffic_is_keyed_per_kernel(tmp_path, monkeypatch):
    srcs = {"tm_match.hip": "match", "tm_library.hip": "library", "tm_topn.h": "topn",
            "tm_polar.hip": "polar", "tm_simulate.hip": "simulate"}
    traffic = {"match_kernel<6, 3, 1, false, 8>": {"fetch_bytes": 10.0, "write_bytes": 2.0},
               "polar_kernel<float, true>": {"fetch_bytes": 100.0, "write_bytes": 20.0},
               "template_kernel": {"fetch_bytes": 5.0, "write_bytes": 5.0}}
    csrc = _tree(tmp_path, srcs, traffic)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic(2, "match_kernel") == 12.0
    assert bench.recorded_traffic(2, "polar_kernel") == 120.0
    assert bench.recorded_traffic(3, "match_kernel") is None          # no record for config 3
    # a change to a source of another kernel leaves the record valid ...
    (csrc / "tm_simulate.hip").write_text("simulate, changed")
    assert bench.recorded_traffic(2, "match_kernel") == 12.0
    assert bench.recorded_traffic(2, "polar_kernel") == 120.0
    # ... but not for kernels without a source list, which check every source
    assert bench.recorded_traffic(2, "template_kernel") is None
    # a change to one of the kernel's own sources makes it stale
    (csrc / "tm_library.hip").write_text("library, changed")
    assert bench.recorded_traffic(2, "match_kernel") is None
    assert bench.recorded_traffic(2, "polar_kernel") == 120.0
    (csrc / "tm_polar.hip").unlink()
    assert bench.recorded_traffic(2, "polar_kernel") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "one gpu" in r.stderr.lower()
