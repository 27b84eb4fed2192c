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


def test_parity_rule_on_sample_counts_clear_ranks():
    """The benchmark's parity rule: ranks whose oracle gap to both
    neighbours exceeds 1e-4 must match in template (and angle where the
    angle margin exceeds 1e-4); near-ties are not compared."""
    import numpy as np
    import torch
    N = 3
    ot = np.array([[5, 7, 9, 11], [1, 2, 3, 4]])
    os_ = np.array([[10, 20, 30, 40], [1, 2, 3, 4]])
    oq = np.array([[0.9, 0.8, 0.79995, 0.5], [0.7, 0.6, 0.5, 0.4]])
    am = np.array([[0.1, 0.1, 0.1], [0.1, 0.00001, 0.1]])
    # pattern 0: ranks 1 and 2 are a near-tie (swapped on the GPU: fine);
    # pattern 1: rank 1's angle is a near-tie (different angle: fine)
    gt = torch.tensor([[5, 9, 7], [1, 2, 3]], dtype=torch.int32)
    gs = torch.tensor([[10, 30, 20], [1, 99, 3]], dtype=torch.int32)
    gq = torch.tensor([[0.9, 0.8, 0.79995], [0.7, 0.6, 0.5]], dtype=torch.float32)
    r = bench.parity_on_sample((gt, gs, gq), [0, 1], (ot, os_, oq, am), N)
    assert r["ranks_with_template_margin_above_1e-4"] == 4
    assert r["template_identical_there"] == 1.0
    assert r["ranks_with_angle_margin_above_1e-4"] == 3
    assert r["passed"]
    # a wrong template on a clear rank fails
    gt2 = gt.clone()
    gt2[1, 2] = 8
    r = bench.parity_on_sample((gt2, gs, gq), [0, 1], (ot, os_, oq, am), N)
    assert not r["passed"] and r["template_identical_there"] == 0.75
    # a score outside the tolerance fails
    gq2 = gq.clone()
    gq2[0, 0] = 0.9 + 1e-4
    assert not bench.parity_on_sample((gt, gs, gq2), [0, 1], (ot, os_, oq, am), N)["passed"]


def test_workload_label_uses_the_actual_batch():
    import synth
    lab = bench.workload_label(synth.WORKLOADS[3], 4096)
    assert "4096 f32 patterns 256x256" in lab and "20000 orthorhombic templates" in lab
