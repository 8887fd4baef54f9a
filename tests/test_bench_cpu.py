"""The benchmark's host-side contract, on the CPU: more than one GPU is
refused with a message before any device work, and the recorded HBM byte
counters belong to the kernel sources they were taken on."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert "one GPU only" in r.stdout + r.stderr
    assert not any(l.startswith("{") for l in r.stdout.splitlines())    # no result line


def test_traffic_record_names_its_sources():
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    assert set(rec) >= {"source_sha256", "note", "kernels"}
    assert len(rec["source_sha256"]) == 64
    for per_key in rec["kernels"].values():
        for v in per_key.values():
            assert v["fetch_bytes"] > 0 and v["write_bytes"] > 0
    # bench reports these bytes only while the sources hash the same
    assert isinstance(bench.kernel_source_hash(), str)


def test_cpu_baseline_record_form():
    """The CPU baseline's record on a small slice: the oracle's float64 values
    on all cores (the value), on one core, and the whole step beside them."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, order2_example
    d = order2_example()
    k = k_samples(3000, d.n_int, seed=(9, 2))
    rec = bench.cpu_baseline(d, k, np.array(DEFAULT_Q), 5.0, 1.0, 0.0, matsubara_freqs(1, 5.0), 0.3)
    assert rec["kind"] == "oracle" and rec["unit"] == "term-evals/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert rec["values_f64_1core"]["processes"] == 1 and rec["values_f64_1core"]["term_evals_per_s"] > 0
    assert rec["step_values_and_gradients"]["term_evals_per_s"] > 0
