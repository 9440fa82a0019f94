"""bench.py's contract on the CPU: more than one GPU is refused with a message,
and the counter-traffic table is consulted only for the profiled sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_counter_traffic_keyed_to_sources():
    table = bench.COUNTER_TRAFFIC["bytes_per_launch"]
    for w, kernels in table.items():
        for k, v in kernels.items():
            expect = v if bench.sources_sha() == bench.COUNTER_TRAFFIC["sources_sha256_16"] else None
            assert bench._measured_traffic(w, k) == expect
    assert bench._measured_traffic("another_workload", "k_adjoint_inplace") is None


def test_cpu_baseline_reports_every_sample():
    """The CPU oracle leg times each workload sample and reports the bench
    workload's figure as its value, with the thread count it used."""
    samples = (("d2q9_channel_64x32", 3), ("d2q9_d2q5_exchanger_512x256", 1))
    r = bench.cpu_baseline("d2q9_d2q5_exchanger_512x256", samples)
    assert r["kind"] == "oracle" and r["unit"] == "MLUPS" and r["cores"] >= 1
    assert [s["workload"] for s in r["samples"]] == [s[0] for s in samples]
    assert r["value"] == r["samples"][1]["mlups"] > 0


def test_kernel_labels_tell_every_profiled_variant_apart():
    """The counter-traffic keys: one label per kernel variant the bench reports."""
    base = dict(flow=19, scalar=0)
    labels = {
        bench.klabel("k_primal_inplace", base, "fp32", "recorded"),
        bench.klabel("k_primal_inplace", base, "fp32", "unrecorded"),
        bench.klabel("k_primal_inplace", dict(base, collision="mrt"), "fp32", "recorded"),
        bench.klabel("k_primal_inplace", base, "fp64", "recorded"),
        bench.klabel("k_primal", base, "fp32", "recorded"),
        bench.klabel("k_primal_batch", base, "fp32", "in place,recorded"),
        bench.klabel("k_primal_batch", base, "fp32", "ping-pong,recorded"),
        bench.klabel("k_primal_inplace", dict(flow=19, scalar=7), "fp32", "recorded"),
    }
    assert len(labels) == 8
    assert bench.klabel("k_adjoint_inplace", base, "fp32") == "k_adjoint_inplace<19,0,float>"
    for wl, kernels in bench.COUNTER_TRAFFIC["bytes_per_launch"].items():
        for k in kernels:
            assert k.split("<")[0] in ("k_primal", "k_primal_inplace", "k_adjoint", "k_adjoint_inplace",
                                       "k_oneshot", "k_oneshot_inplace", "k_primal_batch", "k_adjoint_batch")
