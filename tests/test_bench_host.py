"""Host-side logic of bench.py, on the CPU: the one-GPU contract, the FIFO latency of the
one-at-a-time baseline, the serving stream's preconditioner policy and the counter-traffic
guard."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench as BN  # noqa: E402
from paper_2502_09323_amd import inputs as I  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_fifo_latency_of_a_single_server():
    arr = np.array([0.0, 0.1, 0.15, 5.0])
    svc = [1.0, 0.5, 0.2, 0.3]
    lat = BN.fifo_latency(arr, svc)
    # starts at 0, 1.0, 1.5 and 5.0; ends at 1.0, 1.5, 1.7 and 5.3
    assert np.allclose(lat, [1.0, 1.4, 1.55, 0.3])


def test_serving_stream_policy():
    reqs, arr = BN.stream(64, "auto")
    assert len(reqs) == 64 and np.all(np.diff(arr) >= 0)
    for _, g in reqs:
        big = min(g.n) >= BN.MG_MIN_N
        assert (g.precond == I.MG) == big
        assert g.precision == I.MIXED
        assert g.inner_rtol == (BN.DELTA_MG if big else BN.DELTA)
    assert all(g.precond == I.JACOBI for _, g in BN.stream(16, "jacobi")[0])
    assert all(g.precond == I.MG for _, g in BN.stream(16, "mg")[0])


def test_counter_traffic_needs_the_fingerprint_it_was_taken_on():
    fp = BN.kernel_fingerprint("mg")
    assert len(fp) == 16 and fp != BN.kernel_fingerprint("solve")
    saved = {k: dict(v) for k, v in BN.COUNTER_TRAFFIC.items()}
    try:
        BN.COUNTER_TRAFFIC["x@y"] = {"sources": "mg", "fingerprint": "0" * 16, "ratio": 1.5}
        assert BN.counter_traffic("x@y", 1000) is None
        BN.COUNTER_TRAFFIC["x@y"] = {"sources": "mg", "fingerprint": fp, "ratio": 1.5}
        assert BN.counter_traffic("x@y", 1000) == 1500
        assert BN.counter_traffic("no_such_kernel", 1000) is None
    finally:
        BN.COUNTER_TRAFFIC.clear()
        BN.COUNTER_TRAFFIC.update(saved)
