"""The bench's host-side contract, without a GPU: more than one GPU is
refused with a message, and the network share of a corrected stage is
computed from the kernel times as the bench line states."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and "--gpus" in line["error"]


def test_network_share_of_a_stage():
    import bench
    plain = {"traces": 0.009, "grad": 0.019, "net": 0.0, "resid": 0.023}
    # separate launches: the network's own time over the three launches
    sep = {"traces": 0.009, "grad": 0.019, "net": 0.035, "resid": 0.023}
    assert abs(bench.network_share(sep, plain) - 0.035 / 0.077) < 1e-12
    # one fused BR1-and-network launch reported as "net": minus plain P = 3's BR1 pass
    fused = {"traces": 0.009, "grad": 0.0, "net": 0.045, "resid": 0.023}
    assert abs(bench.network_share(fused, plain) - (0.045 - 0.019) / 0.068) < 1e-12
