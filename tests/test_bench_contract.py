"""Host-side checks of bench.py (no GPU): it refuses several GPUs with a
message, and the committed HBM-traffic counters belong to the current
kernel sources (otherwise the bench would report no traffic)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_counters_match_kernel_sources():
    for phase in ("m2m", "p2m", "l2p", "m2l", "compress", "decompress"):
        b = bench.traffic_for(phase)
        assert b is not None and b > 0, phase


def test_phase_work_counts():
    info = {"n": 1000, "nleaf": 40, "nfar": 30, "nV": 200, "m2m_pairs": 100, "l2p_pairs": 4000,
            "near_pairs": 50000}
    import numpy as np
    tree = {"level": np.array([0, 1, 2, 2, 3]), "isleaf": np.array([0, 0, 0, 1, 1])}
    w = bench.phase_work(info, 20, tree, 117, True)
    # eq. 3.7 per child transfer: two p x p passes over 3 components
    assert w["m2m"][1] == 4.0 * 20 ** 3 * 3 * 100
    # executed: an x pass per child, two y passes per parent (one parent here)
    assert w["m2m"][4] == 2.0 * 20 ** 3 * 3 * 100 + 4.0 * 20 ** 3 * 3 * 1
    # eqs. 3.9-3.11: an L2L transfer per child and the interpolation at each point
    assert w["l2p"][1] == 4.0 * 20 ** 3 * 3 * 100 + 2.0 * 20 ** 2 * 3 * 1000
    assert w["p2p"][1] == bench.FLOP_PER_PAIR * 50000
    assert w["m2l"][1] == 2.0 * 117 * 117 * 200
    assert all(v[0] in ("hbm", "alu", "mfma") for v in w.values())
