"""The benchmark's CPU-baseline leg on a tiny workload (host logic only):
the oracle's step plus the side rows' oracles, each reported with its
unit, sample description and a positive rate."""
import numpy as np

import bench
from synthetic import scenes


def test_cpu_baseline_leg_reports_every_row():
    w = scenes.Workload("tiny", scenes.clustered_gaussians(2000, 1), scenes.sphere_cameras(2, 12, 64, 48), None)
    rng = np.random.default_rng(0)
    n = 300
    P = np.zeros((59, n))
    P[3:6] = rng.normal(-3.0, 0.7, (3, n))
    P[6] = 1.0
    P[10] = rng.normal(size=n)
    side = {"dssim": (rng.random((3, 48, 64)), rng.random((3, 48, 64)), 16),
            "densify": {"P": P, "m": np.zeros((59, n)), "v": np.zeros((59, n)), "accum": rng.random(n),
                        "count": rng.integers(0, 3, n), "noise": rng.normal(size=(2, 3, n)),
                        "hp": (0.5, -3.0, -1.0, float("inf"))}}
    out = bench.cpu_baseline(w, side=side)
    assert out["kind"] == "oracle" and out["unit"] == "views/s" and out["value"] > 0 and out["cores"] >= 1
    assert "2 views" in out["sample"] and out["cpu_model"]
    c1 = out["single_view_256_10k"]
    assert c1["all_cores_ms"] > 0 and c1["one_core_ms"] > 0
    assert out["l1_dssim"]["unit"] == "batches/s" and out["l1_dssim"]["value"] > 0
    assert out["densify"]["unit"] == "Gaussians/s" and out["densify"]["value"] > 0
    assert "1 of 16 views" in out["l1_dssim"]["sample"] and "300 Gaussians" in out["densify"]["sample"]
