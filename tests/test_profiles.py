"""The committed PMC summaries are read by bench.py to report HBM traffic: the
launch-shape keys must be in the form the bench looks up, and every shape must
carry the per-launch byte figures it reads."""
import glob
import json
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pmc_summaries_match_the_bench_lookup():
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.json")))
    assert paths
    for p in paths:
        with open(p) as fh:
            d = json.load(fh)
        assert re.fullmatch(r"[0-9a-f]{16}", d["kernel_source_hash"]), p
        shapes = d["per_launch_shape"]
        assert shapes, p
        for key, e in shapes.items():
            assert re.fullmatch(r"(split|fused|onepass),\d+,\d+", key), (p, key)
            kern, rows, kz = key.split(",")
            got = bench.traffic_from_profiles(d["kernel_source_hash"],
                                              {"kernel": kern, "tile_rows": int(rows), "tile_kz": int(kz)},
                                              os.path.basename(p))
            assert got == e["hbm_bytes_per_launch"] and got > d["algorithmic_bytes_per_step"] * 0.5, (p, key)
