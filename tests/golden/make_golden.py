"""Writes tests/golden/c1_oracle_summary.json from the oracle alone.

Regression fixture: the 1k-Gaussian 128x128 scene rendered by the FP64
oracle.  The paper prints no per-pixel or per-Gaussian values, so this file
pins later oracle edits to the reviewed version, nothing more.  Run:
    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import scenes  # noqa: E402


def summary():
    sc = scenes.make_scene("C1")
    cam = scenes.default_camera(128, 128)
    r = oracle.render(sc, cam)
    return {
        "workload": "1k Gaussians uniform in [-1,1]^3, SH0, 128x128, seed 1",
        "num_pairs": int(len(r["keys"])),
        "visible": int(r["proj"]["visible"]),
        "keys_sha256": hashlib.sha256(r["keys"].tobytes()).hexdigest(),
        "values_sha256": hashlib.sha256(r["values"].tobytes()).hexdigest(),
        "image_sum": float(r["image"].sum()),
        "image_max": float(r["image"].max()),
        "final_T_sum": float(r["final_T"].sum()),
        "n_contrib_sum": int(r["n_contrib"].sum()),
        "pixel_64_64": [float(x) for x in r["image"][:, 64, 64]],
    }


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle_summary.json")
    with open(out, "w") as f:
        json.dump(summary(), f, indent=1)
    print("wrote", out)
