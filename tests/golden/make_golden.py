"""Writes the stored expected values under tests/golden/ by calling only the oracle.

The paper prints no worked numeric example for this path (its only numbers are
timings), so the fixtures here are oracle outputs on small seeded scenes; they
guard the oracle against accidental change. Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402


def tiny_fixture():
    w = synth.make_tiny()
    cam = w.view.camera
    mask, _ = O.select(w.scene, cam, w.view.select)
    pr = O.project(w.scene, cam, (16, 16), mask=mask, M=w.view.recolor.M, b=w.view.recolor.b)
    img = O.render_image(pr, brute=True)
    ts, zs, ids = O.sorted_keys(pr)
    px = [(5, 7), (64, 64), (100, 30), (127, 127), (40, 90), (70, 60)]
    return {
        "source": "oracle on the seeded tiny scene (4,096 Gaussians, 128x128, 16x16 tiles), "
                  "selection + fused 120 degree hue rotation; eq. (1)-(3), (6)",
        "n_selected": int(mask.sum()),
        "tile_counts_sum": int(pr.col("count").sum()),
        "first_64_sorted_indices": [int(v) for v in ids[:64]],
        "first_64_sorted_tiles": [int(v) for v in ts[:64]],
        "pixels": [{"x": x, "y": y, "rgb": [float(v) for v in img.rgb[y, x]], "T": float(img.T[y, x]),
                    "last": int(img.last[y, x])} for (x, y) in px],
        "image_sum": [float(v) for v in img.rgb.reshape(-1, 3).sum(0)],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(tiny_fixture(), f, indent=1)
