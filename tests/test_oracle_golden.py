"""The oracle still reproduces its stored fixture (tests/golden/tiny_oracle.json)."""
import json
import os

import numpy as np

from tests.golden.make_golden import tiny_fixture

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tiny_fixture_unchanged(orc):
    with open(os.path.join(HERE, "tiny_oracle.json")) as f:
        ref = json.load(f)
    now = tiny_fixture()
    for k in ("n_selected", "tile_counts_sum", "first_64_sorted_indices", "first_64_sorted_tiles"):
        assert now[k] == ref[k], k
    for a, b in zip(now["pixels"], ref["pixels"]):
        assert a["last"] == b["last"]
        np.testing.assert_allclose(a["rgb"], b["rgb"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(a["T"], b["T"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(now["image_sum"], ref["image_sum"], rtol=1e-12)
