"""Pins for the oracle's Philox4x32-10 generator and its normal draws."""
import json
import os

import numpy as np

from oracle import philox


def test_known_answer_vectors():
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = np.array([int(x, 16) for x in v["counter"]], np.uint32).reshape(4, 1)
        k = [int(x, 16) for x in v["key"]]
        out = philox.philox4x32_10(ctr, k[0], k[1])[:, 0]
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_normal_field_moments():
    z = philox.normal_field(12345, 64).astype(np.float64).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(z ** 4) - 3) < 5 * np.sqrt(96 / n)
    assert not np.array_equal(z, philox.normal_field(12346, 64).ravel())
