"""Seeded input generator: determinism, prefix property, FP32 exactness."""
import json
import os

import numpy as np

import synth
from tests.golden.write_synth_manifest import manifest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_manifest_matches_committed_hashes():
    with open(os.path.join(HERE, "golden", "synth_manifest.json")) as f:
        want = json.load(f)
    assert manifest() == want


def test_prefix_property_and_fp32_exact():
    a = synth.workload("arm131k", targets=32)["groups"][0]
    b = synth.workload("arm131k", targets=64)["groups"][0]
    np.testing.assert_array_equal(a["q_star"], b["q_star"][:32])
    np.testing.assert_array_equal(a["seeds"], b["seeds"][:256])
    for arr in [a["q_star"], a["seeds"], synth.tree34(5).offset, synth.hand16(8).upper]:
        assert np.array_equal(arr, arr.astype(np.float32).astype(np.float64))


def test_configs_within_limits_and_shapes():
    for t in [synth.arm7(0), synth.tree34(5), synth.hand16(8)]:
        q = synth.uniform_configs(t, 1000, 1)
        assert q.shape == (1000, t.n)
        assert np.all(q >= t.lower) and np.all(q <= t.upper)
        assert np.all(t.parent < np.arange(t.n))
        assert np.all(t.upper >= np.float32(np.pi / 2)) and np.all(t.upper <= np.float32(np.pi))
    assert synth.tree34(5).n == 34 and synth.tree34(5).m == 4
    assert synth.hand16(8).n == 16 and list(synth.hand16(8).ee_kind) == [1, 1, 1, 1]
