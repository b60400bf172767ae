"""The committed rocprofv3 summaries behind the bench line (CPU only): every
pair-evaluation summary exists and gives the command that made it, and the HBM-traffic
figure of the 20 x 10 000 search without time windows belongs to the current evaluation
sources (the bench reports traffic only then; a change to those sources needs new
counters)."""
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pair_profiles_exist_and_give_their_command():
    for name in bench.PAIR_PROFILES.values():
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "rocprofv3" in text, name
        assert "traffic_bytes_per_launch:" in text and "kernel-source-sha256:" in text, name


def test_traffic_of_the_20x10000_search_matches_the_current_sources():
    t = bench.measured_traffic("config3")
    assert t is not None, "evaluation sources changed since the counters were taken"
    assert t > 0
