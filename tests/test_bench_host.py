"""Host-side checks of bench.py's bookkeeping (no GPU): the algorithmic work
counts, the blended roofline and the hash gate on the HBM-traffic
summaries."""
import hashlib
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_c2_launch_flop_matches_the_hand_count():
    # 4096 x [50 (2 28^2 + 6 28 + 6 14) + 2 10 28 14], counted by hand from
    # the knot-precompute form of the step
    assert 4096 * bench.linear_flop_per_candidate(28, 14, 50, 10) == 404_848_640


def test_flop_counts_scale_with_the_horizon():
    a = bench.linear_flop_per_candidate(72, 36, 20, 5)
    b = bench.linear_flop_per_candidate(72, 36, 40, 5)
    assert b - a == 20 * (2 * 72 * 72 + 6 * 72 + 6 * 36)  # the knot term does not grow
    assert bench.chain_flop_per_candidate(36, 100) == 2 * bench.chain_flop_per_candidate(36, 50)
    n, m = 14, 7
    assert (bench.full_weight_flop_per_candidate(n, m, 2) - bench.full_weight_flop_per_candidate(n, m, 1)
            == 4 * n * n + 2 * n * m + 2 * m * m + 4 * n + 6 * m)


def test_c5_flop_splits_linear_and_chain():
    probs, ga = W.config_c5(16, 0)
    lin, ch = bench.c5_flop(probs, ga)
    want_lin = sum(ga.pop * bench.linear_flop_per_candidate(p.n, p.m, p.T, p.p)
                   for p in probs if p.model == W.LINEAR)
    want_ch = sum(ga.pop * 25 * p.m * p.T for p in probs if p.model != W.LINEAR)
    assert (lin, ch) == (want_lin, want_ch)
    assert lin > 0 and ch > 0


def test_blended_roofline_reduces_to_each_peak():
    r = bench.blended_roofline(1e12, 0.0, 1.0)
    assert r["peak"] == pytest.approx(bench.PEAK_FP32_MFMA / 1e12)
    r = bench.blended_roofline(0.0, 1e12, 1.0)
    assert r["peak"] == pytest.approx(bench.PEAK_FP32_VALU / 1e12)
    # frac = time both shares take at their peaks / measured time
    lin, ch, secs = 3e12, 1e12, 0.25
    r = bench.blended_roofline(lin, ch, secs)
    t_peak = lin / bench.PEAK_FP32_MFMA + ch / bench.PEAK_FP32_VALU
    assert r["frac"] == pytest.approx(t_peak / secs)
    assert r["achieved"] == pytest.approx((lin + ch) / secs / 1e12)


def test_traffic_bytes_are_reported_only_for_the_profiled_sources(tmp_path):
    src = tmp_path / "kernel.hpp"
    src.write_text("// kernel source\n")
    good = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "summary.md"
    summary.write_text("text\n\nbytes_per_launch: 1234\nsrc_sha256: %s\n" % good)
    assert bench._counted_bytes(str(summary), [str(src)], "src_sha256", "bytes_per_launch") == 1234.0
    src.write_text("// kernel source, changed\n")
    assert bench._counted_bytes(str(summary), [str(src)], "src_sha256", "bytes_per_launch") is None
    assert bench._counted_bytes(str(tmp_path / "absent.md"), [str(src)], "src_sha256",
                                "bytes_per_launch") is None
