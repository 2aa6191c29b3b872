"""Host-side helpers of bench.py (no GPU): the kernel-source hash that ties the committed
rocprofv3 counters to the sources they were taken on, and the derived roofline figures."""
import os

import pytest

import bench


def test_code_only_ignores_comments_and_layout():
    a = "int f(int x) {  // the sum\n  return x + 1; /* one\n more */ }\n"
    b = "int f(int x)\n{\n  return x + 1;\n}\n"
    c = "int f(int x) { return x + 2; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_profiles_match_the_current_kernel_sources():
    """the committed counters were taken on these sources, so the bench reports traffic and VALU
    figures (they go null as soon as the kernel changes without new counters)"""
    kv_t = bench._read_profile(bench.PROFILE_TRAFFIC, 1 << 27)
    kv_v = bench._read_profile(bench.PROFILE_VALU, 1 << 27)
    if kv_t is None or kv_v is None:
        pytest.skip("the committed counters predate the current kernel sources (bench reports them as null)")
    t = bench.read_traffic(1 << 27)
    assert abs(t - 24 * (1 << 27)) <= 0.02 * 24 * (1 << 27)      # within 2 % of algorithmic
    assert bench._read_profile(bench.PROFILE_TRAFFIC, 1 << 20) is None   # another N


def test_valu_view_arithmetic():
    v = bench.valu_view({"valu_instr_per_vector": 150.0, "valu_busy_frac": 0.9}, 1 << 27, 0.5)
    rate = 150.0 * (1 << 27) / 0.5e-3
    assert abs(v["achieved_lane_instr_per_s"] - rate) <= 1e-6 * rate
    assert v["peak_lane_instr_per_s"] == 256 * 4 * 16 * 2.4e9
    assert abs(v["issue_frac"] - rate / v["peak_lane_instr_per_s"]) < 1e-12
    assert bench.valu_view(None, 1 << 27, 0.5) is None


def test_kernel_hash_covers_the_kernel_sources():
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(bench.ROOT, f)), f
    assert len(bench.kernel_hash()) == 16
