"""The committed rocprofv3 summaries belong to the kernels in the tree.

bench.py reports HBM traffic and VALU rates from profiles/ only when a summary
was taken on the current kernel source (its kernel_source_hash); these checks
fail when a kernel source changes without the profiles being taken again, and
check that each summary states the commands that made it.
"""
import os
import re

import bench

PROFILES = os.path.join(bench.ROOT, "profiles")


def read(name):
    with open(os.path.join(PROFILES, name)) as f:
        return f.read()


def test_headline_profiles_match_the_kernel_source():
    h = bench.kernel_source_hash()
    for name in ("pass_kernel_48x48x48x48_trace.md", "pass_kernel_48x48x48x48_counters.md"):
        m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", read(name))
        assert m and m.group(1) == h, name
    traffic = bench.traffic_from_profile()
    algorithmic = bench.BYTES_PER_UPDATE * 48 ** 4 // 2
    assert traffic is not None and algorithmic <= traffic < 2 * algorithmic


def test_su3_profile_matches_the_kernel_source():
    h = bench.su3_source_hash()
    for key in ("hbm_bytes_per_launch", "valu_instructions_per_update", "timed_pass_avg_us"):
        assert bench.profile_value(bench.SU3_PROFILE, key, h) is not None, key
    traffic = bench.profile_value(bench.SU3_PROFILE, "hbm_bytes_per_launch", h)
    algorithmic = bench.SU3_BYTES_PER_UPDATE * 48 ** 4 // 2
    assert algorithmic <= traffic < 2 * algorithmic


def test_every_summary_states_its_commands():
    names = [n for n in os.listdir(PROFILES) if n.endswith((".md", ".txt"))]
    assert names
    for name in names:
        text = read(name)
        assert "rocprofv3" in text and "bench.py" in text, name
        assert len(text) < 16384, name  # summaries, not raw output


def test_fp64_profile_matches_the_kernel_source():
    v = bench.profile_value(bench.F64_PROFILE, "hbm_bytes_per_launch", bench.f64_source_hash(),
                            key_name="f64_source_hash")
    algorithmic = 256 * 48 ** 4 // 2
    assert v is not None and algorithmic <= v < 2 * algorithmic
