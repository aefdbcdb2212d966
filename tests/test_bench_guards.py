"""The counter-derived figures of the bench line (search traffic and issue
fraction, force-pass L1 rate and traffic) are constants taken from the
rocprofv3 runs summarised under profiles/, each keyed to a hash of the
kernel sources it was taken on; the bench reports null once the sources
change (the counters no longer describe the kernel).  These checks keep the
committed constants and the profile summaries in agreement, and check that
the guard does turn a figure into null for other sources."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _read(name):
    with open(os.path.join(PROFILES, name)) as f:
        return f.read()


def test_counter_figures_are_null_unless_taken_on_the_current_sources():
    live = bench._digest("search.hip", "internal.h") == bench.NLIST_TRAFFIC_SOURCE_SHA256
    assert (bench.nlist_traffic() == bench.NLIST_TRAFFIC_BYTES) == live
    assert (bench.nlist_traffic() is None) == (not live)
    assert (bench.nlist_valu_rate() is None) == (not live)
    live_f = bench._digest("sph.hip", "pairs.h", "internal.h") == bench.FORCE_SOURCES_SHA256
    assert (bench.force_l1_rate() is None) == (not live_f)


def test_profile_summaries_name_the_guarded_sources():
    for name in ("neighbour_kernels_periodic_3d_8388608_traffic.md", "neighbour_kernels_periodic_3d_8388608_issue.md"):
        text = _read(name)
        assert f"`{bench.NLIST_TRAFFIC_SOURCE_SHA256}`" in text, name
    assert f"`{bench.FORCE_SOURCES_SHA256}`" in _read("neighbour_kernels_periodic_3d_8388608_issue.md")


def test_search_traffic_constant_is_the_summarised_one():
    text = _read("neighbour_kernels_periodic_3d_8388608_traffic.md")
    m = re.search(r"traffic per launch: ([0-9.]+) GB read \+ ([0-9.]+) GB written = ([0-9.]+) GB", text)
    assert m, "traffic line missing"
    read, written, total = (float(x) for x in m.groups())
    assert abs(read + written - total) < 2e-3
    assert abs(total * 1e9 - bench.NLIST_TRAFFIC_BYTES) < 1e6


def test_lane_slots_per_candidate_is_the_summarised_figure():
    text = _read("neighbour_kernels_periodic_3d_8388608_issue.md")
    m = re.search(r"([0-9.]+) lane-slots per candidate", text)
    assert m, "lane-slot line missing"
    assert f"{bench.NLIST_VALU_INSTS:.3e}" in text
    live = bench._digest("search.hip", "internal.h") == bench.NLIST_TRAFFIC_SOURCE_SHA256
    got = bench.nlist_lane_slots_per_candidate(3.135e9)
    assert (got is None) == (not live)
    if live:
        assert abs(got - float(m.group(1))) < 0.1
