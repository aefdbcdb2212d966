"""The counter-derived figures of the bench line (search traffic and issue
fraction, force-pass L1 rate and traffic) are constants taken from the
rocprofv3 runs summarised under profiles/, each keyed to a hash of the
kernel sources it was taken on; the bench reports null once the sources
change.  These checks keep the committed constants, the committed sources
and the profile summaries in agreement, so the committed bench line carries
live figures that the summaries back."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _read(name):
    with open(os.path.join(PROFILES, name)) as f:
        return f.read()


def test_search_counters_match_the_committed_search_source():
    assert bench._digest("search.hip", "internal.h") == bench.NLIST_TRAFFIC_SOURCE_SHA256
    assert bench.nlist_traffic() == bench.NLIST_TRAFFIC_BYTES
    assert bench.nlist_issue_frac() == bench.NLIST_VALU_ISSUE_FRAC


def test_force_counters_match_the_committed_pair_sources():
    assert bench._digest("sph.hip", "pairs.h", "internal.h") == bench.FORCE_SOURCES_SHA256
    assert bench.force_l1_rate() == bench.FORCE_L1_ACCESS_RATE


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
