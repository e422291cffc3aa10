"""The committed rocprofv3 traffic summaries belong to the kernels as they stand.

bench.py reports a raster kernel's HBM bytes per launch (its roofline `traffic`) from
profiles/<kernel>_traffic*.txt only while the hash of the kernel's sources recorded there
matches the sources; a kernel edited without new counters would report null.  Each
summary also names the command that produced it.
"""
import os

import pytest

import bench


@pytest.mark.parametrize("kname,batch", [("k_raster_fwd", 32), ("k_raster_fwd", 64), ("k_raster_fwd", 128),
                                         ("k_raster_fwd", 256), ("k_raster_bwd", 64)])
def test_traffic_summary_matches_current_sources(kname, batch):
    got = bench.committed_traffic(kname, 32, batch)
    assert got is not None and got > 0


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(os.path.join(bench.ROOT, "profiles"))
                                        if f.endswith("_traffic.txt") or "_traffic_batch" in f))
def test_traffic_summary_names_its_command(name):
    text = open(os.path.join(bench.ROOT, "profiles", name)).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
