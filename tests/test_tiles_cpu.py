"""Workgroup shapes of the stage kernel (host logic, no GPU): every tile
variant of every 3D degree and precision fits the hardware -- at most 1024
lanes in whole 64-lane waves, one node per lane in the node layout, the
LDS the kernel declares within a CU's 160 KiB and, for the variants that
are not the fallback default, within the 80 KiB budget that lets two
workgroups share a CU."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CAP = 80 * 1024


@pytest.fixture(scope="module")
def shapes(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("tiles") / "tile_shapes")
    cmd = [HIPCC, "-std=c++17", "-O1", "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "paper_2112_10517_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "tile_shapes.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    rows = []
    for line in out.stdout.splitlines():
        f = line.split()
        rows.append({f[i]: (f[i + 1] if f[i] == "prec" else int(f[i + 1])) for i in range(0, len(f), 2)})
    # variants 0-4 for N = 2..8; four (precision, flux, mesh) combinations each
    assert len(rows) == 7 * 5 * 4
    return rows


def test_lanes_and_waves(shapes):
    for s in shapes:
        assert 64 <= s["threads"] <= 1024 and s["threads"] % 64 == 0, s
        assert s["epb"] >= 1, s
        assert s["npt"] * s["threads"] >= s["epb"] * s["nn"], s  # every node has a lane
        assert 1 <= s["waves"] <= 8, s


def test_node_layout_one_node_per_lane(shapes):
    for s in (s for s in shapes if s["variant"] == 3):
        assert s["npt"] == 1 and s["threads"] >= s["epb"] * s["nn"], s
        assert s["threads"] - s["epb"] * s["nn"] < 64, s  # idle lanes only in the last wave
        # at least 128 lanes unless a single element already has fewer nodes... with 80% of them busy
        if s["threads"] >= 128 and s["nn"] >= 27:
            assert 5 * s["epb"] * s["nn"] >= 4 * s["threads"] or s["epb"] == 1, s


def test_pair_layout_shape(shapes):
    """The pair layout: one lane per node; at N = 8 (and at N = 7 for FP64
    curved tiles) one element per workgroup and one wave per z-plane (N^2 of
    its lanes; the x- and y-lines stay inside a wave); otherwise also enough
    lanes for the lines of one direction, floor(64/N) whole lines per wave.
    Two workgroups fit a CU's LDS."""
    pairs = [s for s in shapes if s["variant"] == 4]
    assert len(pairs) == 7 * 4
    for s in pairs:
        N = round(s["nn"] ** (1.0 / 3.0))
        assert s["npt"] == 1 and s["threads"] >= s["epb"] * s["nn"], s
        lines = s["epb"] * N * N
        assert s["threads"] // 64 * (64 // N) >= lines, s
        assert s["threads"] - s["epb"] * s["nn"] < 128, s  # at most one wave more than the nodes need
        assert 2 * s["lds"] <= 160 * 1024, s
        if N == 8 or (N == 7 and s["prec"] == "fp64" and s["mesh"] == 1):  # one z-plane per wave
            assert s["epb"] == 1 and s["threads"] == 64 * N and s["waves"] == 4, s


def test_lds_within_budget(shapes):
    for s in shapes:
        assert s["lds"] <= 160 * 1024, s
        if s["variant"] in (1, 2) and s["epb"] != s["epb0"]:
            assert s["lds"] <= CAP + 4096, s  # the variant's own LDS estimate is within the budget
        if s["variant"] == 3 and s["epb"] > 1:
            assert s["lds"] <= CAP + 4096, s
