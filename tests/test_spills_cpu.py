"""Register spills of the stage kernels (host logic, no GPU), from the
compiler's resource report that build() writes beside the library.

Two wrong-result incidents in the development of the line-layout tiles came
with spilled scalar operands (D~ held as 128 scalar registers in the FP64
N = 8 tile; a spilling FP32 N = 8 tile).  Every N = 8 tile has read D~ from
LDS since.  This test keeps spills from coming back unnoticed:
  * the node and pair layouts (tile variants 3 and 4) spill nothing;
  * no LGL tile at N = 8 spills scalar registers;
  * any other spilling instantiation is listed in tests/data/spill_allowlist.txt
    with its largest allowed scratch use and spill counts, which must not grow;
  * the one-generation form of a tile (PRIO) spills no more than the tile.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT = os.path.join(ROOT, "paper_2112_10517_amd", "lib", "resource_usage.txt")
ALLOW = os.path.join(ROOT, "tests", "data", "spill_allowlist.txt")
PAT = re.compile(r"stage_kernelILi(\d)ELi(\d)ELi(\d)ELi(\d)E([df])Li(\d+)ELi(\d)ELi(\d)ELb([01])E")


def read_report():
    """({8 template arguments: spills} of the stage kernels, the same of their
    one-generation forms (PRIO = true)); spills = (scratch, VGPR, SGPR)."""
    if not os.path.exists(REPORT):
        from paper_2112_10517_amd import build
        build.build()
    plain, prio = {}, {}
    with open(REPORT) as f:
        for line in f:
            name, *kv = line.split()
            m = PAT.search(name)
            if not m:
                continue
            d = dict(x.split("=", 1) for x in kv)
            sp = (int(d["ScratchSize_[bytes/lane]"]), int(d["VGPRs_Spill"]), int(d["SGPRs_Spill"]))
            (prio if m.group(9) == "1" else plain)[m.groups()[:8]] = sp
    assert len(plain) > 400, "resource report incomplete: %d stage kernels" % len(plain)
    return plain, prio


@pytest.fixture(scope="module")
def kernels():
    return read_report()[0]


def allowlist():
    out = {}
    with open(ALLOW) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            f_ = line.split()
            out[tuple(f_[:8])] = tuple(int(x) for x in f_[8:11])
    return out


def test_node_and_pair_layouts_do_not_spill(kernels):
    for key, sp in kernels.items():
        if key[7] in ("1", "2", "3"):  # LAY_NODES, LAY_PAIRS, LAY_PLANES
            assert sp == (0, 0, 0), (key, sp)


def test_no_scalar_spills_at_degree_seven(kernels):
    for key, sp in kernels.items():
        if key[1] == "8" and key[6] == "0":  # N = 8, LGL nodes
            assert sp[2] == 0, (key, sp)


def test_spills_only_where_allowed(kernels):
    allow = allowlist()
    for key, sp in kernels.items():
        if sp == (0, 0, 0):
            continue
        assert key in allow, "stage kernel %s spills %s and is not in the allowlist" % (key, sp)
        lim = allow[key]
        assert all(a <= b for a, b in zip(sp, lim)), "stage kernel %s spills %s, more than %s" % (key, sp, lim)


def test_priority_forms_match_their_tiles():
    # the one-generation form exists for the default 3D LGL line tiles up to
    # N = 4 only, and spills no more than the plain kernel of its tile
    plain, prio = read_report()
    assert prio, "no one-generation stage kernels in the report"
    for key, sp in prio.items():
        assert key[0] == "3" and int(key[1]) <= 4 and key[6] == "0" and key[7] == "0", key
        assert key in plain, key
        assert all(a <= b for a, b in zip(sp, plain[key])), (key, sp, plain[key])
