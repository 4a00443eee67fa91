"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, validates descriptors before touching a device, and its host-side
LGL operators (Sec. 2 LGL-DGSEM example; Sec. 2.1 D~) satisfy polynomial
exactness, the SBP property and skew-symmetry.  No compute call is made."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def E():
    from paper_2112_10517_amd import esdg, build
    if not os.path.exists(esdg.LIB_PATH):
        build.build()
    esdg.load_library()
    return esdg


def header_symbols():
    text = open(os.path.join(ROOT, "include", "esdg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esdg_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(E):
    syms = header_symbols()
    assert len(syms) >= 18
    lib = E.load_library()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(E.EXPORTS)
    assert "gfx950" in E.version()


@pytest.mark.parametrize("p", range(1, 8))
def test_host_operators(E, p):
    x, w, D, Dt = E.operators(p)
    N = p + 1
    for k in range(N):
        ref = k * x ** (k - 1) if k else np.zeros(N)
        assert np.abs(D @ x ** k - ref).max() < 1e-13 * (1 + k) * N
    B = np.zeros((N, N))
    B[0, 0], B[-1, -1] = -1, 1
    assert np.abs(np.diag(w) @ D + D.T @ np.diag(w) - B).max() < 1e-14 * N
    MDt = np.diag(w) @ Dt
    assert np.abs(MDt + MDt.T).max() < 2e-14 * N
    assert np.all(np.diag(Dt) == 0.0)
    assert np.allclose(Dt - np.diag(np.diag(Dt)), 2 * D - np.diag(np.diag(2 * D)), atol=0, rtol=0)
    # the library's operators agree with the oracle's independent construction
    import oracle
    xo, wo, Do = oracle.lgl(p)
    assert np.abs(x - xo).max() < 1e-15 and np.abs(w - wo).max() < 1e-15
    assert np.abs(D - Do).max() < 1e-13 * N * N


def test_operator_range(E):
    with pytest.raises(E.EsdgError):
        E.operators(0)
    with pytest.raises(E.EsdgError):
        E.operators(8)


@pytest.mark.parametrize("kw,msg", [
    (dict(dim=4, p=3, n=(2, 2, 2)), "dim"),
    (dict(dim=3, p=0, n=(2, 2, 2)), "p must"),
    (dict(dim=3, p=8, n=(2, 2, 2)), "p must"),
    (dict(dim=2, p=3, n=(0, 2)), "element counts"),
    (dict(dim=2, p=3, n=(2, 2), gamma=1.0), "gamma"),
    (dict(dim=2, p=3, n=(2, 2), volume_flux="llf"), "volume flux"),
])
def test_descriptor_validation(E, kw, msg):
    with pytest.raises(E.EsdgError) as ei:
        E.Problem(**kw)
    assert ei.value.status == E.EINVAL and msg in str(ei.value)


def test_null_handle_calls(E):
    import ctypes as C
    lib = E.load_library()
    assert lib.esdg_sync(None) == E.EINVAL
    assert b"NULL" in lib.esdg_last_error(None)
    lib.esdg_destroy(None)  # NULL-safe


@pytest.mark.parametrize("kw", [
    dict(dim=3, p=3, n=(4, 3, 5)),
    dict(dim=3, p=7, n=(2, 2, 2), warp=0.1),
    dict(dim=2, p=4, n=(6, 5), precision="fp32"),
    dict(dim=3, p=5, n=(3, 3, 3), warp=0.1, precision="fp32"),
])
def test_footprint_matches_buffer_sizes(E, kw):
    # host-only: five state-sized arrays, FP64 staging for FP32, metrics and
    # face normals on curved meshes, scalars; no device is touched
    dim, p, n = kw["dim"], kw["p"], kw["n"]
    rs = 4 if kw.get("precision") == "fp32" else 8
    N = p + 1
    nn, nf = N ** dim, N ** (dim - 1)
    Ecount = int(np.prod(n))
    ns = Ecount * (dim + 2) * nn
    expect = 5 * ns * rs + (ns * 8 if rs == 4 else 0)
    if kw.get("warp", 0.0):
        expect += (Ecount * (dim * dim + 1) * nn + dim * Ecount * dim * nf) * rs
    got = E.footprint(**kw)
    assert expect <= got <= expect + 64 * 1024 + 8 * 8 * 2048


def test_footprint_of_gauss_problem(E):
    base = E.footprint(3, 3, (4, 4, 4))
    gauss = E.footprint(3, 3, (4, 4, 4), nodes="gauss")
    assert gauss - base == 64 * 6 * 7 * 16 * 8  # entropy-projected face states
    with pytest.raises(E.EsdgError):
        E.footprint(3, 3, (4, 4, 4), warp=0.1, nodes="gauss")


def test_server_admission_rule(E):
    # arrival order, budget, cap; no device involved
    plan = E.server_plan
    assert plan([10, 20, 30], used=0, budget=35) == 2
    assert plan([10, 20, 5], used=0, budget=35) == 3          # exactly at the budget
    assert plan([40, 5], used=0, budget=35) == 0              # the head blocks: no overtaking
    assert plan([10, 10, 10], used=20, budget=35) == 1        # memory of admitted jobs counts
    assert plan([1, 1, 1, 1], used=0, budget=100, active=3, max_active=4) == 1
    assert plan([1, 1], used=0, budget=100, active=4, max_active=4) == 0
    assert plan([1, 1, 1], used=0, budget=100, active=50, max_active=0) == 3  # 0: no cap
    assert plan([], used=0, budget=10) == 0
    with pytest.raises(E.EsdgError):
        plan([5, -1], used=0, budget=10)
    with pytest.raises(E.EsdgError):
        plan([5], used=-1, budget=10)
    # the served workload's jobs: footprints in arrival order against a budget
    sizes = [E.footprint(3, p, (n, n, n), precision="fp32") for n, p in ((8, 3), (32, 5), (16, 4), (8, 5))]
    budget = sizes[0] + sizes[1] + sizes[2] // 2
    assert plan(sizes, used=0, budget=budget) == 2


def test_load_library_path_selects_the_build(E):
    """A library loaded by path is the one the module's classes use; a
    second, different build in the same process is refused."""
    lib = E.load_library(E.LIB_PATH)
    assert E.load_library() is lib
    assert E.load_library(E.LIB_PATH) is lib
    with pytest.raises(RuntimeError):
        E.load_library(os.path.join(os.path.dirname(E.LIB_PATH), "another", "libesdg.so"))
