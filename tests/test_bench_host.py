"""Host logic of bench.py (no GPU): the algorithmic byte model of the stage
kernel, the rocprofv3 counter records keyed on the kernel source, and the
one-GPU guard."""
import hashlib
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("dim,N,curved,rb,expect", [
    (3, 4, True, 8, 318.0),   # p = 3 curved FP64: state 160 + metrics 80 + traces 60 + normals 18
    (3, 4, True, 4, 159.0),   # the same in FP32
    (3, 8, True, 8, 279.0),   # p = 7 curved FP64: 160 + 80 + 30 + 9
    (3, 4, False, 8, 220.0),  # affine drops metrics and normals: 160 + 60
    (2, 4, True, 8, 208.0),   # 2D p = 3 curved: state 16 + metrics 5 + traces 4 + normals 1 values
])
def test_algorithmic_stage_bytes(dim, N, curved, rb, expect):
    assert bench.algorithmic_stage_bytes(dim, N, curved, rb) == pytest.approx(expect)


def _write(path, text):
    with open(path, "w") as f:
        f.write(text)
    return str(path)


def test_records_follow_the_kernel_source(tmp_path):
    src = _write(tmp_path / "kernels.hpp", "// kernel source\n")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = _write(tmp_path / "p.md",
                  "# profile\n\n"
                  "traffic-record: kernels_sha256 %s fetch_kib 100.0 write_kib 50.0 fetch_factor 2.0 "
                  "write_factor 1.0\n"
                  "valu-record: kernels_sha256 %s valu_insts 1000000 fp64_add 100 fp64_mul 200 "
                  "fp64_fma 300 fp64_trans 10\n" % (digest, digest))
    assert bench.recorded_traffic(src, prof) == pytest.approx((100.0 * 2.0 + 50.0 * 1.0) * 1024.0)
    v = bench.recorded_valu(src, prof, 1e-3)
    flops = 64.0 * (100 + 200 + 10 + 2 * 300)
    assert v["fp64_tflops"] == pytest.approx(round(flops / 1e-3 / 1e12, 3))
    assert v["fp64_frac_of_peak"] == pytest.approx(round(flops / 1e-3 / 1e12 / bench.FP64_VALU_PEAK_TF, 4))
    assert v["valu_issue_frac"] == pytest.approx(round(1e6 * 4.0 / (1024 * 2.4e9 * 1e-3), 4))
    assert bench.recorded_valu(src, prof, 0.0) is None
    # a changed kernel source makes both records stale
    _write(src, "// kernel source, edited\n")
    assert bench.recorded_traffic(src, prof) is None
    assert bench.recorded_valu(src, prof, 1e-3) is None
    # a missing record, a missing file, a malformed value
    assert bench.recorded_counters(src, prof, "other-record") is None
    assert bench.recorded_traffic(src, str(tmp_path / "absent.md")) is None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    bad = _write(tmp_path / "bad.md", "traffic-record: kernels_sha256 %s fetch_kib x\n" % digest)
    assert bench.recorded_traffic(src, bad) is None


@pytest.mark.parametrize("key", sorted(bench.PROFILE_OF))
def test_bench_profiles_hold_both_records(key):
    """Every bench configuration with a profile points at a committed summary
    that holds a traffic and a VALU record (they count only while their
    kernel-source digest is the current one)."""
    path = os.path.join(ROOT, "profiles", bench.PROFILE_OF[key])
    text = open(path).read()
    for tag in ("traffic-record:", "valu-record:"):
        lines = [ln for ln in text.splitlines() if ln.startswith(tag)]
        assert len(lines) == 1, (path, tag)
        fields = lines[0].split()[1:]
        rec = dict(zip(fields[0::2], fields[1::2]))
        assert len(rec["kernels_sha256"]) == 64
    dim, p, n, flux = key
    assert dim == 3 and flux in ("ranocha", "shima") and "p%d" % p in bench.PROFILE_OF[key]


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_entropy_scale_against_oracle_entropy_variables(orc):
    """bench.entropy_scale = sum_i J_i W_i |w(u_i) . du_i| with the oracle's
    entropy variables and LGL weights (a stand-in for the problem supplies
    1/J; the library's weights come from esdg_operators, a host call)."""
    import numpy as np
    from paper_2112_10517_amd import esdg
    if not os.path.exists(esdg.LIB_PATH):
        pytest.skip("HIP library not built")
    p, E = 2, 3
    N = p + 1
    nn = N ** 3
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 2.0, (E, nn))
    v = rng.uniform(-0.5, 0.5, (E, 3, nn))
    pr = rng.uniform(0.5, 2.0, (E, nn))
    u = np.empty((E, 5, nn))
    u[:, 0] = rho
    u[:, 1:4] = rho[:, None] * v
    u[:, 4] = pr / 0.4 + 0.5 * rho * (v ** 2).sum(axis=1)
    du = rng.standard_normal((E, 5, nn))
    inv_j = rng.uniform(0.5, 4.0, (E, nn))

    class Stand:
        def inv_jacobian(self):
            return inv_j

    m = orc.Mesh(3, p, (E, 1, 1))
    W = m.weights()
    expect = 0.0
    for e in range(E):
        for i in range(nn):
            w = orc.entropy_vars(3, 1.4, u[e, :, i])
            expect += W[i] / inv_j[e, i] * abs(float(np.dot(w, du[e, :, i])))
    assert bench.entropy_scale(esdg, Stand(), u, du, p) == pytest.approx(expect, rel=1e-12)
