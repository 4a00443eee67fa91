"""The library's host-built curl-form metrics against the oracle's (CPU).

Both sides evaluate the conservative curl form of the metric terms (Sec. 2.3,
reading R10) independently in FP64; the library on coordinates shifted by an
element-local constant, which the form annihilates because derivatives along
different directions commute.  The curl form applies a derivative operator
twice, so each construction carries rounding of order eps * max|D~|^2
relative to max|Ja|.  This test pins the agreement at that scale on warped
boxes of degree 3, 5 and 7 (it is the geometric part of the FP64 GPU parity
floor), checks both against the discrete metric identities
sum_i D_i Ja^i = 0 at the same scale, and 1/J to a few hundred eps.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def dump_exe(tmp_path_factory):
    csrc = os.path.join(ROOT, "paper_2112_10517_amd", "csrc")
    exe = str(tmp_path_factory.mktemp("geo") / "geometry_dump")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-pthread", "-I", csrc, os.path.join(csrc, "host_ops.cpp"),
                        os.path.join(ROOT, "tests", "c", "geometry_dump.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def identity_residual(D, A, N):
    """max |sum_i D_i Ja^i_m| over max|Ja|, A = [E][n][m][z][y][x]."""
    r = (np.einsum("ij,emzyj->emzyi", D, A[:, 0]) + np.einsum("ij,emzjx->emzix", D, A[:, 1])
         + np.einsum("ij,emjyx->emiyx", D, A[:, 2]))
    return np.abs(r).max() / np.abs(A).max()


@pytest.mark.parametrize("p,n", [(3, (4, 3, 5)), (5, (2, 3, 2)), (7, (2, 1, 2))])
def test_library_metrics_match_oracle(orc, dump_exe, tmp_path, p, n):
    out = str(tmp_path / "metric.bin")
    r = subprocess.run([dump_exe, str(p), *map(str, n), "0.1", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    m = orc.Mesh(3, p, n, warp=0.1)
    Ja, J = m.metrics()
    E, nn, N = m.n_elem, m.nodes, p + 1
    lib = np.fromfile(out).reshape(E, 10, nn)
    ja_orc = Ja.reshape(E, 3, 3, nn)
    ja_lib = lib[:, :9].reshape(E, 3, 3, nn)
    _, _, D = m.operators()
    scale = EPS * np.abs(2 * D - np.diag(np.diag(2 * D))).max() ** 2  # eps * max|D~|^2 (D~ = 2D off the diagonal)
    diff = np.abs(ja_lib - ja_orc).max() / np.abs(ja_orc).max()
    print("p=%d metric difference %.2e = %.2f eps max|D~|^2" % (p, diff, diff / scale))
    assert diff <= 4 * scale, (diff, scale)
    for A in (ja_orc, ja_lib):
        assert identity_residual(D, A.reshape(E, 3, 3, N, N, N), N) <= 4 * scale
    assert np.abs(lib[:, 9] * J - 1.0).max() <= 200 * EPS
