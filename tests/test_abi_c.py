"""The C ABI from a plain C99 program (tests/c/abi_client.c): the header
compiles as strict C, the program links against the shared library, and the
host-side calls run without a GPU; on the GPU the same program steps problems
through host buffers and checks free stream, conservation, the entropy rate
and batch-vs-alone identity."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2112_10517_amd", "lib")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    from paper_2112_10517_amd import esdg, build
    if not os.path.exists(esdg.LIB_PATH):
        build.build()
    exe = str(tmp_path_factory.mktemp("abi") / "abi_client")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-O1",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_client.c"),
           "-L", LIBDIR, "-lesdg", "-Wl,-rpath," + LIBDIR, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_client_host_calls(client):
    r = subprocess.run([client], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi client ok" in r.stdout


@pytest.mark.gpu
def test_c_client_on_gpu(client):
    r = subprocess.run([client, "--gpu"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi client ok (gpu)" in r.stdout
