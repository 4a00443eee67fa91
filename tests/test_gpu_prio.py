"""The one-generation form of the line tiles gives the bits of the plain kernel.

A launch whose workgroups are all resident at once (one generation, more
than one workgroup per compute unit) runs the form of tile variant 0 whose
prologue and surface fluxes execute at raised wave priority and whose RK
stage results are stored with the nontemporal hint.  On a 256-CU
MI355X the 16^3 p = 3 launches (1,024 workgroups of 4 elements, four
resident per CU), the 12^3 p = 3 launches (432) and the 16^3 p = 2 launches
(586 workgroups of 7 elements) are such launches.  Tile variant 2 (twice the
elements per workgroup) has no one-generation form and adds the same terms
in the same order, so right-hand sides, states and CFL times must agree bit
for bit.  Inputs are seeded and synthetic.
"""
import numpy as np
import pytest

from paper_2112_10517_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def esdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10517_amd import esdg as E
    E.load_library()
    return E


CASES = [
    # p, n, warp, precision, integrator
    (3, (16, 16, 16), 0.1, "fp64", "rk4"),
    (3, (16, 16, 16), 0.0, "fp64", "rk4"),
    (3, (16, 16, 16), 0.1, "fp32", "rk4"),
    (3, (12, 12, 12), 0.1, "fp64", "rk4"),
    (2, (16, 16, 16), 0.1, "fp64", "rk4"),
    (3, (16, 16, 16), 0.1, "fp64", "ck45"),  # 2N-storage stages (plain stores in both forms)
]


@pytest.mark.parametrize("p,n,warp,prec,integrator", CASES)
def test_priority_form_equals_plain_tile(esdg, p, n, warp, prec, integrator):
    label = "one-generation form p=%d %s warp %.1f %s %s" % (p, n, warp, prec, integrator)
    print(label, flush=True)
    g = esdg.Problem(3, p, n, warp=warp, volume_flux="ranocha", surface_flux="llf", precision=prec,
                     integrator=integrator)
    u = inputs.random_fourier(g.coords(), 7)
    v_before = g.tile_variant()[0]
    out = {}
    try:
        for v in (0, 2):
            g.set_tile_variant(v)
            g.set_state(u)
            du = g.rhs()
            t = g.step(dt=0.0, nsteps=3, cfl=0.4, t=0.0)
            out[v] = (du, g.get_state(), t)
        assert np.array_equal(out[0][0], out[2][0]), label + ": right-hand side"
        assert np.array_equal(out[0][1], out[2][1]), label + ": state after 3 CFL steps"
        assert out[0][2] == out[2][2], label + ": time"
    finally:
        g.set_tile_variant(v_before)
        g.close()
