"""esdg_totals_noalloc (the allocation-free variant of esdg_totals, its
partial sums in the library's static device array) against esdg_totals on
two calls in a row, the second on a smaller problem, through the C ABI.
Both run the same kernels over the same block partition, so the results
must have the same bits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_totals_noalloc_matches_totals():
    import torch
    from paper_2112_10517_amd import esdg, inputs
    cases = [dict(dim=3, p=4, n=(9, 7, 8), warp=0.1, precision="fp64"),   # 504 elements, 63,000 nodes
             dict(dim=2, p=2, n=(3, 2), warp=0.0, precision="fp32")]      # smaller, fewer blocks
    for k, c in enumerate(cases):
        print("case", k, c, flush=True)
        g = esdg.Problem(c["dim"], c["p"], c["n"], warp=c["warp"], precision=c["precision"])
        g.set_state(inputs.random_fourier(g.coords(), 7 + k))
        want = g.totals()
        out = torch.full((g.n_var,), float("nan"), dtype=torch.float64, device="cuda")
        g.totals_noalloc(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (k, got, want)
        # and again, into the same buffer, after a step changed the state
        g.step(dt=1e-4, nsteps=1)
        want2 = g.totals()
        g.totals_noalloc(out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want2), k
        del g
