"""Batched stepping, tile variants and serving on the GPU.

A batch launches one stage kernel per group of problems with equal kernel
parameters; the per-element arithmetic does not depend on the other members,
the tile variant or graph replay, so every comparison with the problem run
alone is exact (np.array_equal).  Per-problem parity of the batched FP32 path
against the FP64 oracle uses the FP32 bar of the single-problem tests.
"""
import numpy as np
import pytest

from paper_2112_10517_amd import inputs

import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def esdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10517_amd import esdg as E
    E.load_library()
    return E


# (dim, p, n, warp, volume flux, surface flux, precision)
MIX = [
    (3, 3, (4, 3, 5), 0.1, "ranocha", "llf", "fp64"),
    (3, 3, (3, 3, 3), 0.0, "ranocha", "llf", "fp64"),
    (3, 3, (5, 4, 3), 0.1, "ranocha", "llf", "fp64"),   # same group as the first
    (3, 5, (2, 3, 2), 0.1, "shima", "llf", "fp64"),
    (2, 4, (6, 5), 0.05, "ranocha", "ranocha", "fp64"),
    (3, 4, (4, 4, 4), 0.0, "ranocha", "llf", "fp32"),
    (3, 6, (2, 2, 3), 0.1, "ranocha", "llf", "fp32"),
    (3, 2, (6, 5, 4), 0.1, "ranocha", "llf", "fp32"),
]


def make(esdg, spec, seed):
    dim, p, n, warp, vf, sf, prec = spec
    q = esdg.Problem(dim, p, n, warp=warp, volume_flux=vf, surface_flux=sf, precision=prec)
    u = inputs.random_fourier(q.coords(), seed)
    q.set_state(u)
    return q, u


def pair(esdg, specs, seed0=10):
    """The same problems twice: one set for the batch, one to run alone."""
    a, b = [], []
    for i, s in enumerate(specs):
        a.append(make(esdg, s, seed0 + i)[0])
        b.append(make(esdg, s, seed0 + i)[0])
    return a, b


@pytest.mark.parametrize("graphs,concurrent", [(False, False), (True, False), (True, True), (False, True)])
def test_batch_cfl_steps_match_alone(esdg, graphs, concurrent):
    batched, alone = pair(esdg, MIX)
    with esdg.Batch(batched, graphs=graphs, concurrent=concurrent) as B:
        groups, tiles = B.info()
        assert groups == len(MIX) - 1 and tiles > 0
        B.step(nsteps=3, cfl=0.4)
        B.step(nsteps=2, cfl=0.4)
        tb = B.times()
        B.sync()
    for q, r, t in zip(batched, alone, tb):
        tr = r.step(nsteps=3, cfl=0.4, t=0.0)
        tr = r.step(nsteps=2, cfl=0.4, t=tr)
        assert t == tr
        assert np.array_equal(q.get_state(), r.get_state())
        assert q.get_time() == t


def test_batch_autotune_times_whole_groups(esdg):
    # the batch autotuner times every variant of a group on the group's own
    # launch (RHS mode into the members' RHS buffers): states unchanged, a
    # variant stored for each 3D group, and the tuned batch still steps
    # exactly as its members alone (which use the same process-wide table)
    batched, alone = pair(esdg, MIX, seed0=70)
    before = [r.tile_variant()[0] for r in alone]
    try:
        u0 = [q.get_state() for q in batched]
        with esdg.Batch(batched, graphs=True) as B:
            B.autotune(reps=2)
            for q, u in zip(batched, u0):
                assert np.array_equal(q.get_state(), u)
            for q in batched:
                v, epb = q.tile_variant()
                assert 0 <= v < esdg.TILE_VARIANTS and epb >= 1
            B.step(nsteps=2, cfl=0.4)
            tb = B.times()
            B.sync()
        for q, r, t in zip(batched, alone, tb):
            tr = r.step(nsteps=2, cfl=0.4, t=0.0)
            assert t == tr
            assert np.array_equal(q.get_state(), r.get_state())
    finally:
        for r, v in zip(alone, before):
            r.set_tile_variant(v)


def test_batch_fixed_dt_and_rhs_match_alone(esdg):
    batched, alone = pair(esdg, MIX, seed0=30)
    with esdg.Batch(batched, graphs=True) as B:
        outs = [np.empty(q.shape) for q in batched]
        B.rhs(outs)
        for q, r, o in zip(batched, alone, outs):
            assert np.array_equal(o, r.rhs())
        B.step(dt=1e-4, nsteps=4)
        tb = B.times()
    for q, r, t in zip(batched, alone, tb):
        r.step(dt=1e-4, nsteps=4)
        assert np.array_equal(q.get_state(), r.get_state())
        assert t == r.get_time()


def test_batch_member_stepped_alone_in_between(esdg):
    # parity alignment: a member stepped outside the batch rejoins it
    batched, alone = pair(esdg, MIX[:4], seed0=50)
    with esdg.Batch(batched) as B:
        B.step(nsteps=1, cfl=0.3)
        batched[1].step(nsteps=1, cfl=0.3)
        B.step(nsteps=2, cfl=0.3)
        tb = B.times()
    for i, r in enumerate(alone):
        r.step(nsteps=1, cfl=0.3, t=0.0)
        if i == 1:
            r.step(nsteps=1, cfl=0.3)
        r.step(nsteps=2, cfl=0.3)
        assert np.array_equal(batched[i].get_state(), r.get_state())
        assert tb[i] == r.get_time()


def test_batch_end_times(esdg):
    specs = MIX[:3]
    batched, _ = pair(esdg, specs, seed0=70)
    dt0 = [q.max_dt(0.5) for q in batched]
    t_end = np.array([2.5 * dt0[0], 1e9, 0.7 * dt0[2]])
    with esdg.Batch(batched, t_end=t_end) as B:
        B.step(nsteps=4, cfl=0.5)
        t = B.times()
        assert t[0] == t_end[0] and t[2] == t_end[2] and t[1] < 1e9
        frozen = [batched[0].get_state(), batched[2].get_state()]
        B.step(nsteps=2, cfl=0.5)
        assert np.array_equal(batched[0].get_state(), frozen[0])
        assert np.array_equal(batched[2].get_state(), frozen[1])
        assert B.times()[0] == t_end[0]


def test_batch_rejects_duplicates(esdg):
    q, _ = make(esdg, MIX[0], 1)
    with pytest.raises(esdg.EsdgError):
        esdg.Batch([q, q])


CASES_VARIANT = [
    # odd element counts leave the last workgroup of the multi-element node
    # tiles partly empty (p = 2 FP32: 26 elements per tile; p = 3 and 5 FP64: 2)
    (3, 2, (3, 3, 3), 0.1, "ranocha", "llf", "fp32"),
    (3, 3, (3, 3, 3), 0.1, "ranocha", "llf", "fp64"),
    (3, 5, (3, 3, 3), 0.1, "ranocha", "llf", "fp64"),
    (3, 5, (3, 3, 1), 0.0, "shima", "llf", "fp64"),
    (3, 6, (1, 1, 3), 0.1, "central", "llf", "fp64"),
    (3, 2, (5, 4, 3), 0.1, "ranocha", "llf", "fp64"),
    (3, 4, (3, 4, 3), 0.0, "ranocha", "llf", "fp64"),
    (3, 5, (3, 2, 3), 0.1, "ranocha", "llf", "fp32"),
    (3, 6, (2, 3, 2), 0.1, "shima", "llf", "fp32"),
    (3, 7, (2, 2, 2), 0.0, "ranocha", "ranocha", "fp32"),
    (3, 7, (2, 2, 2), 0.1, "ranocha", "llf", "fp32"),
    (3, 7, (2, 1, 2), 0.1, "ranocha", "llf", "fp64"),
]


# variants that add the same terms in the same order (line layouts 0-2, node
# layout 3); the pair layout (4, N = 8) sums in the order of its rounds
BITWISE_VARIANTS = (0, 1, 2, 3)


@pytest.mark.parametrize("spec", CASES_VARIANT)
def test_tile_variants_are_bit_identical(orc, esdg, spec):
    """The line layouts (0-2) and the node layout (3) give the same bits.
    The pair layout (4) sums each node's terms in another order: it meets
    the parity bar against the oracle and differs from the others by
    rounding only.  The autotuner picks one of them."""
    q, u = make(esdg, spec, 5)
    ref = None
    shapes = set()
    v_before = q.tile_variant()[0]
    try:
        for v in BITWISE_VARIANTS:
            q.set_tile_variant(v)
            shapes.add(q.tile_variant()[1])
            d = q.rhs()
            if ref is None:
                ref = d
            assert np.array_equal(d, ref), "variant %d" % v
        dim, p, n, warp, vf, sf, prec = spec
        if dim == 3:
            q.set_tile_variant(4)
            d4 = q.rhs()
            m = orc.Mesh(dim, p, n, warp=warp, vol_flux=vf, surf_flux=sf)
            o, sig = m.rhs(u), m.rhs_scale(u)
            label = "pair layout p=%d %s %s warp %.1f" % (p, prec, vf, warp)
            if prec == "fp64":
                assert parity.rhs64(d4, o, sig, label=label, u=u) <= 1.0
                assert parity.rhs64(ref, o, sig, label=label + " (node layout)", u=u) <= 1.0
            else:
                assert parity.rhs32(d4, o, sig, label=label) <= parity.SIGMA32
        best, us = q.autotune(reps=3)
        assert 0 <= best < esdg.TILE_VARIANTS and us[best] > 0
        if best in BITWISE_VARIANTS:
            assert np.array_equal(q.rhs(), ref)
        print("%s: elements per workgroup %s, us per variant %s, best %d" % (spec[:3], sorted(shapes), us, best))
    finally:
        q.set_tile_variant(v_before)


def test_batched_fp32_subset_vs_oracle(orc, esdg):
    """Seeded subset of a mixed batch (degrees 2..7, Cartesian and warped,
    FP32 bulk): every member's batched RHS against the FP64 oracle."""
    rng = np.random.default_rng(4)
    specs = []
    for i in range(16):
        p = int(rng.integers(2, 8))
        n = tuple(int(x) for x in rng.integers(2, 5, size=3))
        warp = 0.1 if i % 2 else 0.0
        specs.append((3, p, n, warp, "ranocha", "llf", "fp32"))
    probs, us = [], []
    for i, s in enumerate(specs):
        q, u = make(esdg, s, 100 + i)
        probs.append(q)
        us.append(u)
    with esdg.Batch(probs, graphs=True) as B:
        outs = B.rhs([np.empty(q.shape) for q in probs])
    worst = 0.0
    for s, u, d in zip(specs, us, outs):
        m = orc.Mesh(3, s[1], s[2], warp=s[3], vol_flux=s[4], surf_flux=s[5])
        ref, sigma = m.rhs(u), m.rhs_scale(u)
        err = parity.rhs32(d, ref, sigma, label="batched fp32 p=%d %s warp %.1f" % (s[1], s[2], s[3]))
        worst = max(worst, err)
        assert err <= parity.SIGMA32, (s, err)
    print("batched fp32 subset: worst err/sigma %.2e over %d problems" % (worst, len(specs)))


def test_batched_fp64_member_vs_oracle(orc, esdg):
    specs = [MIX[0], MIX[3], MIX[4]]
    probs, us = [], []
    for i, s in enumerate(specs):
        q, u = make(esdg, s, 200 + i)
        probs.append(q)
        us.append(u)
    with esdg.Batch(probs) as B:
        outs = B.rhs([np.empty(q.shape) for q in probs])
    for s, u, d in zip(specs, us, outs):
        m = orc.Mesh(s[0], s[1], s[2], warp=s[3], vol_flux=s[4], surf_flux=s[5])
        ref, sigma = m.rhs(u), m.rhs_scale(u)
        assert parity.rhs64(d, ref, sigma, label="batched fp64 %dD p=%d %s" % (s[0], s[1], s[2]), u=u) <= 1.0


# ---- serving

def job(kind, n, p, prec="fp32"):
    """(mesh keywords, initial state) of a served job: density wave on
    [-1,1]^3 or Taylor-Green vortex on [0,2pi]^3, affine, FP32 bulk unless
    prec says otherwise."""
    if kind == "dw":
        mesh = dict(dim=3, p=p, n=(n, n, n), precision=prec)
        lo, hi = (-1.0,) * 3, (1.0,) * 3
    else:
        mesh = dict(dim=3, p=p, n=(n, n, n), lo=(0.0,) * 3, hi=(2 * np.pi,) * 3, precision=prec)
        lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
    from oracle import Mesh
    x = Mesh(3, p, (n, n, n), lo=lo, hi=hi).coords()
    u = inputs.density_wave(x) if kind == "dw" else inputs.taylor_green(x)
    return mesh, u


def serve(esdg, jobs, t_end, steps_per_tick=4, budget=0, max_active=0):
    """Submit jobs (list of (tick to submit at, kind, n, p[, precision])); run to completion.
    Returns {index: final state} and the largest number of admitted jobs."""
    S = esdg.Server(cfl=0.5, steps_per_tick=steps_per_tick, hbm_budget=budget, max_active=max_active)
    ids, out, peak, tick = {}, {}, 0, 0
    pending = sorted(range(len(jobs)), key=lambda i: jobs[i][0])
    try:
        while pending or len(out) < len(jobs):
            while pending and jobs[pending[0]][0] <= tick:
                i = pending.pop(0)
                mesh, u = job(*jobs[i][1:])
                ids[S.submit(u, t_end, **mesh)] = i
            done, active, queued = S.tick()
            peak = max(peak, active)
            for jid in done:
                st, t, _ = S.job(jid)
                assert st == esdg.JOB_DONE and t == t_end
                out[ids[jid]] = S.fetch(jid)
            tick += 1
            assert tick < 10000
        assert S.memory()[0] == 0
    finally:
        S.close()
    return out, peak


def test_server_result_alone_equals_in_mix(esdg):
    t_end = 0.02
    target = (0, "dw", 3, 3)
    alone, _ = serve(esdg, [target], t_end)
    mix = [(0, "tgv", 4, 4), (1, "dw", 2, 5), target, (2, "tgv", 3, 3), (3, "dw", 3, 4)]
    mixed, peak = serve(esdg, mix, t_end)
    assert peak >= 3
    assert np.array_equal(alone[0], mixed[2])
    # and alone with another tick length: the same steps, the same result
    alone2, _ = serve(esdg, [target], t_end, steps_per_tick=7)
    assert np.array_equal(alone[0], alone2[0])


def served_on_oracle(m, u, t_end, cfl):
    """A served job on the oracle: classical RK4 steps of the CFL step size
    of R17, the last one shortened to end at t_end (the server's rule, R22)."""
    t, k = 0.0, 0
    while t < t_end:
        dt = min(m.max_dt(u, cfl), t_end - t)
        u, _ = m.rk4(u, dt, 1)
        t += dt
        k += 1
    return u, t, k


def test_served_results_vs_oracle(orc, esdg):
    """Each served result against the oracle's RK4 run of the same job to
    the same end time: FP32 jobs in a mix at the FP32 state bar, one FP64
    job (in the same mix) at the FP64 state bar."""
    t_end, cfl = 0.02, 0.5
    mix = [(0, "dw", 3, 3), (0, "tgv", 3, 4), (1, "dw", 2, 5), (1, "tgv", 2, 3, "fp64")]
    out, peak = serve(esdg, mix, t_end)
    assert peak >= 3
    for i, spec in enumerate(mix):
        kind, n, p = spec[1:4]
        prec = spec[4] if len(spec) > 4 else "fp32"
        _, u = job(kind, n, p)
        lo, hi = ((-1.0,) * 3, (1.0,) * 3) if kind == "dw" else ((0.0,) * 3, (2 * np.pi,) * 3)
        m = orc.Mesh(3, p, (n, n, n), lo=lo, hi=hi, vol_flux="ranocha", surf_flux="llf")
        uo, t, k = served_on_oracle(m, u, t_end, cfl)
        assert t == t_end
        sigma0 = m.rhs_scale(u)
        label = "served %s %s %d^3 p=%d, %d steps to t=%.2f" % (prec, kind, n, p, k, t_end)
        if prec == "fp64":
            assert parity.state64(out[i], uo, sigma0, t_end, label=label, u0=u) <= 1.0
        else:
            assert parity.state32(out[i], uo, sigma0, t_end, k, label=label) <= 1.0


def test_server_density_wave_accuracy(esdg):
    # the served FP32 result is the density wave at t_end up to the scheme's
    # error: within 20% of the error of the FP64 single-problem path stepped
    # to the same end time with a fixed step below the CFL step
    t_end, n, p = 0.05, 4, 4
    out, _ = serve(esdg, [(0, "dw", n, p)], t_end)
    q = esdg.Problem(3, p, (n, n, n))
    x = q.coords()
    q.set_state(inputs.density_wave(x))
    k = int(np.ceil(t_end / q.max_dt(0.5)))
    q.step(dt=t_end / k, nsteps=k)
    exact = inputs.density_wave(x, t=t_end)
    err = np.abs(out[0][:, 0] - exact[:, 0]).max()
    err64 = np.abs(q.get_state()[:, 0] - exact[:, 0]).max()
    print("served density wave %d^3 p=%d to t=%.2f: rho Linf error %.3e (fp64 single problem %.3e)"
          % (n, p, t_end, err, err64))
    assert err <= 1.2 * err64 + 1e-5


def test_server_admission_by_memory(esdg):
    one = esdg.footprint(3, 3, (3, 3, 3), precision="fp32")
    jobs = [(0, "dw", 3, 3)] * 4
    out, peak = serve(esdg, jobs, 0.01, budget=int(2.5 * one))
    assert peak == 2 and len(out) == 4
    for i in range(1, 4):
        assert np.array_equal(out[0], out[i])


def test_graph_replays_match_eager_step_by_step(esdg):
    """Each replay of a captured step is checked against the eager batch,
    with host reads (eager work and synchronisation) between the replays."""
    a, b = pair(esdg, MIX[:6], seed0=90)
    with esdg.Batch(a, graphs=True, concurrent=True) as G, esdg.Batch(b, graphs=False) as E:
        for step in range(5):
            kw = dict(dt=2e-4) if step == 2 else dict(cfl=0.4)
            G.step(nsteps=1, **kw)
            E.step(nsteps=1, **kw)
            assert np.array_equal(G.times(), E.times()), step
            for qa, qb in zip(a, b):
                assert np.array_equal(qa.get_state(), qb.get_state()), step


def test_server_reports_failed_job_and_releases_memory(esdg):
    # a job whose initial pressure is negative is flagged by the stage kernel
    # (non-physical state), retired as FAILED and its memory returned
    S = esdg.Server(cfl=0.5, steps_per_tick=2)
    try:
        mesh, u = job("dw", 2, 3)
        good = S.submit(u, 0.01, **mesh)
        bad_u = u.copy()
        bad_u[:, 4] = -1.0  # rho e < 0 -> p < 0
        bad = S.submit(bad_u, 0.01, **mesh)
        seen = {}
        for _ in range(200):
            done, active, queued = S.tick()
            for jid in done:
                seen[jid] = S.job(jid)[0]
            if len(seen) == 2:
                break
        assert seen[bad] == esdg.JOB_FAILED and seen[good] == esdg.JOB_DONE
        S.fetch(bad)
        u_good = S.fetch(good)
        assert np.all(np.isfinite(u_good))
        assert S.memory()[0] == 0
        with pytest.raises(esdg.EsdgError):
            S.submit(u, 0.0, **mesh)  # t_end must exceed t0
        with pytest.raises(esdg.EsdgError):
            S.fetch(good)  # already released
    finally:
        S.close()


def test_server_rejects_job_larger_than_budget(esdg):
    mesh, u = job("dw", 2, 3)
    S = esdg.Server(cfl=0.5, hbm_budget=1024)
    try:
        with pytest.raises(esdg.EsdgError):
            S.submit(u, 0.01, **mesh)
    finally:
        S.close()
