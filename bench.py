"""Benchmark of the flux-differencing DGSEM hot path on one MI355X.

Workload (default): 3D compressible Euler, warped periodic 16^3-element mesh
on [-1,1]^3 (x_m = xi_m + 0.1 sin(pi xi) sin(pi eta) sin(pi zeta)), p = 3
(262,144 nodes, 1.31 M node-variables), FP64, seeded smooth random state
(rho, p in [0.8,1.2], |v| <= 0.1, |k| <= 4, seed 2), Ranocha volume flux,
local Lax-Friedrichs surface flux.  A step is one classical RK4 step in CFL
mode: the FP64 CFL reduction, then four launches of the fused stage kernel
(surface flux + volume term + lifting + stage update).  The metric is the paper's
performance index PID = time per RHS evaluation / #DOF (Sec. 4, one DOF per
volume node), here wall time per step / (4 x #nodes), lower is better.

Prints one JSON line with the roofline of the dominant kernel (the fused
stage kernel, HBM-bound; its average launch duration from the hipEvent pair
around the timed steps on the library's stream) and the CPU oracle timed on a
bounded sample of the same workload.  The default warm-up (400 steps, about
35 ms) lets the clocks settle before the timed region.  Only one GPU: --gpus
above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_VALU_PEAK_TF = 78.6    # MI355X FP64 vector
KERNEL_SOURCE = os.path.join(ROOT, "paper_2112_10517_amd", "csrc", "kernels.hpp")
# rocprofv3 records (HBM traffic, FP64 VALU instruction counts) of the stage
# kernel, by (dim, p, elements per direction, volume flux) of the bench line
# they were taken on; used only while the kernel source is unchanged
PROFILE_OF = {(3, 3, 16, "ranocha"): "stage_kernel_3d_p3_warped16_fp64.md",
              (3, 7, 32, "ranocha"): "stage_kernel_3d_p7_warped32_fp64.md"}


def algorithmic_stage_bytes(dim: int, N: int, curved: bool, real_bytes: int = 8) -> float:
    """Bytes per node one fused stage launch must move, averaged over the RK4 stages.

    state registers: stage 1 reads U, writes R and Y (3 arrays); stages 2-3 read
    Y, U, R and write R, Y (5); stage 4 reads Y, R and writes U (3): mean 4
    arrays of (dim+2) values.  Metrics (curved): dim*dim contravariant
    components + 1/J per node.  Surface: the neighbours' traces, 2*dim faces of
    N^(dim-1) nodes and (dim+2) values per element, i.e. 2*dim*(dim+2)/N per
    node, and one dim-vector normal per face node, dim*dim/N per node
    (curved).
    """
    nv = dim + 2
    state = 4 * nv
    metric = (dim * dim + 1) if curved else 0
    traces = 2 * dim * nv / N
    normals = dim * dim / N if curved else 0
    return (state + metric + traces + normals) * real_bytes


def recorded_counters(kernel_source: str, profile: str, tag: str):
    """The `tag:` record of rocprofv3 counters in `profile` as a dict, if it
    was taken on the current kernel source (else None)."""
    import hashlib
    try:
        with open(kernel_source, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        with open(profile) as f:
            for line in f:
                if line.startswith(tag + ":"):
                    fl = line.split()
                    rec = dict(zip(fl[1::2], fl[2::2]))
                    if rec.get("kernels_sha256") != digest:
                        return None
                    return {k: float(v) for k, v in rec.items() if k != "kernels_sha256"}
    except (OSError, ValueError, IndexError):
        return None
    return None


def recorded_traffic(kernel_source: str, profile: str):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE record
    in `profile`, if it was taken on the current kernel source (else None)."""
    rec = recorded_counters(kernel_source, profile, "traffic-record")
    if rec is None:
        return None
    try:
        return (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"]) * 1024.0
    except KeyError:
        return None


def recorded_valu(kernel_source: str, profile: str, launch_s: float):
    """FP64 VALU rate of the stage kernel from the rocprofv3 instruction-count
    record in `profile` (current kernel source only): hardware FP64 flops =
    64 lanes x (ADD + MUL + TRANS + 2 FMA) wave instructions; issue fraction =
    VALU wave instructions x 4 cycles / (1,024 SIMDs x 2.4 GHz x launch)."""
    rec = recorded_counters(kernel_source, profile, "valu-record")
    if rec is None or launch_s <= 0:
        return None
    try:
        flops = 64.0 * (rec["fp64_add"] + rec["fp64_mul"] + rec["fp64_trans"] + 2.0 * rec["fp64_fma"])
        tflops = flops / launch_s / 1e12
        out = {"fp64_tflops": round(tflops, 3), "fp64_frac_of_peak": round(tflops / FP64_VALU_PEAK_TF, 4),
               "valu_issue_frac": round(rec["valu_insts"] * 4.0 / (1024 * 2.4e9 * launch_s), 4)}
    except KeyError:
        return None
    # the combined roofline: hardware flops per measured HBM byte, and the
    # achieved rate over min(FP64 peak, intensity x HBM peak)
    traffic = recorded_traffic(kernel_source, profile)
    if traffic:
        oi = flops / traffic
        out["flop_per_hbm_byte"] = round(oi, 3)
        out["roofline_frac"] = round(tflops / min(FP64_VALU_PEAK_TF, oi * HBM_PEAK_GBS / 1e3), 4)
    return out


def time_steps(g, steps, warmup, cfl, torch):
    """ms per CFL-mode RK4 step of problem g (state already set)."""
    for _ in range(warmup):
        g.step(dt=0.0, nsteps=1, cfl=cfl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(dt=0.0, nsteps=1, cfl=cfl)
    torch.cuda.synchronize()
    g.sync()
    return 1e3 * (time.perf_counter() - t0) / steps


# Comparisons of GPU results with the CPU oracle.  The GPU sections record
# what they computed (right-hand sides or states, per precision, on the
# elements listed) with the recipe of the input; the cpu_baseline leg runs
# the oracle on its own mesh and inputs and fills in the errors.
ORACLE_CHECKS = []


def sample_elements(n, count, seed):
    """Seeded element sample of an n^3 box: seams and corners of the periodic
    box plus `count` random elements."""
    import numpy as np
    E = n ** 3
    rng = np.random.default_rng(seed)
    corners = [0, n - 1, n * (n - 1), E - 1, E // 2]
    return np.unique(np.concatenate([corners, rng.choice(E, min(count, E), replace=False)])).astype(np.int64)


def record_check(where, key, mesh, state, gpu, elems=None, steps=None, dt=None, sample=""):
    """Queue an oracle comparison.  where: the dict the result goes into,
    under `key`; mesh: oracle.Mesh arguments; state: (generator name, args)
    of the input; gpu: {precision: host array [elem][var][node]} on `elems`
    (None: every element); steps/dt: compare states after `steps` RK4 steps
    of fixed dt instead of right-hand sides."""
    ORACLE_CHECKS.append(dict(where=where, key=key, mesh=mesh, state=state, gpu=gpu, elems=elems, steps=steps,
                              dt=dt, sample=sample))


def error_figures(gpu, ref, sigma=None):
    """Per conserved variable: relative L2 (over the compared nodes) and Linf
    errors of gpu against ref, and max|gpu - ref| / max sigma."""
    import numpy as np
    nv = ref.shape[1]
    l2 = [float("%.3e" % (np.linalg.norm(gpu[:, v] - ref[:, v]) / np.linalg.norm(ref[:, v]))) for v in range(nv)]
    li = [float("%.3e" % (np.abs(gpu[:, v] - ref[:, v]).max() / np.abs(ref[:, v]).max())) for v in range(nv)]
    out = {"rel_l2": l2, "rel_linf": li}
    if sigma is not None:
        out["max_err_over_sigma"] = float("%.3e" % max(np.abs(gpu[:, v] - ref[:, v]).max() / sigma[:, v].max()
                                                        for v in range(nv)))
    return out


def run_oracle_checks(oracle, inputs):
    """The oracle side of every recorded comparison (cpu_baseline leg)."""
    import numpy as np
    for c in ORACLE_CHECKS:
        t0 = time.perf_counter()
        m = oracle.Mesh(**c["mesh"])
        gen, gargs = c["state"]
        u = getattr(inputs, gen)(m.coords(), **gargs)
        res = {"vs": "FP64 oracle", "sample": c["sample"]}
        if c["steps"]:
            ref, _ = m.rk4(u, c["dt"], c["steps"])
            for prec, arr in c["gpu"].items():
                res[prec] = error_figures(arr, ref)
        else:
            if c["elems"] is None:
                ref, sig = m.rhs(u), m.rhs_scale(u)
            else:
                ref, sig = m.rhs_elements(u, c["elems"])
            for prec, arr in c["gpu"].items():
                res[prec] = error_figures(arr, ref, sig)
        res["oracle_s"] = round(time.perf_counter() - t0, 2)
        del m
        c["where"][c["key"]] = res


def variants(args, esdg, inputs, u0_dev, x, nodes, dim, p, n):
    """Same workload in FP32 bulk precision and with the Shima volume flux."""
    import numpy as np
    import torch
    out = {}
    steps = max(10, args.steps // 2)
    # FP32 bulk (state, metrics, fluxes in FP32; FP64 reductions) against FP64
    # and, in the cpu_baseline leg, both against the oracle: the right-hand
    # side of the initial state and the state after 10 equal steps (the FP64
    # problem's step size for both)
    res = {}
    dt = None
    for prec in ("fp64", "fp32"):
        g = esdg.Problem(dim, p, (n, n, n), warp=0.1, volume_flux=args.flux, surface_flux="llf", precision=prec)
        g.set_state(u0_dev)
        res[prec + "_rhs"] = g.rhs()
        if dt is None:
            dt = 0.5 * g.max_dt(args.cfl)
        g.step(dt=dt, nsteps=10)
        res[prec] = g.get_state()
        g.set_state(u0_dev)
        ms = time_steps(g, steps, 200, args.cfl, torch)
        res[prec + "_ms"] = ms
        g.close()
    err = max(np.abs(res["fp32"][:, v] - res["fp64"][:, v]).max() / np.abs(res["fp64"][:, v]).max()
              for v in range(dim + 2))
    out["fp32_bulk"] = {
        "pid_ns": round(res["fp32_ms"] * 1e6 / (4 * nodes), 6),
        "ms_per_step": round(res["fp32_ms"], 6),
        "speedup_vs_fp64": round(res["fp64_ms"] / res["fp32_ms"], 3),
        "state_max_rel_err_vs_fp64_after_10_steps": float("%.3e" % err),
    }
    mesh = dict(dim=dim, p=p, n=(n, n, n), warp=0.1, vol_flux=args.flux, surf_flux="llf")
    record_check(out["fp32_bulk"], "rhs_vs_oracle", mesh, ("random_fourier", {"seed": 2}),
                 {"fp64": res["fp64_rhs"], "fp32": res["fp32_rhs"]}, sample="every node, initial state")
    record_check(out["fp32_bulk"], "state_vs_oracle_after_10_steps", mesh, ("random_fourier", {"seed": 2}),
                 {"fp64": res["fp64"], "fp32": res["fp32"]}, steps=10, dt=dt,
                 sample="every node, 10 RK4 steps of dt %.4e" % dt)
    # Shima (KEP, no log means) volume flux, FP64
    g = esdg.Problem(dim, p, (n, n, n), warp=0.1, volume_flux="shima", surface_flux="llf")
    g.set_state(u0_dev)
    ms = time_steps(g, steps, 200, args.cfl, torch)
    g.close()
    out["shima_fp64"] = {"pid_ns": round(ms * 1e6 / (4 * nodes), 6), "ms_per_step": round(ms, 6)}
    # the five-stage 2N-storage integrator (five fused stage launches per step)
    g = esdg.Problem(dim, p, (n, n, n), warp=0.1, volume_flux=args.flux, surface_flux="llf", integrator="ck45")
    g.set_state(u0_dev)
    ms = time_steps(g, steps, 200, args.cfl, torch)
    g.close()
    out["ck45_fp64"] = {"pid_ns": round(ms * 1e6 / (5 * nodes), 6), "ms_per_step": round(ms, 6), "rhs_per_step": 5}
    # Legendre-Gauss collocation with entropy projection against LGL, both on
    # the affine box (Gauss collocation is built for affine meshes), FP64
    res = {}
    for kind in ("lgl", "gauss"):
        g = esdg.Problem(dim, p, (n, n, n), volume_flux=args.flux, surface_flux="llf", nodes=kind)
        xg = torch.from_numpy(g.coords()).to(u0_dev.device)
        g.set_state(random_fourier_device(xg, 2, torch))
        res[kind] = time_steps(g, steps, 200, args.cfl, torch)
        if kind == "gauss":
            g.timing(True)
            g.timing_reset()
            g.step(dt=0.0, nsteps=2, cfl=args.cfl)
            st_ms, st_n = g.timing_read(esdg.KERNEL_STAGE)
            pr_ms, pr_n = g.timing_read(esdg.KERNEL_PROJECT)
            g.timing(False)
        g.close()
    # the paper's timing workload (Sec. 4.1): isentropic vortex of strength 20
    # on [-5,5]^3 with 8 elements per direction, p = 3, the same two-point flux
    # in the volume and at the faces; Cartesian, and a warped box standing in
    # for the paper's curved mesh.  Context for its single-core CPU PIDs.
    ctx = {}
    for mesh, warp in (("cartesian", 0.0), ("warped", 0.5)):
        for vf in ("shima", "ranocha"):
            g = esdg.Problem(3, 3, (8, 8, 8), lo=(-5.0,) * 3, hi=(5.0,) * 3, warp=warp, volume_flux=vf,
                             surface_flux=vf)
            g.set_state(torch.from_numpy(inputs.isentropic_vortex(g.coords())).to(u0_dev.device))
            g.step(dt=0.0, nsteps=20, cfl=args.cfl)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(dt=0.0, nsteps=100, cfl=args.cfl)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / 100
            g.sync()
            ctx["%s_%s_pid_ns" % (mesh, vf)] = round(ms * 1e6 / (4 * g.n_dof), 4)
            g.close()
    ctx["paper_cpu_one_core_pid_ns"] = {"cartesian_shima": 26, "curved_shima": 43, "cartesian_ranocha": 42,
                                        "curved_ranocha": 65}
    ctx["workload"] = ("isentropic vortex (strength 20) on [-5,5]^3, 8^3 elements (32,768 nodes), p = 3, FP64, "
                       "RK4 steps at CFL %.2f, 100 steps in one call" % args.cfl)
    out["paper_setup_vortex_8cubed"] = ctx
    out["faces_once_fp64"] = faces_once_ab(args, esdg, torch, u0_dev, dim, p, n)
    out["gauss_vs_lgl_affine_fp64"] = {
        "lgl_pid_ns": round(res["lgl"] * 1e6 / (4 * nodes), 6),
        "gauss_pid_ns": round(res["gauss"] * 1e6 / (4 * nodes), 6),
        "gauss_over_lgl": round(res["gauss"] / res["lgl"], 3),
        "gauss_projection_share": round(pr_ms / (pr_ms + st_ms), 3),
    }
    return out


def faces_once_ab(args, esdg, torch, u0_dev, dim, p, n):
    """Surface fluxes evaluated once per face (a face kernel before every
    stage, Sec. 2.4) against the default fused evaluation (each element
    evaluates its own faces inside the stage kernel), FP64, warped box: the
    headline workload and 32^3 at p = 7.  Steps are timed alternately (best of
    three); the two modes must give bitwise the same states."""
    out = {}
    for pp, nn, steps, warmup in ((p, n, max(10, args.steps // 2), 100), (7, 32, 10, 5)):
        probs = []
        for mode in (esdg.FACES_FUSED, esdg.FACES_ONCE):
            g = esdg.Problem(dim, pp, (nn,) * 3, warp=0.1, volume_flux=args.flux, surface_flux="llf")
            g.set_face_flux_mode(mode)
            probs.append(g)
        if pp == p and nn == n:
            u = u0_dev
        else:
            u = random_fourier_device(torch.from_numpy(probs[0].coords()).to(u0_dev.device), 2, torch)
        best = [float("inf"), float("inf")]
        for _ in range(3):
            for k, g in enumerate(probs):
                g.set_state(u)
                best[k] = min(best[k], time_steps(g, steps, warmup, args.cfl, torch))
        states = []
        for g in probs:
            g.set_state(u)
            g.step(dt=0.0, nsteps=3, cfl=args.cfl)
            st = torch.empty(g.shape, dtype=torch.float64, device=u0_dev.device)
            g.get_state(st)
            states.append(st)
        torch.cuda.synchronize()
        once = probs[1]
        once.timing(True)
        once.timing_reset()
        once.step(dt=0.0, nsteps=2, cfl=args.cfl)
        fc_ms, _ = once.timing_read(esdg.KERNEL_FACE)
        st_ms, _ = once.timing_read(esdg.KERNEL_STAGE)
        once.timing(False)
        nodes = probs[0].n_dof
        out["%dcubed_p%d" % (nn, pp)] = {
            "fused_ms_per_step": round(best[0], 6),
            "once_ms_per_step": round(best[1], 6),
            "once_over_fused": round(best[1] / best[0], 4),
            "fused_pid_ns": round(best[0] * 1e6 / (4 * nodes), 6),
            "once_pid_ns": round(best[1] * 1e6 / (4 * nodes), 6),
            "once_face_kernel_us": round(1e3 * fc_ms / 8, 3),
            "once_stage_kernel_us": round(1e3 * st_ms / 8, 3),
            "bitwise_equal_after_3_steps": bool(torch.equal(states[0], states[1])),
        }
        for g in probs:
            g.sync()
            g.close()
        del states
    return out


def random_fourier_device(x, seed, torch, gamma=1.4):
    """inputs.random_fourier evaluated with torch on the device (same seeded
    modes and scaling; for the large batched workload)."""
    import numpy as np
    from paper_2112_10517_amd import inputs
    d = x.shape[1]
    s = x  # box [-1,1]^3

    def field(modes):
        g = torch.zeros((x.shape[0], x.shape[2]), dtype=torch.float64, device=x.device)
        for k, a, phi in modes:
            arg = sum(float(k[j]) * s[:, j] for j in range(d))
            g += a * torch.sin(np.pi * arg + phi)
        return g / g.abs().max()

    fields = [field(m) for m in inputs.random_fourier_modes(seed, d)]
    rho = 1.0 + 0.2 * fields[0]
    p = 1.0 + 0.2 * fields[1]
    v = [0.1 * f for f in fields[2:]]
    u = torch.empty((x.shape[0], d + 2, x.shape[2]), dtype=torch.float64, device=x.device)
    u[:, 0] = rho
    for j in range(d):
        u[:, 1 + j] = rho * v[j]
    u[:, d + 1] = p / (gamma - 1.0) + 0.5 * rho * sum(vj * vj for vj in v)
    return u


def entropy_scale(esdg, g, u, du, p, gamma=1.4):
    """sum_i J_i W_i |w(u_i) . du_i| over a 3D mesh (host FP64): the size of
    the terms whose sum is dS/dt, the scale an entropy-rate residual is
    measured on.  w: the entropy variables of U = -rho s/(gamma - 1),
    s = ln p - gamma ln rho; J: the library's (esdg_get_inv_jacobian); W: the
    tensor-product LGL weights.  u, du: [elem][var][node] host arrays."""
    import numpy as np
    _, w1, _, _ = esdg.operators(p)
    N = p + 1
    idx = np.arange(N ** 3)
    W = w1[idx % N] * w1[(idx // N) % N] * w1[idx // (N * N)]
    rho = u[:, 0]
    rv2 = (u[:, 1] ** 2 + u[:, 2] ** 2 + u[:, 3] ** 2) / rho
    pr = (gamma - 1.0) * (u[:, 4] - 0.5 * rv2)
    s = np.log(pr) - gamma * np.log(rho)
    wdu = ((gamma - s) / (gamma - 1.0) - 0.5 * rv2 / pr) * du[:, 0]
    wdu += (u[:, 1] * du[:, 1] + u[:, 2] * du[:, 2] + u[:, 3] * du[:, 3] - rho * du[:, 4]) / pr
    return float(np.sum(W[None, :] / g.inv_jacobian() * np.abs(wdu)))


def precision_sweep(args, esdg, inputs, torch, dev):
    """Density wave on the warped 32^3 box at p = 4 and 7, Ranocha + LLF: FP32
    bulk against FP64.  PID of both (CFL-mode RK4 steps); relative L2 and Linf
    differences of the FP32 right-hand side and of the FP32 state after a
    fixed number of equal fixed-dt steps, against the FP64 ones (per
    conserved variable), and both precisions against the oracle on sampled
    elements (cpu_baseline leg); the
    entropy rate (FP64 reduction) of the initial state with the LLF surface
    flux and, as the discrete residual, with the entropy-conservative one,
    relative to sum J W |w . du|.  The
    density wave's momentum and energy right-hand sides are O(|v|) remainders
    of an O(p) pressure-flux divergence that cancels, so their FP32 relative
    error is that of the cancelled terms, not of the result."""
    import numpy as np
    out = {}
    n = args.sweep_n
    for p in [int(q) for q in args.sweep_p.split(",") if q]:
        res, u0 = {}, None
        dt = None
        el = sample_elements(n, 40, p)
        for prec in ("fp64", "fp32"):
            g = esdg.Problem(3, p, (n, n, n), warp=0.1, volume_flux="ranocha", surface_flux="llf", precision=prec)
            if u0 is None:
                u0_host = inputs.density_wave(g.coords())
                u0 = torch.from_numpy(u0_host).to(dev)
            g.set_state(u0)
            res[prec + "_rhs"] = g.rhs()
            res[prec + "_rhs_el"] = res[prec + "_rhs"][el]
            res[prec + "_dsdt_llf"] = g.entropy_rate()
            if dt is None:
                dt = 0.5 * g.max_dt(args.sweep_cfl)
            g.step(dt=dt, nsteps=args.sweep_steps)
            g.sync()
            res[prec + "_u"] = g.get_state()
            g.set_state(u0)
            res[prec + "_ms"] = time_steps(g, args.sweep_steps, 10, args.sweep_cfl, torch)
            res[prec + "_tile"] = g.tile_variant()  # (variant, elements per workgroup)
            nodes = g.n_dof
            g.close()
            # the discrete entropy-rate residual: the same state with the
            # entropy-conservative flux on the faces as well, where dS/dt is
            # zero up to round-off (FP64 reduction in both precisions)
            ge = esdg.Problem(3, p, (n, n, n), warp=0.1, volume_flux="ranocha", surface_flux="ranocha",
                              precision=prec)
            ge.set_state(u0)
            res[prec + "_dsdt_ec"] = ge.entropy_rate()
            res[prec + "_dsdt_scale"] = entropy_scale(esdg, ge, u0_host, ge.rhs(), p)
            ge.close()

        def diff(a, b):
            # per conserved variable (rho, rho v1..v3, rho e)
            l2 = [float("%.3e" % (np.linalg.norm(a[:, v] - b[:, v]) / np.linalg.norm(b[:, v]))) for v in range(5)]
            li = [float("%.3e" % (np.abs(a[:, v] - b[:, v]).max() / np.abs(b[:, v]).max())) for v in range(5)]
            return l2, li

        r2, ri = diff(res["fp32_rhs"], res["fp64_rhs"])
        s2, si = diff(res["fp32_u"], res["fp64_u"])
        out["p%d" % p] = {
            "nodes": nodes,
            "fp64_pid_ns": round(res["fp64_ms"] * 1e6 / (4 * nodes), 6),
            "fp32_pid_ns": round(res["fp32_ms"] * 1e6 / (4 * nodes), 6),
            "fp32_speedup": round(res["fp64_ms"] / res["fp32_ms"], 3),
            "rhs_rel_l2": r2, "rhs_rel_linf": ri,
            "state_rel_l2_after_steps": s2, "state_rel_linf_after_steps": si,
            "steps": args.sweep_steps, "dt": float("%.4e" % dt),
            # tile variant (3 = one lane per node, 0-2 = one lane per line) and elements per workgroup
            "tile_variant_epb": {"fp64": list(res["fp64_tile"]), "fp32": list(res["fp32_tile"])},
            # dS/dt of the initial state with the LLF surface flux and, as the
            # discrete residual, with the entropy-conservative one, and both
            # relative to the scale sum J W |w . du| of the latter (the
            # continuous initial interpolant has no jumps at the faces, so the
            # LLF rate is a residual too)
            "entropy_rate": {prec: {"llf": float("%.4e" % res[prec + "_dsdt_llf"]),
                                    "ec_residual": float("%.4e" % res[prec + "_dsdt_ec"]),
                                    "scale": float("%.4e" % res[prec + "_dsdt_scale"]),
                                    "llf_rel": float("%.3e" % (abs(res[prec + "_dsdt_llf"]) /
                                                               res[prec + "_dsdt_scale"])),
                                    "ec_residual_rel": float("%.3e" % (abs(res[prec + "_dsdt_ec"]) /
                                                                       res[prec + "_dsdt_scale"]))}
                             for prec in ("fp64", "fp32")},
        }
        record_check(out["p%d" % p], "rhs_vs_oracle",
                     dict(dim=3, p=p, n=(n, n, n), warp=0.1, vol_flux="ranocha", surf_flux="llf"),
                     ("density_wave", {}), {"fp64": res["fp64_rhs_el"], "fp32": res["fp32_rhs_el"]}, elems=el,
                     sample="%d elements (seed %d: seams, corners and random), initial state" % (len(el), p))
        del res
    out["workload"] = ("density wave rho = 1 + 0.98 sin(pi(x+y+z)), v = (0.1,0.2,0.3), p = 20 on the warped %d^3 "
                       "box, Ranocha + LLF, RK4 at CFL %.2f" % (n, args.sweep_cfl))
    return out


def batched(args, esdg, torch, dev, fp64_pid):
    """256 uneven periodic 3D problems (n ~ U{4..24}, p ~ U{2..7}, Cartesian or
    warped with equal probability, seeded random Fourier states, seed =
    problem index), FP32 bulk, Ranocha + LLF, one launch per (p, mesh kind)
    group per RK stage, each step replayed as a HIP graph, tiles autotuned.
    The groups' launches of a stage run one after another or on forked
    streams; both are timed and the faster is reported."""
    import numpy as np
    rng = np.random.default_rng(args.batch_seed)
    specs = [(int(rng.integers(4, 25)), int(rng.integers(2, 8)), 0.1 if rng.random() < 0.5 else 0.0)
             for _ in range(args.batch_problems)]
    t0 = time.perf_counter()
    probs = []
    for i, (n, p, warp) in enumerate(specs):
        q = esdg.Problem(3, p, (n, n, n), warp=warp, precision="fp32")
        x = torch.from_numpy(q.coords()).to(dev)
        q.set_state(random_fourier_device(x, i, torch))
        del x
        probs.append(q)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nodes = sum(q.n_dof for q in probs)
    # FP32 right-hand sides of a seeded subset of members, computed by the
    # batch at the initial states, for the oracle comparison (cpu_baseline
    # leg; at most 6 sampled elements per member)
    pick = sorted(set(int(i) for i in np.random.default_rng(args.batch_seed + 1).choice(len(probs), 12, replace=False)))
    outs = [np.empty(q.shape) if i in pick else None for i, q in enumerate(probs)]
    B = esdg.Batch(probs, graphs=True)
    B.rhs(outs)
    checks = {}
    for i in pick:
        n, p, warp = specs[i]
        el = sample_elements(n, 4, 100 + i)[:6]
        record_check(checks, "member%d_p%d_n%d_%s" % (i, p, n, "warped" if warp else "affine"),
                     dict(dim=3, p=p, n=(n, n, n), warp=warp, vol_flux="ranocha", surf_flux="llf"),
                     ("random_fourier", {"seed": i}), {"fp32": outs[i][el]}, elems=el,
                     sample="%d elements of member %d, initial state" % (len(el), i))
    del outs
    t0 = time.perf_counter()
    B.autotune(args.batch_tune_reps)
    tune_s = time.perf_counter() - t0
    groups, tiles = B.info()
    B.close()
    chosen = {}
    for q, (n, p, warp) in zip(probs, specs):
        chosen["p%d_%s" % (p, "warped" if warp else "affine")] = q.tile_variant()
    # the groups of a stage launched one after another, and on forked
    # streams (parallel branches of the step's graph): both timed, the faster
    # reported as the batched figure
    timing = {}
    modes = {"both": (False, True), "sequential": (False,), "concurrent": (True,)}[args.batch_groups]
    for conc in modes:
        B = esdg.Batch(probs, graphs=True, concurrent=conc)
        B.step(nsteps=args.batch_warmup, cfl=args.batch_cfl)
        B.sync()
        torch.cuda.synchronize()
        B.timing(True)
        B.timing_read()
        t0 = time.perf_counter()
        B.step(nsteps=args.batch_steps, cfl=args.batch_cfl)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev_ms, ev_n = B.timing_read()
        B.timing(False)
        B.sync()
        B.close()
        timing[conc] = (1e3 * wall / args.batch_steps, ev_ms / max(ev_n, 1))
    conc = min(timing, key=lambda c: timing[c][0])
    ms, ev_step_ms = timing[conc]
    pid = ms * 1e6 / (4 * nodes)
    # the same problems stepped one after another (no batch): launch-bound small problems
    seq_ms = None
    if args.batch_seq_steps > 0:
        t0 = time.perf_counter()
        for _ in range(args.batch_seq_steps):
            for q in probs:
                q.step(dt=0.0, nsteps=1, cfl=args.batch_cfl)
        torch.cuda.synchronize()
        seq_ms = 1e3 * (time.perf_counter() - t0) / args.batch_seq_steps
    B.close()
    for q in probs:
        q.close()
    return {
        "workload": "%d periodic 3D Euler problems, n ~ U{4..24}, p ~ U{2..7}, Cartesian/warped 50/50 (seed %d), "
                    "random Fourier states (seed = problem index), FP32 bulk, Ranocha + LLF, RK4 in CFL %.2f"
                    % (args.batch_problems, args.batch_seed, args.batch_cfl),
        "nodes": nodes,
        "groups": groups,
        "tiles": tiles,
        "concurrent_groups": bool(conc),
        "ms_per_step_sequential_groups": round(timing[False][0], 4) if False in timing else None,
        "ms_per_step_concurrent_groups": round(timing[True][0], 4) if True in timing else None,
        "pid_ns": round(pid, 6),
        "ms_per_step": round(ms, 4),
        "event_ms_per_step": round(ev_step_ms, 4),
        "steps": args.batch_steps,
        "vs_fp64_plain_pid": round(fp64_pid / pid, 3),
        "unbatched_ms_per_step": None if seq_ms is None else round(seq_ms, 4),
        "batching_speedup": None if seq_ms is None else round(seq_ms / ms, 3),
        "tile_variant_epb": {k: chosen[k] for k in sorted(chosen)},
        "setup_s": round(setup_s, 1),
        "autotune_s": round(tune_s, 2),
        "fp32_members_vs_oracle": checks,
    }


def box_coords(esdg, p, n, lo, hi):
    """Node coordinates [elem][3][node] of the affine periodic n^3 box."""
    import numpy as np
    xi = esdg.operators(p)[0]
    N = p + 1
    h = (hi - lo) / n
    i = np.arange(n)
    line = lo + h * (i[:, None] + 0.5 * (xi[None, :] + 1.0))  # [n][N]
    ex, ey, ez = np.meshgrid(i, i, i, indexing="ij")
    ex, ey, ez = ex.transpose(2, 1, 0).ravel(), ey.transpose(2, 1, 0).ravel(), ez.transpose(2, 1, 0).ravel()
    q = np.arange(N ** 3)
    qx, qy, qz = q % N, (q // N) % N, q // (N * N)
    x = np.empty((n ** 3, 3, N ** 3))
    x[:, 0] = line[ex][:, qx]
    x[:, 1] = line[ey][:, qy]
    x[:, 2] = line[ez][:, qz]
    return x


def serve_run(args, esdg, jobs, arrivals):
    """Run the server over jobs [(kind, n, p, u0)] arriving at the given
    times (s, relative to the start); returns per-job latencies and totals."""
    import numpy as np
    S = esdg.Server(cfl=args.cfl, steps_per_tick=args.serve_tick, graphs=True, max_active=args.serve_max_active,
                    hbm_budget=int(args.serve_hbm_gib * (1 << 30)))
    t_end = args.serve_t_end
    ids, lat, steps_of, pending = {}, {}, {}, list(range(len(jobs)))
    dw_err = None
    max_active, depth = 0, []
    t_start = time.perf_counter()
    while len(lat) < len(jobs):
        now = time.perf_counter() - t_start
        while pending and arrivals[pending[0]] <= now:
            i = pending.pop(0)
            kind, n, p, u0 = jobs[i]
            lo, hi = (-1.0, 1.0) if kind == "dw" else (0.0, 2 * np.pi)
            ids[S.submit(u0, t_end, dim=3, p=p, n=(n, n, n), lo=(lo,) * 3, hi=(hi,) * 3, precision="fp32")] = i
        done, active, queued = S.tick()
        max_active = max(max_active, active)
        depth.append(queued)
        if not done and active == 0 and pending:
            time.sleep(max(0.0, arrivals[pending[0]] - (time.perf_counter() - t_start)))
        for jid in done:
            i = ids[jid]
            st, t, nsteps = S.job(jid)
            if st != esdg.JOB_DONE:
                raise RuntimeError("served job %d failed" % i)
            want = dw_err is None and jobs[i][0] == "dw"
            u = S.fetch(jid, want_state=want)
            lat[i] = time.perf_counter() - t_start - arrivals[i]
            steps_of[i] = nsteps
            if want:
                kind, n, p, _ = jobs[i]
                from paper_2112_10517_amd import inputs
                exact = inputs.density_wave(box_coords(esdg, p, n, -1.0, 1.0), t=t_end)
                dw_err = {"n": n, "p": p, "rho_linf_error": float("%.3e" % np.abs(u[:, 0] - exact[:, 0]).max())}
    elapsed = time.perf_counter() - t_start
    S.close()
    node_rhs = sum(4 * steps_of[i] * jobs[i][1] ** 3 * (jobs[i][2] + 1) ** 3 for i in range(len(jobs)))
    L = np.array([lat[i] for i in range(len(jobs))])
    return {
        "jobs": len(jobs),
        "elapsed_s": round(elapsed, 3),
        "jobs_per_s": round(len(jobs) / (elapsed - arrivals[0]), 4),
        "p50_latency_s": round(float(np.percentile(L, 50)), 3),
        "p99_latency_s": round(float(np.percentile(L, 99)), 3),
        "max_latency_s": round(float(L.max()), 3),
        "max_active": max_active,
        "mean_queue_depth": round(float(np.mean(depth)), 2),
        "served_pid_ns": round(elapsed * 1e9 / node_rhs, 6),
        "density_wave_error": dw_err,
        "max_active_cap": args.serve_max_active,
        "hbm_budget_gib": args.serve_hbm_gib,
    }


def served(args, esdg):
    """Poisson request stream (rate 200/s, seeded) of 3D Euler jobs: density
    wave on [-1,1]^3 or Taylor-Green vortex (Mach 0.1) on [0,2pi]^3 with equal
    probability, n ~ U{8..32}, p ~ U{3,4,5}, affine, t_end 0.5, CFL 0.5, FP32
    bulk, Ranocha + LLF.  The offered load exceeds one GPU's capacity by far,
    so the first `serve_jobs` arrivals are served to completion (saturated
    throughput), then a second window at 80% of the measured capacity."""
    import numpy as np
    from paper_2112_10517_amd import inputs
    rng = np.random.default_rng(args.serve_seed)
    njobs = max(args.serve_jobs, args.serve_sub_jobs)
    gaps = rng.exponential(1.0 / args.serve_rate, size=njobs)
    specs = [("dw" if rng.random() < 0.5 else "tgv", int(rng.integers(8, 33)), int(rng.integers(3, 6)))
             for _ in range(njobs)]
    jobs = []
    for kind, n, p in specs:  # initial states are built before the clock starts
        if kind == "dw":
            u0 = inputs.density_wave(box_coords(esdg, p, n, -1.0, 1.0))
        else:
            u0 = inputs.taylor_green(box_coords(esdg, p, n, 0.0, 2 * np.pi))
        jobs.append((kind, n, p, u0))
    arr = np.cumsum(gaps) - gaps[0]
    sat = serve_run(args, esdg, jobs[:args.serve_jobs], arr[:args.serve_jobs])
    # the density-wave job whose FP32 error is reported, served alone in FP64
    # (same mesh, end time and CFL): the error of the discretisation itself
    de = sat["density_wave_error"]
    if de is not None:
        S = esdg.Server(cfl=args.cfl, steps_per_tick=args.serve_tick, graphs=True)
        n, p = de["n"], de["p"]
        jid = S.submit(inputs.density_wave(box_coords(esdg, p, n, -1.0, 1.0)), args.serve_t_end, dim=3, p=p,
                       n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3, precision="fp64")
        while True:
            done, _, _ = S.tick()
            if jid in done:
                break
        u64 = S.fetch(jid, want_state=True)
        S.close()
        exact = inputs.density_wave(box_coords(esdg, p, n, -1.0, 1.0), t=args.serve_t_end)
        de["rho_linf_error_fp64_alone"] = float("%.3e" % np.abs(u64[:, 0] - exact[:, 0]).max())
    out = {"workload": "Poisson arrivals %.0f/s (seed %d): density wave or Taylor-Green vortex, n ~ U{8..32}, "
                       "p ~ U{3,4,5}, affine, t_end %.2f, CFL %.2f, FP32 bulk, Ranocha + LLF"
                       % (args.serve_rate, args.serve_seed, args.serve_t_end, args.cfl),
           "saturated": sat}
    if args.serve_sub_jobs > 0:
        rate = 0.8 * sat["jobs_per_s"]
        arr2 = np.cumsum(gaps * args.serve_rate / rate) - gaps[0] * args.serve_rate / rate
        sub = serve_run(args, esdg, jobs[:args.serve_sub_jobs], arr2[:args.serve_sub_jobs])
        sub["arrival_rate_per_s"] = round(rate, 4)
        out["sub_saturation"] = sub
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--flux", default="ranocha", choices=["ranocha", "shima"])
    ap.add_argument("--n", type=int, default=16, help="elements per direction")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-single-seconds", type=float, default=5.0,
                    help="seconds of the oracle on one host thread (0: skip)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of --steps steps from the initial state (PID mean and std)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the FP32/FP64 precision sweep")
    ap.add_argument("--sweep-n", type=int, default=32)
    ap.add_argument("--sweep-p", default="4,7")
    ap.add_argument("--sweep-steps", type=int, default=10)
    ap.add_argument("--sweep-cfl", type=float, default=0.3)
    ap.add_argument("--timing-steps", type=int, default=10,
                    help="steps with per-kernel hipEvent timing (after the timed region)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32-bulk and Shima variants of the workload")
    ap.add_argument("--faces-ab-only", action="store_true",
                    help="of the variants, run only the once-per-face vs fused surface-flux comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched FP32 workload")
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-seed", type=int, default=4)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-warmup", type=int, default=2)
    ap.add_argument("--batch-seq-steps", type=int, default=2)
    ap.add_argument("--batch-tune-reps", type=int, default=5)
    ap.add_argument("--batch-groups", default="both", choices=["both", "sequential", "concurrent"],
                    help="launch the groups of a stage one after another, on forked streams, or time both")
    ap.add_argument("--batch-concurrent", action="store_true",  # kept for old command lines: see --batch-groups
                    help="run the groups of a batch step on concurrent streams")
    ap.add_argument("--batch-cfl", type=float, default=0.3,
                    help="CFL number of the batched workload (classical RK4 with this CFL definition is "
                         "unstable at 0.5 for p >= 6)")
    ap.add_argument("--no-served", action="store_true", help="skip the served workload")
    ap.add_argument("--serve-jobs", type=int, default=48, help="arrivals served in the saturated window")
    ap.add_argument("--serve-sub-jobs", type=int, default=32, help="arrivals of the 80%%-capacity window (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-seed", type=int, default=5)
    ap.add_argument("--serve-t-end", type=float, default=0.5)
    ap.add_argument("--serve-tick", type=int, default=4, help="RK steps per server tick")
    ap.add_argument("--serve-max-active", type=int, default=0,
                    help="slots: most jobs stepped together (0: no cap; admission in arrival order as memory frees up)")
    ap.add_argument("--serve-hbm-gib", type=float, default=4.0,
                    help="HBM budget of the admitted jobs' footprints (GiB)")
    ap.add_argument("--preheat-ms", type=float, default=60.0,
                    help="before the warm-up steps, step the problem for this long (untimed, reported as "
                         "preheat_steps): the GPU's clocks ramp over the first tens of milliseconds of load")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (HBM "
                         "counter calibration under a profiler)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d / WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2112_10517_amd import esdg, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dim, p, n = 3, args.p, args.n
    g = esdg.Problem(dim, p, (n, n, n), warp=0.1, volume_flux=args.flux, surface_flux="llf")
    x = g.coords()
    u0 = inputs.random_fourier(x, 2)
    u0_dev = torch.from_numpy(u0).to(dev)
    g.set_state(u0_dev)  # resident in HBM before the timed region
    nodes = g.n_dof

    def run(k):
        for _ in range(k):
            g.step(dt=0.0, nsteps=1, cfl=args.cfl)

    # device pre-heat: the clocks ramp over the first tens of milliseconds of
    # load (after 10 warm-up steps alone the timed region reads ~6% slower)
    preheat_steps = 0
    if args.preheat_ms > 0:
        torch.cuda.synchronize()
        t_ph = time.perf_counter()
        while (time.perf_counter() - t_ph) * 1e3 < args.preheat_ms:
            run(20)
            preheat_steps += 20
            torch.cuda.synchronize()
        g.set_state(u0_dev)
    run(args.warmup)
    g.sync()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    run(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.sync()  # no non-physical state met
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / args.steps
    pid_ns = ms_per_step * 1e6 / (4 * nodes)

    # the paper's PID protocol (Sec. 4.1): mean and standard deviation over
    # five runs, each the same number of steps from the same initial state
    runs = []
    for _ in range(args.repeats):
        g.set_state(u0_dev)
        g.step(dt=0.0, nsteps=1, cfl=args.cfl)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run(args.steps)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t1) * 1e9 / (args.steps * 4 * nodes))
    g.sync()

    # per-kernel durations (hipEvents around each launch on the library's stream)
    g.timing(True)
    g.timing_reset()
    run(args.timing_steps)
    vol_ms, vol_n = g.timing_read(esdg.KERNEL_STAGE)
    red_ms, red_n = g.timing_read(esdg.KERNEL_REDUCE)
    g.timing(False)
    g.timing_reset()
    # average stage-launch duration for the roofline: in the steady state a
    # step is four stage launches and nothing else (the CFL value comes from
    # the previous step's last stage; the timing pass shows no reduction), so
    # the event pair around the timed region -- recorded on torch's current
    # stream, the stream the problem was created on -- divided by the number
    # of launches is the back-to-back launch duration, gaps included.  The
    # per-launch event pairs of the timing pass separate the launches and
    # read higher.
    steady = red_n == 0 and g.stream_ptr() == torch.cuda.current_stream().cuda_stream
    vol_avg_s = ev_ms * 1e-3 / (4 * args.steps) if steady else vol_ms / vol_n * 1e-3
    bytes_per_node = algorithmic_stage_bytes(dim, p + 1, curved=True)
    traffic_bytes = bytes_per_node * nodes
    achieved_gbs = traffic_bytes / vol_avg_s / 1e9

    # the bandwidth a plain streaming copy reaches on this device (512 MiB
    # device to device, read + write bytes, five copies between events)
    cb = 512 << 20
    src = torch.ones(cb // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * cb / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    profile = PROFILE_OF.get((dim, p, n, args.flux))
    line = {
        "metric": "PID (ns per DOF per RHS) FP64 plain vs FP32 batched; served jobs/s + p99 latency",
        "value": round(pid_ns, 6),
        "unit": "ns/DOF/RHS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "preheat_steps": preheat_steps,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3D Euler, warped periodic %d^3 mesh on [-1,1]^3 (warp 0.1), p=%d, "
                        "smooth random Fourier state seed 2, %s volume flux + LLF surface flux, "
                        "RK4 step (CFL %.2f) = CFL reduction + 4 fused stage launches (surface+volume+lift+update)"
                        % (n, p, args.flux, args.cfl),
            "elements": g.n_elem, "nodes": nodes, "node_vars": nodes * g.n_var,
            "rhs_per_step": 4,
        },
        "pid_per_node_var_ns": round(pid_ns / g.n_var, 6),
        "pid_runs_ns": {"mean": round(float(np.mean(runs)), 6), "std": round(float(np.std(runs, ddof=1)), 6),
                        "runs": len(runs), "steps_per_run": args.steps} if len(runs) > 1 else None,
        "dof_per_s": 4 * nodes / (ms_per_step * 1e-3),
        "event_ms_per_step": round(ev_ms / args.steps, 6),
        "kernels_us": {
            "stage": round(vol_avg_s * 1e6, 3),
            "stage_event_pair": round(1e3 * vol_ms / vol_n, 3),
            "reduce": round(1e3 * red_ms / max(red_n, 1), 3),
        },
        "roofline": {
            "kernel": "stage_kernel<3,%d,%s,curved,double>" % (p + 1, args.flux),
            "bound": "hbm",
            "achieved": round(achieved_gbs, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(KERNEL_SOURCE, os.path.join(ROOT, "profiles", profile)) if profile else None,
            "algorithmic_bytes_per_node": bytes_per_node,
            "bytes_per_launch": traffic_bytes,
            "avg_launch_us": round(vol_avg_s * 1e6, 3),
            "copy_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved_gbs / copy_gbs, 4),
            "valu": recorded_valu(KERNEL_SOURCE, os.path.join(ROOT, "profiles", profile), vol_avg_s) if profile else None,
        },
        "cpu_baseline": None,
    }

    if args.faces_ab_only and not args.no_variants:
        line["variants"] = {"faces_once_fp64": faces_once_ab(args, esdg, torch, u0_dev, dim, p, n)}
    elif not args.no_variants:
        line["variants"] = variants(args, esdg, inputs, u0_dev, x, nodes, dim, p, n)

    if not args.no_sweep:
        line["precision_sweep"] = precision_sweep(args, esdg, inputs, torch, dev)
    if not args.no_batched:
        line["batched"] = batched(args, esdg, torch, dev, pid_ns)
    if not args.no_served:
        line["served"] = served(args, esdg)

    if args.calibrate_copy_mib > 0:
        nb = args.calibrate_copy_mib * (1 << 20)
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = {"read": nb, "write": nb}
        del src, dst

    if not args.no_cpu_baseline:
        # the cpu_baseline leg: the CPU oracle timed on the host's cores (the
        # paper's protocol, mean and standard deviation of five runs of
        # equal length from the same initial state), then the oracle side of
        # every recorded comparison with the GPU results
        import oracle
        m = oracle.Mesh(dim, p, (n, n, n), warp=0.1, vol_flux=args.flux, surf_flux="llf")
        uc0 = inputs.random_fourier(m.coords(), 2)
        # steps per run from a first step, so that five runs take about cpu_seconds
        t0 = time.perf_counter()
        m.rk4(uc0, 0.0, 1, cfl=args.cfl)
        per_step = time.perf_counter() - t0
        k = max(1, int(args.cpu_seconds / 5 / per_step))
        pids = []
        for _ in range(5):
            t0 = time.perf_counter()
            m.rk4(uc0, 0.0, k, cfl=args.cfl)
            pids.append((time.perf_counter() - t0) * 1e9 / (k * 4 * nodes))
        line["cpu_baseline"] = {
            "value": round(float(np.mean(pids)), 3),
            "unit": "ns/DOF/RHS",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "std": round(float(np.std(pids, ddof=1)), 3),
            "runs": 5,
            "sample": "5 runs of %d RK4 steps (CFL %.2f, %d RHS each) of the same %d^3 p=%d workload from its "
                      "initial state, %.1f s in all; value = mean, std over the runs"
                      % (k, args.cfl, 4 * k, n, p, sum(pids) * k * 4 * nodes * 1e-9),
        }
        del m
        run_oracle_checks(oracle, inputs)
        if args.cpu_single_seconds > 0:
            # one host thread: like for like with the paper's serial PIDs
            nt = oracle.num_threads()
            oracle.set_num_threads(1)
            try:
                m = oracle.Mesh(dim, p, (n, n, n), warp=0.1, vol_flux=args.flux, surf_flux="llf")
                uc = inputs.random_fourier(m.coords(), 2)
                steps = 0
                t0 = time.perf_counter()
                while True:
                    uc, _ = m.rk4(uc, 0.0, 1, cfl=args.cfl)
                    steps += 1
                    if time.perf_counter() - t0 >= args.cpu_single_seconds:
                        break
                el = time.perf_counter() - t0
            finally:
                oracle.set_num_threads(nt)
            line["cpu_single_core"] = {
                "value": round(el * 1e9 / (steps * 4 * nodes), 3), "unit": "ns/DOF/RHS", "cores": 1,
                "kind": "oracle",
                "sample": "%d RK4 steps (%d RHS) of the same workload, %.1f s" % (steps, 4 * steps, el)}
    print(json.dumps(line), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
