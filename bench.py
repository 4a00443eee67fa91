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
stage kernel, HBM-bound; durations from hipEvents around its launches on the
library's stream) and the CPU oracle timed on a bounded sample of the same
workload.  Only one GPU: --gpus above 1 exits with a message.
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


def variants(args, esdg, inputs, u0_dev, x, nodes, dim, p, n):
    """Same workload in FP32 bulk precision and with the Shima volume flux."""
    import numpy as np
    import torch
    out = {}
    steps = max(10, args.steps // 2)
    # FP32 bulk (state, metrics, fluxes in FP32; FP64 reductions) against FP64
    res = {}
    for prec in ("fp64", "fp32"):
        g = esdg.Problem(dim, p, (n, n, n), warp=0.1, volume_flux=args.flux, surface_flux="llf", precision=prec)
        g.set_state(u0_dev)
        dt = 0.5 * g.max_dt(args.cfl)
        g.step(dt=dt, nsteps=10)
        res[prec] = g.get_state()
        g.set_state(u0_dev)
        ms = time_steps(g, steps, 3, args.cfl, torch)
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
    # Shima (KEP, no log means) volume flux, FP64
    g = esdg.Problem(dim, p, (n, n, n), warp=0.1, volume_flux="shima", surface_flux="llf")
    g.set_state(u0_dev)
    ms = time_steps(g, steps, 3, args.cfl, torch)
    g.close()
    out["shima_fp64"] = {"pid_ns": round(ms * 1e6 / (4 * nodes), 6), "ms_per_step": round(ms, 6)}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--flux", default="ranocha", choices=["ranocha", "shima"])
    ap.add_argument("--n", type=int, default=16, help="elements per direction")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="budget of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-steps", type=int, default=10,
                    help="steps with per-kernel hipEvent timing (after the timed region)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32-bulk and Shima variants of the workload")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (HBM "
                         "counter calibration under a profiler)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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

    # per-kernel durations (hipEvents around each launch on the library's stream)
    g.timing(True)
    g.timing_reset()
    run(args.timing_steps)
    vol_ms, vol_n = g.timing_read(esdg.KERNEL_STAGE)
    red_ms, red_n = g.timing_read(esdg.KERNEL_REDUCE)
    g.timing(False)
    g.timing_reset()
    vol_avg_s = vol_ms / vol_n * 1e-3
    bytes_per_node = algorithmic_stage_bytes(dim, p + 1, curved=True)
    traffic_bytes = bytes_per_node * nodes
    achieved_gbs = traffic_bytes / vol_avg_s / 1e9

    line = {
        "metric": "PID (ns per DOF per RHS), FP64 plain single problem",
        "value": round(pid_ns, 6),
        "unit": "ns/DOF/RHS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
        "dof_per_s": 4 * nodes / (ms_per_step * 1e-3),
        "event_ms_per_step": round(ev_ms / args.steps, 6),
        "kernels_us": {
            "stage": round(1e3 * vol_ms / vol_n, 3),
            "reduce": round(1e3 * red_ms / max(red_n, 1), 3),
        },
        "roofline": {
            "kernel": "stage_kernel<3,%d,%s,curved,double>" % (p + 1, args.flux),
            "bound": "hbm",
            "achieved": round(achieved_gbs, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes_per_node": bytes_per_node,
            "bytes_per_launch": traffic_bytes,
            "avg_launch_us": round(vol_avg_s * 1e6, 3),
        },
        "cpu_baseline": None,
    }

    if not args.no_variants:
        line["variants"] = variants(args, esdg, inputs, u0_dev, x, nodes, dim, p, n)

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
        import oracle
        m = oracle.Mesh(dim, p, (n, n, n), warp=0.1, vol_flux=args.flux, surf_flux="llf")
        uc = inputs.random_fourier(m.coords(), 2)
        steps = 0
        t0 = time.perf_counter()
        while True:
            uc, _ = m.rk4(uc, 0.0, 1, cfl=args.cfl)
            steps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": round(el * 1e9 / (steps * 4 * nodes), 3),
            "unit": "ns/DOF/RHS",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d RK4 steps (CFL %.2f, %d RHS) of the same %d^3 p=%d workload, %.1f s"
                      % (steps, args.cfl, 4 * steps, n, p, el),
        }
    print(json.dumps(line), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
