"""Benchmark: LDG-Stokes multigrid on one MI355X.

Workload (the configuration the metric is quoted on): 2D steady viscous-stress
Stokes on the unit square with Dirichlet walls, 256x256 elements, Q_3
(48 unknowns per element, 3,145,728 unknowns), mu = 1 + 0.9 sin(2 pi x) sin(2 pi y),
the paper's manufactured solution.  Synthetic data, generated in-process.

One step = one solve from x = 0 to ||b - A x|| <= 1e-10 ||b|| with the FP32
V-cycle (V(3,3), parity colouring) inside FP64 iterative refinement: every
stage of the hot path (smoother colour passes, residual + restriction,
prolongation, bottom pseudo-inverse, FP64 outer residual) runs in the HIP
library.  value = V-cycle DOF/s inside those solves (unknowns x V-cycles /
solve time).  The plain FP64 stationary V-cycle to the same tolerance, and
the BF16-block variant, are measured beside it.

The roofline object covers the dominant kernel (the finest-level smoother
colour pass), timed with HIP event pairs on the library's stream, one pair
around the back-to-back colour passes of every 4th finest sweep of the timed
solves (the average per pass includes the short gaps between those
launches); the algorithmic bytes per launch are (elements in the colour) x
(n_b^2 inverse entries + 3 n_b vector entries + (p+2)^d viscosity values) x
the storage width, the method's byte model (the kernel moves only the upper
tiles of the symmetric inverse: an effective bandwidth; `traffic` gives the
bytes the counters saw); on levels whose blocks are all equal (periodic, constant
coefficients) the one inverse is not streamed and that term is dropped.  cpu_baseline times the FP64 oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_smooth_colour_c2_n256_p3.json")


def smoother_bytes_per_launch(prob, ncolours, inv_bytes, vec_bytes):
    # the byte model of the method: every element's n_b x n_b inverse once per
    # sweep, x and b in, x out, (p+2)^d viscosity values (the kernel stores and
    # moves only the upper 16 x 16 tiles of the symmetric inverse, so this is
    # an effective bandwidth in the model's units; the measured HBM traffic is
    # reported beside it)
    nb = prob.nb
    per_elem = nb * nb * inv_bytes + 3 * nb * vec_bytes + (prob.p + 2) ** prob.dim * vec_bytes
    return prob.n_elements / ncolours * per_elem


def cpu_baseline(n_sample=64, cycles=25):
    """The FP64 oracle's V-cycle on the n_sample^2 grid of the same problem."""
    from threadpoolctl import threadpool_limits
    from synth import c2_dirichlet_varmu
    from oracle import build_hierarchy
    from oracle.rhs import assemble_rhs
    from oracle.solvers import Solver
    prob = c2_dirichlet_varmu(n=n_sample, p=3)
    with threadpool_limits(limits=1):
        H = build_hierarchy(prob)
        b = assemble_rhs(prob, H.fine.ops)
        S = Solver(H)
        t0 = time.perf_counter()
        x = None
        for _ in range(cycles):
            x = S.vcycle_unscaled(b, x)
        dt = time.perf_counter() - t0
    return dict(value=prob.n_dof * cycles / dt, unit="DOF/s", cores=1, kind="oracle",
                sample=f"FP64 oracle V(3,3) cycles on the {n_sample}x{n_sample} Q_3 grid of the same problem "
                       f"({prob.n_dof} unknowns, {cycles} cycles, {dt:.1f} s); scipy sparse products, one thread")


def train_correction(ctx, prob, nseeds=16, ncycles=8, ncrops=16, crop=16, steps=2000, batch=16):
    """Training pairs from plain V-cycles of the benchmark operator on random
    smooth exact solutions (not the benchmark's right-hand side), then Adam on
    bf16 crops; returns (flat params, c_vel, c_pre, info)."""
    import torch
    from paper_1911_05888_amd import learned_train, init_net_params
    from synth.learning import random_smooth_coeffs, crop_origins, batch_order
    t0 = time.perf_counter()
    feats, targs, stats = [], [], []
    per = tuple(bc == "periodic" for bc in prob.bc)
    for s in range(nseeds):
        xs = torch.tensor(random_smooth_coeffs(1000 + s, prob.dim, prob.n, prob.p), device="cuda")
        ctx.project_kernel(xs)
        org = crop_origins(2000 + s, ncycles, ncrops, prob.dim, prob.n, crop, per)
        f, t, st = ctx.learned_collect(xs, ncycles, crop, org)
        feats.append(f)
        targs.append(t)
        stats.append(st)
    feat, targ, st = torch.cat(feats), torch.cat(targs), np.concatenate(stats)
    c_vel, c_pre = float(np.sqrt(np.mean(st[:, 2] ** 2))), float(np.sqrt(np.mean(st[:, 3] ** 2)))
    ncr = nseeds * ncycles * ncrops
    params, losses, _ = learned_train(prob.dim, prob.p, crop, ncr, feat, targ, c_vel, c_pre,
                                      init_net_params(prob.dim, prob.p, 0), batch_order(5, steps, batch, ncr))
    torch.cuda.synchronize()
    info = dict(train_s=time.perf_counter() - t0, pairs=nseeds * ncycles, crops=ncr, steps=steps,
                loss_first=float(np.mean(losses[:50])), loss_last=float(np.mean(losses[-50:])))
    return params, c_vel, c_pre, info


WORKLOADS = {
    # name: (problem factory, description, extra precisions built beside FP32)
    "c2": ("2D viscous-stress Stokes, Dirichlet walls, {n}x{n} elements, Q_3, "
           "mu = 1 + 0.9 sin2pi x sin2pi y, manufactured solution; FP32 V(3,3) in FP64 iterative refinement to 1e-10"),
    "c4a": ("2D two-phase viscous-stress Stokes, square inclusion (1/4,3/4)^2 with mu 1e4 inside and 1 outside, "
            "Dirichlet walls, {n}x{n} elements, Q_2, two-phase manufactured solution, mod-3 colouring, diagonal scaling; "
            "FP32 V(3,3) in FP64 iterative refinement to 1e-10"),
    "c3": ("3D unsteady viscous-stress Stokes, periodic, {n}^3 elements, Q_2, rho = mu = 1, delta = h^2 / 10 "
           "(Re_eff = 10), seeded Fourier forcing (seed 0), parity colouring; FP32 V(3,3) in FP64 iterative "
           "refinement to 1e-10"),
    "c5": ("3D viscous-stress Stokes, Dirichlet walls, {n}^3 elements, Q_2, log-normal viscosity (random Fourier "
           "features, seed 1001), manufactured solution, parity colouring, diagonal scaling; FP32 V(3,3) in FP64 "
           "iterative refinement to 1e-10"),
}


def make_problem(workload, n):
    from synth import c2_dirichlet_varmu, c3_unsteady_periodic, c4a_square_inclusion, c5_lognormal
    if workload == "c2":
        return c2_dirichlet_varmu(n=n or 256, p=3)
    if workload == "c3":
        return c3_unsteady_periodic(n=n or 64, p=2, re_eff=10.0)
    if workload == "c4a":
        return c4a_square_inclusion(n=n or 512, p=2)
    return c5_lognormal(n=n or 128, p=2)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="elements per axis (default: the workload's)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2",
                    help="c2 (default, the benchmark configuration); c3, c4a and c5 measure the other configurations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 / BF16 comparison solves")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run 3 plain device copies of 256 MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; a domain decomposition over several is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_05888_amd import Context, V_FP64, V_FP32, V_FP32_BF16BLK, STATIONARY, IR
    from synth import c2_dirichlet_varmu

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prob = make_problem(args.workload, args.n)
    n = prob.n
    # the 3D workload keeps FP32 (and BF16-block) V-cycle data only: its FP64
    # block inverses alone would take 196 GB
    builds = (1 << V_FP32_BF16BLK) if args.workload == "c5" else (1 << V_FP64) | (1 << V_FP32_BF16BLK)
    t0 = time.perf_counter()
    ctx = Context(prob, vprec=V_FP32, build_precisions=builds)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"[bench] setup {t_setup:.1f} s, {ctx.ndof} unknowns, {ctx.n_levels} levels", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    b0 = ctx.assemble_rhs(prob.rhs_source())
    print(f"[bench] right-hand side assembled in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ncol = ctx.level_info(0)[2]

    def solve(vprec, outer, tol=1e-10, maxit=60, learned=False):
        ctx.set_vprec(vprec)
        b = b0.clone()
        x = torch.zeros_like(b)
        st, info = ctx.solve(b, x, tol=tol, maxit=maxit, outer=outer, use_learned=learned)
        if st != 0:
            raise RuntimeError(f"solve failed: status {st}, {info}")
        return info

    for _ in range(args.warmup):
        solve(V_FP32, IR)
    torch.cuda.synchronize()
    ctx.profile(4)        # every 4th finest sweep: one event pair around its colour passes
    iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = solve(V_FP32, IR)
        iters += info["iters"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_launches = ctx.profile_read()
    ctx.profile(False)
    value = ctx.ndof * iters / dt
    ms_per_step = 1e3 * dt / args.steps
    print(f"[bench] mixed FP32-in-IR: {iters / args.steps:.1f} V-cycles/solve, {ms_per_step:.2f} ms/solve",
          file=sys.stderr, flush=True)

    # a level whose blocks are all equal holds one inverse: no inverse
    # entries are streamed, the colour pass is the residual + shared update
    shared = ctx.level_shared_inverse(0)
    bytes_launch = smoother_bytes_per_launch(prob, ncol, 0 if shared else 4, 4)
    kname = (f"k_colour_residual<float,{prob.dim},{prob.p}> + k_shared_update_mfma<{prob.nb}> (FP32 matrix cores "
             f"for colours of 8192 elements or more)" if shared else f"k_smooth_colour<float,float,{prob.dim},{prob.p},64>")
    avg_s = k_ms * 1e-3 / max(k_launches, 1)
    achieved = bytes_launch / avg_s / 1e9
    traffic = None
    if args.workload == "c2" and n == 256 and os.path.exists(TRAFFIC_FILE):
        # counters are valid only for the kernel source they were measured on
        import hashlib
        with open(TRAFFIC_FILE) as fh:
            tj = json.load(fh)
        with open(os.path.join(ROOT, "paper_1911_05888_amd", "csrc", "kernels.hip"), "rb") as fh:
            sha = hashlib.sha1(fh.read()).hexdigest()
        if tj.get("kernels_hip_sha1") == sha:
            traffic = tj.get("bytes_per_launch")

    extras = {}
    if not args.no_extras:
        runs = [("fp32_bf16blk_ir", V_FP32_BF16BLK, IR, False)]
        if args.workload != "c5":
            runs = [("plain_fp64_stationary", V_FP64, STATIONARY, False), ("plain_fp64_ir", V_FP64, IR, False)] + runs
        if args.workload == "c2":
            ctx.set_vprec(V_FP32)
            params, c_vel, c_pre, tinfo = train_correction(ctx, prob)
            ctx.set_learned(params, c_vel, c_pre)
            print(f"[bench] learned correction trained in {tinfo['train_s']:.1f} s, loss "
                  f"{tinfo['loss_first']:.3f} -> {tinfo['loss_last']:.3f}", file=sys.stderr, flush=True)
            runs.append(("fp32_learned_ir", V_FP32, IR, True))
        for label, vp, outer, learned in runs:
            solve(vp, outer, learned=learned)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            reps = 3
            its = 0
            for _ in range(reps):
                info = solve(vp, outer, learned=learned)
                its += info["iters"]
            torch.cuda.synchronize()
            tt = (time.perf_counter() - t1) / reps
            extras[label] = dict(time_to_tol_s=tt, iters=its / reps, vcycle_dof_per_s=ctx.ndof * its / reps / tt)
            if learned:
                extras[label].update(fallback_events=info["fallback_events"], training=tinfo)
            print(f"[bench] {label}: {its / reps:.1f} iters, {tt * 1e3:.2f} ms", file=sys.stderr, flush=True)

    line = dict(
        metric="V-cycle DOF/s + wall time to 1e-10 rel. residual, plain FP64 vs mixed/learned",
        value=value, unit="DOF/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="fp32 V-cycle, fp64 outer residual", data="synthetic",
        config=dict(workload=WORKLOADS[args.workload].format(n=n),
                    n=n, p=prob.p, dim=prob.dim, unknowns=ctx.ndof, levels=ctx.n_levels, colours=ncol,
                    time_to_tol_s=dt / args.steps, vcycles_per_solve=iters / args.steps,
                    setup_s=t_setup, **extras),
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                      kernel=kname + " (finest level)",
                      avg_launch_us=avg_s * 1e6, algorithmic_bytes_per_launch=bytes_launch,
                      launches=k_launches, timing="event pairs around whole finest sweeps, every 4th"),
    )
    if not args.no_cpu_baseline and args.workload == "c2":
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
