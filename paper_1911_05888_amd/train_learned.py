"""Training and evaluation of the learned correction for the 3D log-normal
viscosity workload (viscous-stress Stokes, Dirichlet walls, Q_2, log10 mu a
smoothed Gaussian field drawn per seed), on the GPU through the library.

Training data: for each of `seeds` independent viscosity fields on the n^3
grid, a random smooth exact solution x* (b = A x*), `cycles` plain FP32
V-cycles from zero; after each cycle the residual r = b - A x and the error
e = x* - x (kernel removed) give one pair, from which `crops` random 16^3
crops (+1 element halo) are stored as bfloat16 (ldgs_learned_collect).  The
output constants c_vel, c_pre are the RMS over all pairs of RMS(e_f) /
RMS(r_f).  Training: Adam on the FP32 master weights with bfloat16 forward
and backward passes (ldgs_learned_train), minibatches drawn uniformly.

Evaluation: on held-out seeds, b = A x* for the L2 projection of the
problem's manufactured solution; FGMRES(m) right-preconditioned by the FP32
V-cycle to 1e-10, without and with the correction (minimal-residual step);
iterations and wall time of each.

    python -m paper_1911_05888_amd.train_learned --n 64 --seeds 250 --out <file.npz>
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

XSTAR_SEED0 = 10_000
CROP_SEED0 = 20_000
ORDER_SEED = 30_000
INIT_SEED = 0


def problem(seed, n, p=2):
    from synth import c5_lognormal
    return c5_lognormal(n=n, p=p, seed=seed)


def collect(seeds, n, p=2, cycles=8, crops=2, crop=16, log=print):
    """Device crops (feat, targ) and the per-pair statistics (pairs, 4)."""
    import torch
    from paper_1911_05888_amd import Context, V_FP32
    from synth.learning import random_smooth_coeffs, crop_origins
    nb = 4 * (p + 1) ** 3
    buf = np.empty(n ** 3 * nb)
    feats, targs, stats = [], [], []
    for i, s in enumerate(seeds):
        t0 = time.perf_counter()
        ctx = Context(problem(s, n, p), vprec=V_FP32)
        random_smooth_coeffs(XSTAR_SEED0 + s, 3, n, p, out=buf)
        xs = torch.from_numpy(buf).to("cuda")
        ctx.project_kernel(xs)
        org = crop_origins(CROP_SEED0 + s, cycles, crops, 3, n, crop, (False, False, False))
        f, t, st = ctx.learned_collect(xs, cycles, crop, org)
        feats.append(f)
        targs.append(t)
        stats.append(st)
        ctx.close()
        del ctx, xs
        torch.cuda.synchronize()
        log(f"[train] seed {s} ({i + 1}/{len(seeds)}) collected in {time.perf_counter() - t0:.1f} s; "
            f"RMS(e)/RMS(r) velocity {st[-1, 2]:.3e} pressure {st[-1, 3]:.3e}")
    return torch.cat(feats), torch.cat(targs), np.concatenate(stats)


def train(feat, targ, stats, ncrops, p=2, crop=16, steps=4000, batch=16, lr=1e-3, log=print):
    from paper_1911_05888_amd import learned_train, init_net_params
    from synth.learning import batch_order
    c_vel = float(np.sqrt(np.mean(stats[:, 2] ** 2)))
    c_pre = float(np.sqrt(np.mean(stats[:, 3] ** 2)))
    t0 = time.perf_counter()
    params, losses, _ = learned_train(3, p, crop, ncrops, feat, targ, c_vel, c_pre, init_net_params(3, p, INIT_SEED),
                                      batch_order(ORDER_SEED, steps, batch, ncrops), lr=lr)
    dt = time.perf_counter() - t0
    w = max(1, steps // 20)
    log(f"[train] {steps} Adam steps in {dt:.1f} s; loss first {np.mean(losses[:w]):.4f} last {np.mean(losses[-w:]):.4f}")
    return params, c_vel, c_pre, losses, dt


def evaluate(params, c_vel, c_pre, seeds, n, p=2, m=150, maxit=400, tol=1e-10, log=print):
    """Per held-out seed: FGMRES(m) with the FP32 V-cycle, plain and with the
    correction: iterations, wall time, final relative residual."""
    import torch
    from paper_1911_05888_amd import Context, V_FP32, FGMRES
    from synth.fields import projected_coeffs
    out = []
    for s in seeds:
        prob = problem(s, n, p)
        ctx = Context(prob, vprec=V_FP32)
        ctx.set_learned(params, c_vel, c_pre)
        xs = torch.tensor(projected_coeffs(prob.exact, prob.dim, n, prob.p), device="cuda")
        b0 = ctx.apply(xs)
        del xs
        rec = dict(seed=s)
        for label, learned in (("plain", False), ("learned", True)):
            runs = []
            for _ in range(2):            # the first run warms up (graph capture, buffers)
                b = b0.clone()
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = ctx.solve(b, x, tol=tol, maxit=maxit, outer=FGMRES, fgmres_m=m, use_learned=learned)
                torch.cuda.synchronize()
                runs.append((time.perf_counter() - t0, info))
                del b, x
            dt, info = runs[-1]
            rec[label] = dict(iters=info["iters"], time_s=dt, relres=info["relres"], converged=bool(st == 0))
        log(f"[eval] seed {s}: plain {rec['plain']['iters']} its {rec['plain']['time_s']:.3f} s; learned "
            f"{rec['learned']['iters']} its {rec['learned']['time_s']:.3f} s")
        out.append(rec)
        ctx.close()
        del ctx, b0
        torch.cuda.empty_cache()
    return out


def save(path, params, c_vel, c_pre, record):
    np.savez(path, params=np.asarray(params, dtype=np.float32), c_vel=c_vel, c_pre=c_pre,
             record=json.dumps(record))


def load(path):
    with np.load(path, allow_pickle=False) as z:
        return (z["params"].astype(np.float32), float(z["c_vel"]), float(z["c_pre"]), json.loads(str(z["record"])))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--seeds", type=int, default=250, help="training viscosity seeds 2000, 2001, ...")
    ap.add_argument("--cycles", type=int, default=8)
    ap.add_argument("--crops", type=int, default=2, help="crops per pair")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-seeds", type=str, default="3000,3001", help="held-out seeds")
    ap.add_argument("--eval-n", type=int, default=0, help="grid of the evaluation (default --n)")
    ap.add_argument("--out", type=str, required=True)
    a = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    seeds = list(range(2000, 2000 + a.seeds))
    t0 = time.perf_counter()
    feat, targ, stats = collect(seeds, a.n, 2, a.cycles, a.crops, log=log)
    t_collect = time.perf_counter() - t0
    ncrops = len(seeds) * a.cycles * a.crops
    params, c_vel, c_pre, losses, t_train = train(feat, targ, stats, ncrops, 2, 16, a.steps, a.batch, a.lr, log=log)
    del feat, targ
    w = max(1, a.steps // 20)
    record = dict(n=a.n, p=2, seeds=[seeds[0], seeds[-1]], cycles=a.cycles, pairs=len(seeds) * a.cycles,
                  crops=ncrops, steps=a.steps, batch=a.batch, lr=a.lr, collect_s=t_collect, train_s=t_train,
                  loss_first=float(np.mean(losses[:w])), loss_last=float(np.mean(losses[-w:])),
                  loss_curve=[float(np.mean(losses[i:i + w])) for i in range(0, a.steps, w)],
                  c_vel=c_vel, c_pre=c_pre)
    ev = [int(s) for s in a.eval_seeds.split(",") if s]
    if ev:
        record["evaluation"] = evaluate(params, c_vel, c_pre, ev, a.eval_n or a.n, log=log)
    save(a.out, params, c_vel, c_pre, record)
    log(f"[train] wrote {a.out}")
    print(json.dumps({k: v for k, v in record.items() if k != "loss_curve"}))


if __name__ == "__main__":
    main()
