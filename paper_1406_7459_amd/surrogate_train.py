"""Train and evaluate the learned demag increment on the film256 workload.

Pairs come from the solver's own trajectories (mm_sur_make_pair): seeded
random initial states in seeded in-plane fields (|mu0 H| <= 50 mT), a few
exact RK4 steps to leave the first transient, then one pair per step.  The
network is trained online with Adam on the GPU by the library's kernels.
Evaluation runs held-out trajectories with (a) the exact path, (b) the
trained network and (c) no network (the stage-1 field reused in stages 2-4),
each gated at the tolerance, and reports residuals, fallbacks, the <m> error
against the exact path and the time per step.

  python -m paper_1406_7459_amd.surrogate_train [--seconds 120] [--out f.json]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def init_params(count_layers, seed):
    """He-style uniform initialisation (same recipe as the FP64 reference)."""
    chans = (3, 32, 32, 32, 32, 32, 3)
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for cin, cout in zip(chans[:-1], chans[1:]):
        bound = math.sqrt(6.0 / (cin * 27)) * 0.5
        out.append(g.uniform(-bound, bound, cout * cin * 27))
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=120.0, help="training time budget")
    ap.add_argument("--pairs", type=int, default=20000, help="training pairs at most")
    ap.add_argument("--per-traj", type=int, default=100)
    ap.add_argument("--lr", type=float, default=3e-4,
                    help="initial Adam step; decays tenfold over the budget (1e-3 diverged after ~2000 pairs)")
    ap.add_argument("--eval-steps", type=int, default=40)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="save the trained parameters (.npy)")
    args = ap.parse_args(argv)

    import torch
    from paper_1406_7459_amd import mm
    from paper_1406_7459_amd import workloads as W

    wl0 = W.film256(0)
    nx, ny, nz = wl0.shape
    plan = mm.Plan(nx, ny, nz, *wl0.cell)
    plan.autotune(reps=3)
    sur = mm.Surrogate(nx, ny, nz)
    sur.set_params(init_params(6, 5000))

    def params_of(wl):
        m = wl.mat
        return mm.LLGParams.make(Ms=m.Ms, A=m.A, alpha=m.alpha, gamma0=m.gamma0, Hext=m.Hext, dt=m.dt)

    # ---- training on solver pairs
    t0 = time.perf_counter()
    losses = []
    tvar = []   # mean square of the normalised target (the loss of a zero network)
    curve = []
    pairs = 0
    traj = 0
    dm = torch.empty((3, nz, ny, nx), device="cuda")
    dh = torch.empty_like(dm)
    while pairs < args.pairs and time.perf_counter() - t0 < args.seconds:
        wl = W.film256(traj)
        p = params_of(wl)
        M = torch.from_numpy((wl.mat.Ms * wl.initial_unit()).astype(np.float32)).cuda()
        plan.step(p, M, 20)
        for _ in range(args.per_traj):
            mm.Surrogate.make_pair(plan, p, M, 1, dm, dh)
            frac = max(pairs / max(1, args.pairs), (time.perf_counter() - t0) / args.seconds)
            lr = args.lr * (0.1 ** min(1.0, frac))
            losses.append(sur.train_step(dm, dh, lr))
            tvar.append(float((dh.pow(2).mean() / dm.pow(2).mean()).item()))
            pairs += 1
            if pairs % 250 == 0:
                curve.append({"pairs": pairs, "loss": float(np.mean(losses[-250:])),
                              "zero_net_loss": float(np.mean(tvar[-250:])), "s": time.perf_counter() - t0})
                print("pairs %d loss %.5f zero-net %.5f" % (pairs, curve[-1]["loss"], curve[-1]["zero_net_loss"]),
                      file=sys.stderr, flush=True)
            if pairs >= args.pairs or time.perf_counter() - t0 >= args.seconds:
                break
        traj += 1
    train_s = time.perf_counter() - t0
    if args.weights:
        np.save(args.weights, sur.get_params())

    # ---- held-out evaluation
    def run(kind, wl, steps):
        p = params_of(wl)
        M = torch.from_numpy((wl.mat.Ms * wl.initial_unit()).astype(np.float32)).cuda()
        plan.step(p, M, 20)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st = None
        if kind == "exact":
            plan.step(p, M, steps)
        else:
            st = sur.step(plan, p, M, steps, tol=args.tol)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - ts) / steps
        mavg = plan.reduce(p, M)["m_avg"]
        return M, st, dt, mavg

    evals = []
    trained = sur.get_params()
    for k in range(2):
        wl = W.film256(900 + k)
        Me, _, te, me = run("exact", wl, args.eval_steps)
        sur.set_params(trained)
        Mt, stt, tt, mt = run("trained", wl, args.eval_steps)
        sur.zero()
        Mz, stz, tz, mz = run("zero", wl, args.eval_steps)
        sur.set_params(trained)
        evals.append({
            "trajectory_seed": 5000 + 900 + k,
            "exact_ms_per_step": te * 1e3,
            "trained": dict(stt, ms_per_step=tt * 1e3,
                            m_avg_err=float(np.abs(np.array(mt) - np.array(me)).max()),
                            state_rel_l2=float(torch.linalg.norm(Mt - Me) / torch.linalg.norm(Me))),
            "no_network": dict(stz, ms_per_step=tz * 1e3,
                               m_avg_err=float(np.abs(np.array(mz) - np.array(me)).max()),
                               state_rel_l2=float(torch.linalg.norm(Mz - Me) / torch.linalg.norm(Me))),
        })
    # surrogate inference time alone
    x = torch.randn((3, nz, ny, nx), device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        sur.forward(x, y, normalize=True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(20):
        sur.forward(x, y, normalize=True)
    torch.cuda.synchronize()
    inf_ms = (time.perf_counter() - ts) / 20 * 1e3
    H = torch.empty_like(x)
    ts = time.perf_counter()
    for _ in range(20):
        plan.demag(x, H)
    torch.cuda.synchronize()
    demag_ms = (time.perf_counter() - ts) / 20 * 1e3
    out = {
        "workload": "film256 (256x256x4, 4 nm, Ms 8e5, A 1.3e-11, alpha 0.1, in-plane |mu0 H| <= 50 mT)",
        "network": "6 x conv3x3x3, channels 3-32-32-32-32-32-3, GELU, BF16 MFMA / FP32 accumulate",
        "pairs": pairs, "trajectories": traj, "train_s": train_s,
        "loss_first": float(np.mean(losses[:20])) if losses else None,
        "loss_last": float(np.mean(losses[-20:])) if losses else None,
        "curve": curve,
        "tol": args.tol, "eval_steps": args.eval_steps, "eval": evals,
        "inference_ms": inf_ms, "exact_demag_ms": demag_ms,
        "speedup_vs_plain_fp32": (np.mean([e["exact_ms_per_step"] for e in evals])
                                  / np.mean([e["trained"]["ms_per_step"] for e in evals])),
    }
    s = json.dumps(out)
    if args.out:
        with open(args.out, "w") as f:
            f.write(s + "\n")
    print(s)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
