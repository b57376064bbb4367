"""Train the trace surrogate on pairs the wave solver generates.

    python -m paper_2603_16393_amd.train_surrogate --pairs 50000 --epochs 8 --out weights.npy \\
        [--ckpt ckpt.npz [--resume]]

Inputs are seeded synthetic models (fwi_inputs.surrogate_training_pair):
each pair is a model v and a smooth perturbation v + delta.  The solver
(fwi_forward) produces both trace sets on the GPU; training runs the
library's BF16-MFMA forward/backward and Adam kernels (fwi_sur_train_step)
on the weighted trace loss plus the finite-difference term that fits the
surrogate's change S(v + delta) - S(v) to the solver's, which is what the
guidance gradient through the surrogate depends on.  The last 2% of the
pairs are held out and reported.  Acquisition: 70 x 70 grid, dx = 10 m,
5 surface shots, 70 receivers, 1000 samples at 1 ms, 15 Hz Ricker,
40-cell sponge.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch-pairs", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=1e-4)
    ap.add_argument("--loss-k", type=float, default=20.0)
    ap.add_argument("--pair-scale", type=float, default=1.0, help="pair weight relative to (rms d / rms delta d)^2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--ckpt", default=None, help="checkpoint written after every epoch (parameters, Adam state, "
                                                 "step, epoch, the batch-order generator's state)")
    ap.add_argument("--resume", action="store_true", help="continue from --ckpt")
    ap.add_argument("--stop-after-epoch", type=int, default=None)
    args = ap.parse_args(argv)

    import torch

    import fwi_inputs as fi
    from .fwi import FwiPlan
    from .surrogate import Surrogate, init_params

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    acq = fi.surface_acquisition(70, 70, ns=5, nt=1000, nb=40)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    NB = 64
    plan = FwiPlan(acq, max_batch=NB, device=dev)
    n = args.pairs
    t0 = time.time()
    V = np.empty((n, 70, 70), np.float32)
    V2 = np.empty_like(V)
    for i in range(n):
        a, b = fi.surrogate_training_pair(i)
        V[i], V2[i] = a, b
    log(f"generated {n} model pairs in {time.time() - t0:.1f} s")
    Vd, V2d = torch.tensor(V, device=dev), torch.tensor(V2, device=dev)
    D = torch.empty((n, 5, 70, 1000), dtype=torch.float32, device=dev)
    D2 = torch.empty_like(D)
    t0 = time.time()
    for i in range(0, n, NB):
        plan.forward(Vd[i:i + NB], w, keep_for_adjoint=False, out=D[i:i + NB])
        plan.forward(V2d[i:i + NB], w, keep_for_adjoint=False, out=D2[i:i + NB])
    torch.cuda.synchronize()
    if plan.status() != 0:
        raise RuntimeError("solver reported a device-side error")
    log(f"solver traces for {2 * n} models in {time.time() - t0:.1f} s")
    n_hold = max(16, n // 50)
    n_tr = n - n_hold
    rms = D[:n_tr].pow(2).mean().sqrt().item()
    drms = (D2[:n_tr] - D[:n_tr]).pow(2).mean().sqrt().item()
    lam = args.pair_scale * (rms / drms) ** 2
    log(f"trace rms {rms:.4e}, pair-difference rms {drms:.4e}, pair weight {lam:.2f}")

    bp = args.batch_pairs
    sur = Surrogate(2 * bp, device=dev)
    sur.set_params(init_params(args.seed, out_scale=rms))
    steps_per_epoch = n_tr // bp
    total = args.epochs * steps_per_epoch
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    loss = torch.zeros(1, device=dev)
    step = 0
    ep0 = 0
    if args.resume and args.ckpt and os.path.exists(args.ckpt):
        ck = np.load(args.ckpt)
        sur.set_params(ck["params"])
        sur.set_adam(ck["adam_m"], ck["adam_v"], int(ck["adam_step"]))
        step, ep0 = int(ck["step"]), int(ck["epoch"])
        gen.set_state(torch.from_numpy(ck["gen_state"]))
        log(f"resumed after epoch {ep0} (step {step})")
    t0 = time.time()
    for ep in range(ep0, args.epochs):
        perm = torch.randperm(n_tr, device=dev, generator=gen)
        acc = torch.zeros(1, device=dev)
        for j in range(steps_per_epoch):
            idx = perm[j * bp:(j + 1) * bp]
            vb = torch.cat([Vd[idx], V2d[idx]]).contiguous()
            db = torch.cat([D[idx], D2[idx]]).contiguous()
            lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1.0 + math.cos(math.pi * step / total))
            sur.train_step(vb, db, lr=lr, loss_k=args.loss_k, pair_weight=lam, loss_out=loss)
            acc += loss
            step += 1
        torch.cuda.synchronize()
        log(f"epoch {ep + 1}/{args.epochs}: loss / rms^2 {acc.item() / steps_per_epoch / rms ** 2:.4f} "
            f"({time.time() - t0:.0f} s)")
        if args.ckpt:
            m, v, astep = sur.get_adam()
            tmp = args.ckpt + ".tmp.npz"
            np.savez(tmp, params=sur.get_params(), adam_m=m, adam_v=v, adam_step=np.int64(astep),
                     step=np.int64(step), epoch=np.int64(ep + 1), gen_state=gen.get_state().numpy())
            os.replace(tmp, args.ckpt)
        if args.stop_after_epoch is not None and ep + 1 >= args.stop_after_epoch:
            log(f"stopped after epoch {ep + 1}")
            return 0
    # held-out pairs: trace error and finite-difference error
    te, de = [], []
    for i in range(n_tr, n, bp):
        j = min(n, i + bp)
        s1 = sur.forward(Vd[i:j].contiguous()).clone()
        s2 = sur.forward(V2d[i:j].contiguous())
        te.append(((s1 - D[i:j]).flatten(1).norm(dim=1) / D[i:j].flatten(1).norm(dim=1)).cpu())
        dd = D2[i:j] - D[i:j]
        de.append((((s2 - s1) - dd).flatten(1).norm(dim=1) / dd.flatten(1).norm(dim=1)).cpu())
    te, de = torch.cat(te), torch.cat(de)
    log(f"held-out {n_hold} pairs: trace rel L2 median {te.median().item():.4f}, "
        f"finite-difference rel L2 median {de.median().item():.4f}")
    np.save(args.out, sur.get_params())
    log(f"saved {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
