"""Train the score network by denoising score matching on the seeded prior.

    python -m paper_2603_16393_amd.train_score --steps 20000 --out weights/score_70x70.npy \\
        --ckpt score_ckpt.npz [--resume]

The prior stands in for the paper's training sets (Sec. 6: OpenFWI families,
unavailable here): fwi_inputs.prior_model draws faulted dipping-layer models
and flat-layer models (seeds 5,000,000 + i for the training pool, 6,000,000 +
i held out), normalised to the diffusion state in [-1, 1].  Each step draws
a batch from the pool, a step index i ~ U{1..N} and Gaussian noise per
sample, and runs the library's DSM step (fwi_score_train_step: x_i =
sqrt(abar_i) x0 + sqrt(1 - abar_i) z, loss = mean (eps_theta(x_i, i/N) - z)^2,
Adam), on the VP schedule of vp_schedule (N = 1000).

Checkpoints hold everything a resumed run needs: parameters, Adam moments and
step, the step counter, the numpy generator's state, the parameter average
(an exponential moving average, the weights that are saved) and the loss history;
--resume continues from --ckpt and reproduces the uninterrupted run.  At the
end the held-out DSM loss is reported per noise level beside the two trivial
predictors (z_hat = 0 and z_hat = x_i / sqrt(1 - abar_i)).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def pool_models(n: int, seed0: int) -> np.ndarray:
    import fwi_inputs as fi

    return np.stack([fi.to_normalised(fi.prior_model(seed0 + i)) for i in range(n)]).astype(np.float32)


def lr_at(step: int, total: int, lr: float, lr_min: float, warmup: int) -> float:
    if step < warmup:
        return lr * (step + 1) / warmup
    f = (step - warmup) / max(1, total - warmup)
    return lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * min(1.0, f)))


def save_ckpt(path, net, step, rng, losses, ema=None):
    m, v, astep = net.get_adam()
    tmp = path + ".tmp.npz"
    extra = {} if ema is None else {"ema": ema}
    np.savez(tmp, params=net.get_params(), adam_m=m, adam_v=v, adam_step=np.int64(astep), step=np.int64(step),
             rng_state=np.array(json.dumps(rng.bit_generator.state)), losses=np.asarray(losses, np.float32), **extra)
    os.replace(tmp, path)


def heldout_report(net, dev, n=256, levels=(20, 100, 300, 500, 700, 900), seed=6_000_000):
    """Held-out DSM loss per step index against the trivial predictors."""
    import torch

    from .score import vp_schedule

    _, abar = vp_schedule()
    X = torch.tensor(pool_models(n, seed), device=dev)
    rng = np.random.default_rng(123)
    out = {}
    B = net.max_batch
    for i in levels:
        ab = float(abar[i - 1])
        errs, base0, base1 = [], [], []
        for s in range(0, n, B):
            x0 = X[s:s + B]
            b = x0.shape[0]
            z = torch.tensor(rng.standard_normal((b, 70, 70)).astype(np.float32), device=dev)
            xi = (math.sqrt(ab) * x0 + math.sqrt(1 - ab) * z).contiguous()
            eps = net.forward(xi, torch.full((b,), i / 1000.0, device=dev))
            errs.append(float(((eps - z) ** 2).mean()))
            base0.append(float((z ** 2).mean()))
            base1.append(float(((xi / math.sqrt(1 - ab) - z) ** 2).mean()))
        out[i] = dict(net=float(np.mean(errs)), zero=float(np.mean(base0)), scaled_state=float(np.mean(base1)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--pool", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=5e-5)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ckpt", default=None, help="checkpoint file (written every --ckpt-every steps)")
    ap.add_argument("--ckpt-every", type=int, default=2000)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--stop-after", type=int, default=None, help="stop (after a checkpoint) at this step")
    ap.add_argument("--ema", type=float, default=0.999, help="decay per step of the parameter average kept on "
                                                            "the host (updated every 50 steps); 0 = off")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch

    from .score import ScoreNet, vp_schedule

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    net = ScoreNet(args.batch, device=dev)
    _, abar = vp_schedule()
    N = len(abar)
    t0 = time.time()
    pool = torch.tensor(pool_models(args.pool, 5_000_000), device=dev)
    log(f"pool of {args.pool} prior models in {time.time() - t0:.1f} s")
    rng = np.random.default_rng(args.seed)
    step, losses = 0, []
    ema = None
    if args.resume and args.ckpt and os.path.exists(args.ckpt):
        ck = np.load(args.ckpt)
        net.set_params(ck["params"])
        net.set_adam(ck["adam_m"], ck["adam_v"], int(ck["adam_step"]))
        step = int(ck["step"])
        rng.bit_generator.state = json.loads(str(ck["rng_state"]))
        losses = list(ck["losses"])
        if "ema" in ck.files:
            ema = ck["ema"].astype(np.float64)
        log(f"resumed at step {step}")
    else:
        net.set_params(init_params(args.seed))
    if args.ema > 0 and ema is None:
        ema = net.get_params().astype(np.float64)
    ema_decay = args.ema ** 50
    loss_t = torch.zeros(1, dtype=torch.float32, device=dev)
    B = args.batch
    t0 = time.time()
    loss_ema = None
    while step < args.steps:
        idx = rng.integers(0, args.pool, B)
        ti = rng.integers(1, N + 1, B)
        z = rng.standard_normal((B, 70, 70), dtype=np.float32)
        ab = abar[ti - 1]
        x0 = pool[torch.tensor(idx, device=dev)].contiguous()
        f = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)  # noqa: E731
        net.train_step(x0, f(z), f(ti / N), f(np.sqrt(ab)), f(np.sqrt(1 - ab)),
                       lr=lr_at(step, args.steps, args.lr, args.lr_min, args.warmup), loss_out=loss_t)
        step += 1
        if ema is not None and step % 50 == 0:
            ema = ema_decay * ema + (1.0 - ema_decay) * net.get_params()
        if step % 50 == 0:
            lv = float(loss_t.item())
            losses.append(lv)
            loss_ema = lv if loss_ema is None else 0.9 * loss_ema + 0.1 * lv
            if step % 1000 == 0:
                log(f"step {step}: DSM loss {lv:.4f} (running mean {loss_ema:.4f}), {time.time() - t0:.0f} s")
        if args.ckpt and (step % args.ckpt_every == 0 or step == args.steps):
            save_ckpt(args.ckpt, net, step, rng, losses, ema)
        if args.stop_after is not None and step >= args.stop_after:
            log(f"stopped at step {step}")
            break
    torch.cuda.synchronize()
    log(f"{step} steps in {time.time() - t0:.1f} s")
    if ema is not None:
        net.set_params(ema.astype(np.float32))   # evaluate and save the averaged parameters
    rep = heldout_report(net, dev)
    for i, r in rep.items():
        log(f"held-out i={i}: net {r['net']:.5f}  zero {r['zero']:.5f}  x_i/sqrt(1-abar) {r['scaled_state']:.5f}")
    if args.out and step >= args.steps:
        np.save(args.out, net.get_params())
        log(f"wrote {args.out}" + (" (parameter average)" if ema is not None else ""))

    net.close()


def init_params(seed: int) -> np.ndarray:
    """He-style initial parameters in the library's layout (biases zero, residual branches and head small)."""
    from ._lib import load

    n = int(load().fwi_score_param_count())
    rng = np.random.default_rng(seed)
    out = np.zeros(n, np.float32)
    # the layout of include/fwi.h, in order: (size, fan_in or 0 for a bias, scale)
    C0, C1, C2, NF, TH, NTB = 32, 64, 128, 16, 128, 320
    parts = [(2 * NF * TH, 2 * NF, 1.0), (TH, 0, 0), (TH * NTB, TH, 0.1), (NTB, 0, 0), (3 * C0, 3, 1.0), (C0, 0, 0)]

    def blk(c):
        return [(9 * c * c, 9 * c, 1.0), (c, 0, 0), (9 * c * c, 9 * c, 0.1), (c, 0, 0)]

    parts += blk(C0) + [(C0 * C1, C0, 1.0), (C1, 0, 0)] + blk(C1) + [(C1 * C2, C1, 1.0), (C2, 0, 0)]
    parts += blk(C2) + [(C2 * C1, C2, 1.0), (C1, 0, 0)] + blk(C1) + [(C1 * C0, C1, 1.0), (C0, 0, 0)]
    parts += blk(C0) + [(C0, C0, 0.1), (1, 0, 0)]
    o = 0
    for size, fan, sc in parts:
        if fan:
            out[o:o + size] = rng.standard_normal(size) * math.sqrt(2.0 / fan) * sc
        o += size
    assert o == n
    return out


if __name__ == "__main__":
    main()
