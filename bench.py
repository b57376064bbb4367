"""Guidance-gradient throughput on one MI355X.

Workload: batch of 16 denoised estimates v0hat (seeded layered/faulted 70 x 70
models, dx = 10 m, 1500-4500 m/s), 5 surface shots x 70 receivers, 1000 time
samples at dt = 1 ms, 15 Hz Ricker, 40-cell sponge, reflecting top.  One step
is the whole guidance path for the batch: forward modelling with the history
kept, W2 misfit and adjoint source, adjoint gradient, preconditioned update.
Observations are synthesised once from a seeded "true" model before timing;
inputs are resident in HBM when the timed region starts.

Prints one JSON line (see the keys below).  --gpus > 1 is refused: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NZ = NX = 70
NS, NT, NB, B = 5, 1000, 40, 16
HBM_PEAK_GBS = 8000.0


def make_inputs():
    import fwi_inputs as fi

    acq = fi.surface_acquisition(NZ, NX, ns=NS, nt=NT, nb=NB)
    v0hat = np.stack([fi.faulted_model(NZ, NX, s) for s in range(B)])
    v_true = fi.faulted_model(NZ, NX, 1000)
    w = fi.ricker(NT, acq.dt, acq.f_peak)
    return acq, v0hat, v_true, w


def host_cpu():
    """CPU model name and the cores this process may use (the oracle's OpenMP threads)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc or 1))
    return {"cpu_model": model, "nproc": nproc, "omp_threads": threads}


def _median3(fn):
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), [round(t, 3) for t in ts]


def cpu_baseline(acq, v0hat, v_true, w, n_samples=4):
    """The FP64 oracle, as it stands, on bounded samples of the four workloads (median of 3 runs each): the
    headline batch (n_samples of its 16 samples), the one-shot 70 x 70 experiment, the 400 x 800 checkpointed
    gradient (one shot, the first 40 of its 4000 steps, with the oracle's own checkpointing) and the uneven batch
    (one shot of one request per grid size, the first 80 steps).  `value` is the headline leg."""
    import oracle

    import fwi_inputs as fi

    host = host_cpu()
    threads = host["omp_threads"]
    legs = {}
    # headline batch
    obs = oracle.w2_prepare(oracle.forward(acq, v_true, w), acq.dt)
    x0 = fi.to_normalised(v0hat[:n_samples])

    def head():
        J, g, _, _ = oracle.objective_and_gradient(acq, v0hat[:n_samples], w, obs)
        oracle.guidance(x0, g, g, x0, unit_scale=1500.0)

    dt, runs = _median3(head)
    nzp, nxp = acq.padded_shape
    pts = 2.0 * n_samples * NS * (NT - 1) * nzp * nxp
    legs["guidance_b16_70x70"] = {"grads_per_s": round(n_samples / dt, 4), "gpts_per_s": round(pts / dt / 1e9, 4),
                                  "seconds": runs, "cores": min(threads, n_samples * NS),
                                  "sample": f"{n_samples} of the {B} samples ({n_samples * NS} shot units)"}
    # one-shot experiment
    a0 = fi.surface_acquisition(NZ, NX, ns=1, shot_cols=[35], nt=NT, nb=NB)
    v0 = fi.layered_model(NZ, NX, 0)
    obs0 = oracle.w2_prepare(oracle.forward(a0, fi.blob_perturbation(v0, 1)[None], w)[0], a0.dt)
    dt, runs = _median3(lambda: oracle.objective_and_gradient(a0, v0[None], w, obs0))
    legs["one_shot_70x70"] = {"grads_per_s": round(1.0 / dt, 4),
                              "gpts_per_s": round(2.0 * (NT - 1) * nzp * nxp / dt / 1e9, 4), "seconds": runs,
                              "cores": 1, "sample": "the whole experiment (1 sample, 1 shot, 1000 steps)"}
    # checkpointed 400 x 800
    nt2 = 40
    a2 = fi.surface_acquisition(400, 800, ns=1, shot_cols=[400], nt=nt2, nb=50, dt=8e-4, f_peak=10.0, v_max=5000.0)
    v2 = fi.large_lens_model()
    w2 = fi.ricker(nt2, 8e-4, 10.0)
    obs2 = oracle.w2_prepare(oracle.forward(a2, v2[None], w2)[0], a2.dt)
    v2p = np.clip(v2 * 1.01, 1500.0, 5000.0)[None]
    dt, runs = _median3(lambda: oracle.objective_and_gradient(a2, v2p, w2, obs2))
    npts2 = 450 * 900
    scale = (3999.0 / (nt2 - 1)) * 20
    legs["checkpointed_400x800"] = {"gpts_per_s": round(2.0 * (nt2 - 1) * npts2 / dt / 1e9, 4), "seconds": runs,
                                    "cores": 1, "est_s_per_gradient": round(dt * scale, 1),
                                    "sample": f"1 of 20 shots, the first {nt2} of 4000 steps (gradient with the "
                                              f"oracle's checkpointing); a full gradient scaled by {scale:.0f}"}
    # uneven batch
    reqs = fi.uneven_requests()
    picked = {}
    for a, v, wv in reqs:
        if a.nz not in picked:
            picked[a.nz] = (a, v, wv)
    nt3 = 80
    units = []
    for n_, (a, v, wv) in sorted(picked.items()):
        au = dataclass_replace(a.subset_shots([0]), nt=nt3)
        wu = wv[:nt3]
        units.append((au, v, wu, oracle.w2_prepare(oracle.forward(au, v[None], wu)[0], au.dt)))
    pts3 = sum(2.0 * (nt3 - 1) * (u[0].padded_shape[0] * u[0].padded_shape[1]) for u in units)

    def uneven():
        for au, v, wu, ob in units:
            oracle.objective_and_gradient(au, np.clip(v * 1.01, 1500.0, 4500.0)[None], wu, ob)

    dt, runs = _median3(uneven)
    legs["uneven_70_140_256"] = {"gpts_per_s": round(pts3 / dt / 1e9, 4), "seconds": runs, "cores": 1,
                                 "sample": f"one shot of one request per grid size ({', '.join(str(k) for k in sorted(picked))}), "
                                           f"the first {nt3} steps, forward + W2 + gradient"}
    h = legs["guidance_b16_70x70"]
    return {
        "value": h["grads_per_s"],
        "unit": "grads/s",
        "cores": h["cores"],
        "kind": "oracle",
        "sample": f"{n_samples} of the {B} samples ({n_samples * NS} shot units), same grid/steps; forward + W2 + "
                  f"reverse-mode gradient + guidance update in FP64, median of 3 runs {h['seconds']} s",
        "gpts_per_s": h["gpts_per_s"],
        "host": host,
        "legs": legs,
        "single_core": cpu_baseline_one_core(),
    }


def dataclass_replace(obj, **kw):
    import dataclasses

    return dataclasses.replace(obj, **kw)


def cpu_baseline_one_core():
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1, no GPU use): forward + W2 + gradient of
    one shot unit of sample 0, scaled to grads/s (a gradient is NS units)."""
    import subprocess

    code = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import bench, oracle\n"
        "acq, v0hat, v_true, w = bench.make_inputs()\n"
        "a1 = acq.subset_shots([0])\n"
        "obs = oracle.w2_prepare(oracle.forward(a1, v_true, w), a1.dt)\n"
        "t0 = time.perf_counter()\n"
        "oracle.objective_and_gradient(a1, v0hat[:1], w, obs)\n"
        "print(json.dumps(time.perf_counter() - t0))\n" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return None
    dt = float(r.stdout.strip().splitlines()[-1])
    nzp, nxp = NZ + NB, NX + 2 * NB
    return {"value": round(1.0 / (NS * dt), 4), "unit": "grads/s", "cores": 1,
            "gpts_per_s": round(2.0 * (NT - 1) * nzp * nxp / dt / 1e9, 4),
            "sample": f"1 shot unit of sample 0 on one thread, {dt:.2f} s, scaled by {NS} units per gradient"}


# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by what the same counter reads
# for the library's plain copy kernel in the same run (profiles/*_hbm_traffic.md).  A figure holds only while the
# sources of its kernel are the ones the counters were taken on (SHA-1 over the listed files); otherwise None.
CSRC = "paper_2603_16393_amd/csrc/"
MEASURED_TRAFFIC = {
    # split LDS-resident sweep of the default workload (profiles/k_wave_split_b16_70x70_hbm_traffic.md)
    "split": {"sources": (CSRC + "wave_lds.hip", CSRC + "wave_lds_body.h", CSRC + "wave_split_body.h"),
              "sha1": "e0d5113fc72f665f11f56be04632f7df5c4f9750", "bytes": {"forward": 9.0976e9, "adjoint": 8.5382e9}},
    # PML row bands (profiles/k_wave_pml_b16_70x70_hbm_traffic.md)
    "pml": {"sources": (CSRC + "wave_pml.hip", CSRC + "pml_stencil.h", CSRC + "wave_split_body.h"),
            "sha1": "b81ad6386bd6265bd3c4f2f4f6a6209533ab3a71",
            "bytes": {"forward": 4.2920e9, "adjoint": 4.3224e9}},
    # two-step tiled sweep of the 400 x 800 workload, per launch (profiles/k_wave_tile2_ckpt_400x800_hbm_traffic.md):
    # forward launch u, w, K read and u, w written; a recomputation launch also writes its two D slices
    "tile2": {"sources": (CSRC + "wave.hip",), "sha1": "0b5141fee21e1db97a56bc6319161c3e02d43582",
              "bytes": {"forward": 9.922e7 + 6.48e7, "recompute": 9.922e7 + 2 * 6.48e7, "adjoint": 2.976e8}},
    # HBM-swept PML, per launch of the 400 x 800 checkpointed workload
    # (profiles/k_pml_hbm_tile_ckpt_400x800_hbm_traffic.md): recomputation (D written) and adjoint
    "pml_hbm": {"sources": (CSRC + "wave_pml_hbm.hip", CSRC + "pml_stencil.h"), "sha1": "67081226c82d5c5b73b66944a505dd0547996631",
                "bytes": {"recompute": 1.680e8, "adjoint": 2.274e8}},
    # uneven persistent forward launch of the 64-request mix (profiles/k_batch_uneven64_hbm_traffic.md)
    "uneven": {"sources": (CSRC + "batch.hip", CSRC + "wave_lds_body.h", CSRC + "wave_split_body.h"),
               "sha1": "4c3b6de45e11beecd404a54bb1784f4e26cd9fa3", "bytes": {"forward": 1.2338e11, "gradient": 6.1162e11}},
}


def measured_traffic(name, kind):
    t = MEASURED_TRAFFIC[name]
    if t["sha1"] is None or t["bytes"].get(kind) is None:
        return None
    h = hashlib.sha1()
    for f in t["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return t["bytes"][kind] if h.hexdigest() == t["sha1"] else None


SURROGATE_WEIGHTS = os.path.join(ROOT, "paper_2603_16393_amd", "weights", "surrogate_70x70.npy")
GUIDED_STEPS = 200
# the judge's cosine threshold: it sees only the farthest prediction of an interval, so it judges with a margin
# over the 0.95 the served gradients are held to
JUDGE_COS = 0.97


def guided_run(plan, wt, v_true, sur, predictor, steps=GUIDED_STEPS, record=False, cos_min=0.95):
    """16 samples x `steps` reverse steps, t from 1 down to 0.005; the clean
    estimates come from the stand-in denoiser v0hat = clip(v_true + t zeta_b).
    Each step: guidance gradient (solver, or judged prediction above t = 0.5)
    and the preconditioned update.  Returns (seconds, stats, served) where
    served lists (step, gradient copy) for predicted steps when record=True."""
    import torch

    import fwi_inputs as fi
    from paper_2603_16393_amd import guidance_step
    from paper_2603_16393_amd.guided import GuidanceGradients

    dev = plan.device
    zeta = torch.tensor(np.stack([fi.stand_in_zeta(NZ, NX, b) for b in range(B)]), dtype=torch.float32, device=dev)
    vt = torch.tensor(v_true, dtype=torch.float32, device=dev)
    ts = np.linspace(1.0, 0.005, steps)
    src = GuidanceGradients(plan, wt, B, surrogate=sur, predictor=predictor, cos_min=cos_min)
    v = torch.empty((B, NZ, NX), dtype=torch.float32, device=dev)
    x0 = torch.empty_like(v)
    vn = torch.empty_like(v)
    rho = torch.empty(B, dtype=torch.float32, device=dev)
    served = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, t in enumerate(ts):
        torch.clamp(vt + float(t) * zeta, fi.V_LO, fi.V_HI, out=v)   # stand-in denoiser output
        n_pred = src.stats.served_predicted
        J, g = src(float(t), v)
        torch.sub(v, fi.V_LO, out=x0).div_(0.5 * (fi.V_HI - fi.V_LO)).sub_(1.0)
        guidance_step(x0, g, g, x0, unit_scale=1500.0, out=vn, rho_out=rho)
        if record and src.stats.served_predicted > n_pred:
            served.append((i, g.clone()))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, src.stats, served


def surrogate_guidance(plan, wt, v_true):
    """Plain solver guidance vs judged surrogate-assisted guidance (and the same
    schedule without the network) over 16 x 200 steps; the served predicted
    gradients are checked against the solver afterwards (untimed)."""
    import torch

    import fwi_inputs as fi
    from paper_2603_16393_amd.surrogate import Surrogate, judge

    if not os.path.exists(SURROGATE_WEIGHTS):
        return {"error": f"no trained weights at {os.path.relpath(SURROGATE_WEIGHTS, ROOT)}"}
    sur = Surrogate(B, device=plan.device)
    sur.set_params(np.load(SURROGATE_WEIGHTS))
    guided_run(plan, wt, v_true, None, "surrogate", steps=8)           # warm-up
    guided_run(plan, wt, v_true, sur, "surrogate", steps=8)
    t_plain, _, _ = guided_run(plan, wt, v_true, None, "surrogate")
    res = {"plain_steps_per_s": round(B * GUIDED_STEPS / t_plain, 2)}
    dev = plan.device
    zeta = torch.tensor(np.stack([fi.stand_in_zeta(NZ, NX, b) for b in range(B)]), dtype=torch.float32, device=dev)
    vt = torch.tensor(v_true, dtype=torch.float32, device=dev)
    ts = np.linspace(1.0, 0.005, GUIDED_STEPS)
    g_ex = torch.empty((B, NZ, NX), dtype=torch.float32, device=dev)
    for name, pred, net, cmin in (("surrogate", "surrogate", sur, JUDGE_COS), ("anchor_only", "anchor", None, JUDGE_COS),
                                  ("surrogate_judge095", "surrogate", sur, 0.95),
                                  ("anchor_only_judge095", "anchor", None, 0.95)):
        t_run, st, _ = guided_run(plan, wt, v_true, net, pred, cos_min=cmin)
        _, _, served = guided_run(plan, wt, v_true, net, pred, record=True, cos_min=cmin)   # same schedule, checked
        cos_all = []
        for i, g in served:
            v = torch.clamp(vt + float(ts[i]) * zeta, fi.V_LO, fi.V_HI)
            d = plan.forward(v, wt, keep_for_adjoint=True)
            _, adj = plan.w2_misfit(d, want_adjoint=True)
            plan.adjoint_gradient(v, adj, out=g_ex)
            cos_all += judge(g, g_ex)[0].tolist()
        c = np.array(cos_all) if cos_all else np.ones(1)
        res[name] = {
            "steps_per_s": round(B * GUIDED_STEPS / t_run, 2),
            "speedup_vs_plain": round(t_plain / t_run, 3),
            "solver_batches": st.exact_batches,
            "surrogate_batches": st.surrogate_batches,
            "predicted_steps": st.served_predicted,
            "judged": st.judged,
            "judge_passed": st.passed,
            "served_cos": {"min": round(float(c.min()), 4), "p1": round(float(np.percentile(c, 1)), 4),
                           "p5": round(float(np.percentile(c, 5)), 4), "median": round(float(np.median(c)), 4),
                           "frac_ge_0.95": round(float(np.mean(c >= 0.95)), 4), "n": int(c.size)},
            "judged_misfit_error_median": round(float(np.median(st.judge_jerr)), 4) if st.judge_jerr else None,
        }
    res["protocol"] = (f"{B} samples x {GUIDED_STEPS} steps, t = 1 -> 0.005; stand-in denoiser clip(v_true + t zeta_b); "
                       f"t > 0.5: anchor + surrogate change, solver judge (cos >= {JUDGE_COS}, misfit error <= 5%) "
                       "with an adaptive interval (4, x2 on pass up to 32, /2 on fail); t <= 0.5: solver; served "
                       "gradients checked against the solver afterwards at cos >= 0.95 (the judge's margin keeps the "
                       "served steps inside an interval, which lie closer to the anchor than the judged one, above "
                       "0.95); the *_judge095 entries judge at 0.95")
    sur.close()
    return res


SCORE_WEIGHTS = os.path.join(ROOT, "paper_2603_16393_amd", "weights", "score_70x70.npy")
REVERSE_STEPS = 100
# the paper's rho0 = 1.15 (Table 'parameter', CurveVel-A) per step of a 1000-step chain, times the 10 chain steps
# that each of the 100 respaced steps stands for
REVERSE_RHO0 = 11.5


def reverse_loop(plan, wt, v_true):
    """Algorithm 2 end to end on the batch: 16 samples x 100 respaced reverse steps from seeded noise, each step
    the trained score network's clean estimate (Eq. v0hat), the DDPM posterior mean plus noise, the guidance
    gradient g (forward, W2 misfit, adjoint) at the clean estimate, its chain rule through the network h =
    (d v0hat / d x_i)^T g (Eq. chain_rule, so h != g) and the preconditioned update.  Steps/s counts one step of
    one sample; the unguided loop (network and DDPM step only) is timed beside it, and the final samples' misfit
    and distance to the true model are reported for both."""
    import torch

    from paper_2603_16393_amd.diffusion import ReverseLoop
    from paper_2603_16393_amd.score import ScoreNet

    if not os.path.exists(SCORE_WEIGHTS):
        return {"error": f"no trained weights at {os.path.relpath(SCORE_WEIGHTS, ROOT)}"}
    dev = plan.device
    net = ScoreNet(B, device=dev)
    net.set_params(np.load(SCORE_WEIGHTS))
    x = torch.tensor(np.random.default_rng(11).standard_normal((B, NZ, NX)).astype(np.float32), device=dev)
    vt = torch.tensor(v_true, dtype=torch.float32, device=dev)
    res = {}
    for name, pl in (("guided", plan), ("unguided", None)):
        loop = ReverseLoop(net, B, REVERSE_STEPS, plan=pl, wavelet=wt, guidance=dict(rho0=REVERSE_RHO0))
        z = loop.step_noise(12)
        loop.run(x, noise=z[:, :, :, :])            # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs = loop.run(x, noise=z)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        v = ((xs.clamp(-1, 1) + 1) * 1500 + 1500).contiguous()
        d = plan.forward(v, wt, keep_for_adjoint=False)
        J, _ = plan.w2_misfit(d, want_adjoint=False)
        e = torch.linalg.vector_norm((v - vt).reshape(B, -1), dim=1) / torch.linalg.vector_norm(vt)
        res[name] = {"steps_per_s": round(B * REVERSE_STEPS / dt, 2), "ms_per_step": round(1e3 * dt / REVERSE_STEPS, 4),
                     "median_J": round(float(J.median()), 5), "median_e_l2": round(float(e.median()), 4)}
    # network forward and VJP per batch of 16 (HIP events on the stream they run on)
    loop = ReverseLoop(net, B, REVERSE_STEPS, plan=plan, wavelet=wt)
    c = loop._coef[REVERSE_STEPS // 2]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    g = torch.randn((B, NZ, NX), device=dev) * 1e-6
    fw = bw = 0.0
    for _ in range(20):
        ev[0].record()
        net.forward(x, c["t"], c["skip"], c["scale"], out=loop.v0)
        ev[1].record()
        net.backward(g, dx=loop.h)
        ev[2].record()
        torch.cuda.synchronize()
        fw += ev[0].elapsed_time(ev[1])
        bw += ev[1].elapsed_time(ev[2])
    res["network_ms_per_batch"] = {"forward": round(fw / 20, 4), "vjp": round(bw / 20, 4)}
    res["protocol"] = (f"{B} samples x {REVERSE_STEPS} respaced DDPM steps of the VP schedule (N = 1000), seeded "
                       "noise; trained score network (weights/score_70x70.npy); guidance: W2 misfit of the "
                       "5-shot workload's observations of the true model, preconditioner rho0 = 11.5 (1.15 per step "
                       "of the 1000-step chain), gamma = 0.55")
    net.close()
    return res


def comparison_variants(plan, acq, wt, dobs, v, x0, steps=10, warmup=2):
    """Whole guidance steps of the comparison and ablation variants on the same batch:
    baseline DPS with the least-squares potential (Algorithm 1, sigma = 0.05, scalar step), its MSE-All
    ablation form (amplitude weight k = 100, misfit-scale normalisation, preconditioned step), and the
    TV-regularised descent baselines W2+TV (raw-trace squared W2, fixed step) and OT-WE+TV (enhanced
    W2, preconditioned step).  Each: forward, misfit, adjoint gradient, [TV subgradient,] update."""
    import torch

    from paper_2603_16393_amd import FwiPlan, guidance_step, tv_subgradient

    dev = plan.device
    plan_raw = FwiPlan(acq, max_batch=B, device=dev)
    plan_raw.set_obs(dobs, k=0.0, squared=True)
    d = torch.empty((B, NS, acq.nr, NT), dtype=torch.float32, device=dev)
    J = torch.empty(B, dtype=torch.float64, device=dev)
    adj = torch.empty_like(d)
    g = torch.empty((B, NZ, NX), dtype=torch.float32, device=dev)
    h = torch.empty_like(g)
    xn = torch.empty_like(g)
    rho = torch.empty(B, dtype=torch.float32, device=dev)
    alpha = 1e-6  # TV weight per m/s of gradient (a fixed setting for timing)

    def lsq(kw, precond):
        def step():
            plan.forward(v, wt, keep_for_adjoint=True, out=d)
            plan.l2_misfit(d, dobs, J_out=J, adj_out=adj, **kw)
            plan.adjoint_gradient(v, adj, out=g)
            extra = {} if precond else dict(gamma=0.0, tau=1e30)
            guidance_step(x0, g, g, x0, unit_scale=1500.0, out=xn, rho_out=rho, **extra)
        return step

    def tv(p, precond):
        def step():
            p.forward(v, wt, keep_for_adjoint=True, out=d)
            p.w2_misfit(d, want_adjoint=True, J_out=J, adj_out=adj)
            p.adjoint_gradient(v, adj, out=g)
            tv_subgradient(v, g, alpha, out=h)
            extra = {} if precond else dict(gamma=0.0, tau=1e30)
            guidance_step(x0, h, g, x0, unit_scale=1500.0, out=xn, rho_out=rho, **extra)
        return step

    variants = {
        "dps_l2": lsq(dict(sigma=0.05), False),
        "mse_all": lsq(dict(sigma=1.0, k=100.0, normalize=True), True),
        "w2_tv": tv(plan_raw, False),
        "ot_we_tv": tv(plan, True),
    }
    res = {}
    for name, step in variants.items():
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"grads_per_s": round(B / (ms / 1e3), 2), "ms_per_step": round(ms, 4)}
    ok = plan.status() == 0 and plan_raw.status() == 0
    plan_raw.close()
    if not ok:
        return {"error": "device-side check failed"}
    res["protocol"] = (f"{B} samples x one step each, {steps} timed steps after {warmup} warm-up: forward, misfit "
                       "(least squares or W2), adjoint gradient, [TV subgradient,] update; same batch and "
                       "observations as the plain line")
    return res


def perturbed_operators(v0hat, v_true, x0, steps=5, warmup=1):
    """The plain guidance step (forward, W2, adjoint gradient, update) of the same 16 models under the
    forward-operator configurations of the robustness study and the anisotropic Marmousi2-crop grids
    (fwi_inputs.operator_acquisition): grads/s of each."""
    import torch

    import fwi_inputs as fi
    from paper_2603_16393_amd import FwiPlan, guidance_step

    dev = torch.device("cuda:0")
    v = torch.tensor(v0hat, dtype=torch.float32, device=dev)
    res = {}
    for name in fi.OPERATORS:
        acq = fi.operator_acquisition(name)
        w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
        plan = FwiPlan(acq, max_batch=B, device=dev)
        dobs = plan.forward(torch.tensor(v_true[None], dtype=torch.float32, device=dev), w, keep_for_adjoint=False)
        plan.set_obs(dobs[0].contiguous())
        d = torch.empty((B, acq.ns, acq.nr, acq.nt), dtype=torch.float32, device=dev)
        J = torch.empty(B, dtype=torch.float64, device=dev)
        adj = torch.empty_like(d)
        g = torch.empty_like(v)
        xn = torch.empty_like(v)

        def step():
            plan.forward(v, w, keep_for_adjoint=True, out=d)
            plan.w2_misfit(d, want_adjoint=True, J_out=J, adj_out=adj)
            plan.adjoint_gradient(v, adj, out=g)
            guidance_step(x0, g, g, x0, unit_scale=1500.0, out=xn)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ok = plan.status() == 0
        info = dict(plan.info)
        plan.close()
        res[name] = {"grads_per_s": round(B / (ms / 1e3), 2) if ok else None, "ms_per_step": round(ms, 3),
                     "shots": acq.ns, "samples": acq.nt, "f_peak": acq.f_peak, "dz": acq.dz, "dx": round(acq.dx, 4),
                     "dt": acq.dt, "src_row": int(acq.src_iz[0]), "lds_split": info.get("lds_split")}
        print(f"operator {name}: {ms:.2f} ms per batch of {B}", file=sys.stderr, flush=True)
    res["protocol"] = (f"{B} faulted 70x70 models, 40-cell sponge, W2 misfit (k = 100); {steps} timed steps after "
                       f"{warmup} warm-up per configuration")
    return res


def pml_guidance(acq, v0hat, v_true, x0, w, steps=10, warmup=2):
    """The plain guidance step on the same batch and shots with the paper's absorbing layer: a 6-cell PML on
    the left, right and bottom (Sec. 6.1) in place of the 40-cell sponge, i.e. a 76 x 82 padded grid; the
    observations are that operator's own traces of v_true.  Reports grads/s, the per-sweep times of the
    LDS-resident PML kernels (HIP events on the plan's stream) and the adjoint sweep's roofline on
    algorithmic bytes: per field and step 16 B per padded point (u^n, u^{n-1}, (v dt)^2 in, u^{n+1} out),
    16 B per layer point (the two auxiliary fields in and out) and 4 B per padded point of the D history."""
    import dataclasses

    import torch

    from paper_2603_16393_amd import FwiPlan, guidance_step

    dev = torch.device("cuda:0")
    pacq = dataclasses.replace(acq, nb=6, pml=True)
    plan = FwiPlan(pacq, max_batch=B, device=dev, timing=True)
    wt = torch.tensor(w, dtype=torch.float32, device=dev)
    dobs = plan.forward(torch.tensor(v_true[None], dtype=torch.float32, device=dev), wt, keep_for_adjoint=False)
    plan.set_obs(dobs[0].contiguous())
    v = torch.tensor(v0hat, dtype=torch.float32, device=dev)
    d = torch.empty((B, pacq.ns, pacq.nr, pacq.nt), dtype=torch.float32, device=dev)
    J = torch.empty(B, dtype=torch.float64, device=dev)
    adj = torch.empty_like(d)
    g = torch.empty_like(v)
    xn = torch.empty_like(v)

    def step():
        plan.forward(v, wt, keep_for_adjoint=True, out=d)
        plan.w2_misfit(d, want_adjoint=True, J_out=J, adj_out=adj)
        plan.adjoint_gradient(v, adj, out=g)
        guidance_step(x0, g, g, x0, unit_scale=1500.0, out=xn)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.sweep_ms()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fwd_ms, adj_ms = plan.sweep_ms()
    ok = plan.status() == 0
    info = dict(plan.info)
    plan.close()
    nzp, nxp = info["nzp"], info["nxp"]
    npts, nlayer = nzp * nxp, nzp * nxp - pacq.nz * pacq.nx
    alg = float(B * pacq.ns * (pacq.nt - 1) * (16 * npts + 16 * nlayer + 4 * npts))
    achieved = alg / (adj_ms / 1e3) / 1e9
    print(f"PML6: {ms:.2f} ms per batch of {B} (forward sweep {fwd_ms:.2f} ms, adjoint {adj_ms:.2f} ms)",
          file=sys.stderr, flush=True)
    return {"grads_per_s": round(B / (ms / 1e3), 2) if ok else None, "ms_per_step": round(ms, 3),
            "padded": [nzp, nxp], "path": info["path"], "bands": info["lds_split"],
            "sweep_ms": {"forward": round(fwd_ms, 3), "adjoint": round(adj_ms, 3)},
            "roofline": {"bound": "hbm",
                         "kernel": ("k_wave_pml_band<adjoint> (row bands)" if info["lds_split"] > 1
                                    else "k_wave_pml<7, adjoint>"),
                         "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic("pml", "adjoint"), "alg_bytes_per_launch": alg,
                         "launch_ms": round(adj_ms, 3)},
            "protocol": f"same {B} models, shots and observations source as the plain line; 6-cell PML, W2 misfit "
                        f"(k = 100); {steps} timed steps after {warmup} warm-up"}


def copy_rate_gbps(dev, nbytes=1 << 30, reps=5):
    """Measured copy bandwidth of the library's plain copy kernel (fwi_copy, read + write counted), the
    practical HBM ceiling beside the published peak: median over `reps` copies of `nbytes`, HIP events."""
    import torch

    from paper_2603_16393_amd import _lib

    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = _lib.load()
    ms = []
    for i in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.check(L.fwi_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, st),
                   "fwi_copy")
        e1.record()
        torch.cuda.synchronize()
        if i:
            ms.append(e0.elapsed_time(e1))
    del src, dst
    return 2.0 * nbytes / (float(np.median(ms)) / 1e3) / 1e9


def ddpm_step_us(dev, v, reps=200):
    """Mean device time of fwi_ddpm_step over the batch (score and noise given), HIP events over `reps` calls."""
    import torch

    from paper_2603_16393_amd import ddpm_step

    s, z, x0, out = torch.randn_like(v), torch.randn_like(v), torch.empty_like(v), torch.empty_like(v)
    ddpm_step(v, 0.01, 0.5, 0.505, score=s, v0hat=x0, z=z, sigma=0.1, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ddpm_step(v, 0.01, 0.5, 0.505, score=s, v0hat=x0, z=z, sigma=0.1, out=out)
    e1.record()
    torch.cuda.synchronize()
    return round(1e3 * e0.elapsed_time(e1) / reps, 2)


def copy_calibration(dev):
    """Three dispatches of the library's plain copy kernel on 512 MiB, whose counter readings scale
    FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch

    from paper_2603_16393_amd import _lib

    nbytes = 512 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        _lib.check(_lib.load().fwi_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "fwi_copy")
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    del src, dst
    print(f"copy calibration: 3 x {nbytes} bytes", file=sys.stderr)


def bench_pml(args):
    """The plain guidance step of the default batch with the 6-cell PML alone (the `pml` field of the default
    run), as its own JSON line; with --copy-calibration the copy kernel runs first (counter passes)."""
    import torch

    import fwi_inputs as fi

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    acq, v0hat, v_true, w = make_inputs()
    x0 = torch.tensor(fi.to_normalised(v0hat), dtype=torch.float32, device=dev)
    if args.copy_calibration:
        copy_calibration(dev)
    r = pml_guidance(acq, v0hat, v_true, x0, w, steps=args.steps, warmup=args.warmup)
    print(json.dumps({
        "metric": "guidance grads/s (70x70, 5 shots, 1k steps, 6-cell PML)", "value": r["grads_per_s"],
        "unit": "grads/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain guidance, 16 x 70x70, 5 shots, 1000 steps, 6-cell PML", "global_batch": B},
        "roofline": r["roofline"], "sweep_ms": r["sweep_ms"], "bands": r["bands"]}))


# work-unit kinds of the uneven batch: whole field in one workgroup's LDS, HBM-swept field (gradient batches),
# LDS-resident row bands over several workgroups (forward batches)
UNIT_KIND = {0: "lds", 1: "hbm", 2: "bands"}
# HBM bytes per forward launch of the 64-request mix from FETCH_SIZE and WRITE_SIZE (None until measured for the
# current batch kernel)


def bench_uneven(args):
    """64 requests (seeds 2000 + r): 70x70 / 140x140 / 256x256 grids with a 40-cell sponge, 1000 / 1500 / 2500
    samples at dt = 1 ms, 5-10 surface shots, faulted or layered models in 1500-4500 m/s; forward modelling of
    every (request, shot) field in one persistent launch with autotuned tiles.  Per-size rates come from
    launches of the same kernel over each size class alone; "gradient" times dJ/dv of the whole batch for given
    adjoint sources (its forward_gpts_per_s counts the forward point-updates only)."""
    import torch

    import fwi_inputs as fi
    from paper_2603_16393_amd.batch import FwiBatch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        copy_calibration(dev)
    reqs = fi.uneven_requests()

    def run(sel, reps):
        t0 = time.perf_counter()
        b = FwiBatch([reqs[r][0] for r in sel], autotune=True, device=dev)
        t_create = time.perf_counter() - t0
        v = b.pack_velocity([reqs[r][1] for r in sel])
        w = b.pack_wavelets([reqs[r][2] for r in sel])
        tr = b.forward(v, w)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.forward(v, w, out=tr)
        e1.record()
        torch.cuda.synchronize()
        if b.status() != 0:
            print("device-side check failed", file=sys.stderr)
            sys.exit(1)
        ms = e0.elapsed_time(e1) / reps
        upd = sum(reqs[r][0].ns * (reqs[r][0].nt - 1) * (reqs[r][0].nz + reqs[r][0].nb) *
                  (reqs[r][0].nx + 2 * reqs[r][0].nb) for r in sel)
        tiles = sorted({(b.info[i]["nzp"], b.info[i]["nxp"], b.info[i]["kind"], b.info[i]["tile_x"],
                         b.info[i]["tile_z"], b.info[i]["parts"]) for i in range(len(sel))})
        b.close()
        return ms, upd, t_create, tiles

    reps = max(1, args.steps)
    ms, upd, t_create, tiles = run(list(range(len(reqs))), reps)
    gpts = upd / (ms / 1e3) / 1e9
    per_size = {}
    for size in (70, 140, 256):
        sel = [r for r in range(len(reqs)) if reqs[r][0].nz == size]
        m2, u2, _, _ = run(sel, reps)
        g2 = u2 / (m2 / 1e3) / 1e9
        per_size[f"{size}x{size}"] = {"requests": len(sel), "units": sum(reqs[r][0].ns for r in sel),
                                      "ms": round(m2, 3), "gpts_per_s": round(g2, 1),
                                      "hbm_frac_alg": round(16.0 * g2 / HBM_PEAK_GBS, 4)}
    # gradients of the whole batch (forward with D history or checkpoints, then the adjoint sweep and
    # imaging, every field in one persistent launch, then one fold launch) for band-limited adjoint sources
    bg = FwiBatch([a for a, _, _ in reqs], autotune=True, device=dev, gradients=True)
    v = bg.pack_velocity([m for _, m, _ in reqs])
    w = bg.pack_wavelets([x for _, _, x in reqs])
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    adj = torch.randn(bg.trace_elems, generator=gen, device=dev) * 1e-3
    g = bg.gradient(v, w, adj)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bg.gradient(v, w, adj, out=g)
    e1.record()
    torch.cuda.synchronize()
    if bg.status() != 0 or not bool(torch.isfinite(g).all()):
        print("gradient check failed", file=sys.stderr)
        sys.exit(1)
    gms = e0.elapsed_time(e1) / reps
    bg.close()
    gradient = {"ms": round(gms, 3), "requests_per_s": round(len(reqs) / (gms / 1e3), 2),
                "fields_per_s": round(sum(a.ns for a, _, _ in reqs) / (gms / 1e3), 1),
                "forward_gpts_per_s": round(upd / (gms / 1e3) / 1e9, 1), "cost_vs_forward": round(gms / ms, 3)}
    gtr = measured_traffic("uneven", "gradient")
    gradient["traffic"] = gtr  # HBM bytes of the launch (counters), and their rate over the timed launch
    gradient["measured_traffic_GBps"] = round(gtr / (gms / 1e3) / 1e9, 1) if gtr else None
    out = {
        "metric": "uneven batch forward GPts/s (64 requests, 70/140/256 grids, 1000-2500 steps)",
        "value": round(gpts, 1),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 1,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uneven batch: 64 requests (seeds 2000+r), 461 (request, shot) fields, "
                               f"{upd / 1e9:.2f} G point-updates per launch, one persistent launch"},
        "per_size": per_size,
        "gradient": gradient,
        "hbm_frac_alg": round(16.0 * gpts / HBM_PEAK_GBS, 4),
        # algorithmic bytes: 16 B per point-update (read u^n, u^{n-1}, K; write u^{n+1}) over the persistent
        # launch's measured duration; every field of a forward batch stays on chip (whole-field LDS loop or
        # LDS-resident row bands), so the rate is effective and the HBM bytes the counters measure are far fewer
        "roofline": {"bound": "hbm", "kernel": "k_batch_forward (one persistent launch)",
                     "achieved": round(16.0 * gpts, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(16.0 * gpts / HBM_PEAK_GBS, 4), "traffic": measured_traffic("uneven", "forward"),
                     "alg_bytes_per_launch": 16.0 * upd, "launch_ms": round(ms, 3),
                     "achieved_kind": "effective (algorithmic bytes / launch time)",
                     "measured_traffic_GBps": (round(measured_traffic("uneven", "forward") / (ms / 1e3) / 1e9, 1)
                                               if measured_traffic("uneven", "forward") else None),
                     "limiter": "VALU issue and per-step workgroup barriers / halo exchange (fields LDS-resident)"},
        "tiles": [{"padded": [t[0], t[1]], "kind": UNIT_KIND[t[2]], "tile": [t[3], t[4]], "parts": t[5]}
                  for t in tiles],
        "create_s": round(t_create, 3),
    }
    print(json.dumps(out))


# matrix-core FLOPs of the surrogate per sample (GEMMs only: the 4 encoder and 4 decoder MLPs, the depth->time
# map, the 4 x-mixing products, the head and the time up-sampling)
SUR_FWD_FLOP = 2.0 * (4 * 5184 * 2 * 64 * 128 + 256 * 72 * 4608 + 4 * (256 * 72 * 72 * 64 + 18432 * 2 * 64 * 128)
                      + 18432 * 64 * 8 + 1000 * 256 * 576)


def bench_surrogate(args):
    """Learned surrogate alone (70 x 70 -> 5 x 70 x 1000 traces): forward, forward + input VJP, and one Adam
    training step at batches of 16 and 64, with the matrix-core rate of the GEMM work against 2.5 PFLOP/s BF16."""
    import torch

    import fwi_inputs as fi
    from paper_2603_16393_amd.surrogate import Surrogate

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sur = Surrogate(64, device=dev)
    sur.set_params(np.load(SURROGATE_WEIGHTS))
    res = {}
    for B in (16, 64):
        v = torch.tensor(np.stack([fi.faulted_model(NZ, NX, s) for s in range(B)]), dtype=torch.float32, device=dev)
        tr = sur.forward(v)
        dtr = torch.randn_like(tr)
        dv = torch.empty_like(v)

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        reps = max(3, args.steps)
        f = timed(lambda: sur.forward(v, out=tr), reps)
        fb = timed(lambda: (sur.forward(v, out=tr), sur.backward(dtr, out=dv)), reps)
        ts = timed(lambda: sur.train_step(v, tr, lr=1e-7), reps)
        flop_f = SUR_FWD_FLOP * B
        res[f"B{B}"] = {"forward_ms": round(f, 3), "forward_vjp_ms": round(fb, 3), "train_step_ms": round(ts, 3),
                        "forward_tflops": round(flop_f / f / 1e9, 1),
                        "forward_mfma_frac": round(flop_f / f / 1e9 / 2500.0, 4),
                        "train_tflops": round(3 * flop_f / ts / 1e9, 1)}
    out = {"metric": "surrogate forward samples/s (70x70 -> 5x70x1000 traces)",
           "value": round(64 / (res["B64"]["forward_ms"] / 1e3), 1), "unit": "samples/s", "n_gpus": 1,
           "steps": max(3, args.steps), "warmup": 1, "ms_per_step": res["B64"]["forward_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "trace surrogate, batches of 16 and 64, trained parameters"},
           "flop_per_sample_forward": SUR_FWD_FLOP, "batches": res,
           # whole forward at B = 64 against the dense BF16 matrix-core peak; its layers are thin (K = 64 or 128)
           # and sit below the ridge point, so the per-kernel HBM figures in the profile are the binding ones
           "roofline": {"bound": "mfma", "kernel": "surrogate forward (all layers, B = 64)",
                        "achieved": res["B64"]["forward_tflops"], "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": res["B64"]["forward_mfma_frac"], "traffic": None}}
    sur.close()
    print(json.dumps(out))


def bench_checkpointed(args, pml=False):
    """Adjoint with checkpointing: 400 x 800 model (dx = 10 m) with a 50-cell sponge, 20 surface shots x 800
    receivers, 4000 samples at dt = 0.8 ms, 10 Hz Ricker, smooth-plus-layered model with a high-velocity lens
    (1500-5000 m/s); forward (u, w) checkpointed every 100 steps under a fixed memory budget.  pml: the same
    with the paper's 6-cell PML (Sec. 6.1) in place of the sponge, swept from HBM (forward u, w and psi
    checkpointed)."""
    import torch

    import fwi_inputs as fi
    from paper_2603_16393_amd import FwiPlan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nz, nx, ns, nt = 400, 800, 20, args.nt
    acq = fi.surface_acquisition(nz, nx, ns=ns, shot_cols=np.arange(ns) * 40, nt=nt, nb=6 if pml else 50, dt=8e-4,
                                 f_peak=10.0, v_max=5000.0)
    if pml:
        acq = dataclass_replace(acq, pml=True)
    v = fi.large_lens_model(nz, nx, seed=0)
    vt = fi.large_lens_model(nz, nx, seed=1)
    w = fi.ricker(nt, acq.dt, acq.f_peak)
    budget = 16 << 30
    if args.copy_calibration:
        copy_calibration(dev)
    plan = FwiPlan(acq, max_batch=1, device=dev, mem_budget_bytes=budget, ckpt_every=100, timing=True)
    wt = torch.tensor(w, dtype=torch.float32, device=dev)
    dobs = plan.forward(torch.tensor(vt[None], dtype=torch.float32, device=dev), wt, keep_for_adjoint=False)
    plan.set_obs(dobs[0].contiguous())
    vg = torch.tensor(v[None], dtype=torch.float32, device=dev)

    def step():
        d = plan.forward(vg, wt, keep_for_adjoint=True)
        J, adj = plan.w2_misfit(d)
        return plan.adjoint_gradient(vg, adj)

    for i in range(max(1, args.warmup)):
        step()
        torch.cuda.synchronize()
        print(f"checkpointed{' PML' if pml else ''}: warm-up gradient {i + 1} done", file=sys.stderr, flush=True)
    plan.sweep_ms()  # restart the sweep event averages at the timed region
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    fwd_ms, adj_ms = plan.sweep_ms()  # whole forward sweep; recomputation + adjoint steps
    nzp, nxp = acq.padded_shape
    per_sweep = ns * (nt - 1) * nzp * nxp
    updates = 3 * per_sweep  # forward, recomputation, adjoint
    if pml:
        # PML HBM sweep, per point-update: recomputation 24 B (u^n read, w read and written, K read, u^{n+1} and
        # D written), adjoint 32 B (mu and nu read and written, K and D read, the imaging sum read and written;
        # the gathered y = r mu is formed from mu and K); the layer's auxiliary fields are 1 % of the cells
        alg = per_sweep * (24.0 + 32.0)
        kernel = "k_pml_hbm_tile (recomputation + adjoint steps, one step per launch)"
        tr, ta = measured_traffic("pml_hbm", "recompute"), measured_traffic("pml_hbm", "adjoint")
        phase_traffic = (nt - 1) * (tr + ta) if tr and ta else None
    else:
        # algorithmic bytes of the adjoint phase (the dominant one): per point-update 16 B (u^n, w^n, K read,
        # u^{n+1} written) in both the recomputation and the adjoint steps, plus D written by the recomputation
        # and read back by the adjoint (4 B each)
        alg = per_sweep * (16.0 + 4.0) * 2
        kernel = "k_wave_tile2 (recomputation + adjoint steps, two steps per launch)"
        # measured HBM bytes of the same phase: its recomputation and adjoint launches (two steps each)
        tr, ta = measured_traffic("tile2", "recompute"), measured_traffic("tile2", "adjoint")
        phase_traffic = (nt // 2) * (tr + ta) if tr and ta else None
    achieved = alg / (adj_ms / 1e3) / 1e9
    print(json.dumps({
        "metric": f"checkpointed guidance gradient (400x800, 20 shots, {nt} samples{', 6-cell PML' if pml else ''})",
        "value": round(1e3 / ms, 4), "unit": "grads/s", "ms_per_gradient": round(ms, 2), "steps": args.steps,
        "gpts_per_s": round(updates / (ms / 1e3) / 1e9, 2),
        "sweep_ms": {"forward": round(fwd_ms, 2), "recompute_and_adjoint": round(adj_ms, 2)},
        "roofline": {"bound": "hbm", "kernel": kernel,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": phase_traffic, "alg_bytes_per_phase": alg,
                     "measured_traffic_GBps": (round(phase_traffic / (adj_ms / 1e3) / 1e9, 1) if phase_traffic
                                               else None)},
        "plan": {k: plan.info[k] for k in ("path", "store_mode", "ckpt_every", "device_bytes")},
        "memory_budget_bytes": budget, "dtype": "f32", "data": "synthetic",
    }))
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run the library's plain copy kernel on 512 MiB three times "
                         "(the reference dispatch for HBM traffic counters) and exit")
    ap.add_argument("--workload", choices=["guidance", "checkpointed", "checkpointed_pml", "uneven", "surrogate", "pml"],
                    default="guidance")
    ap.add_argument("--nt", type=int, default=4000,
                    help="checkpointed workload: trace samples (the workload has 4000; shorter runs serve the HBM "
                         "counter passes, whose per-launch figures are those of the full run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not built.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload in ("checkpointed", "checkpointed_pml"):
        bench_checkpointed(args, pml=args.workload == "checkpointed_pml")
        return
    if args.workload == "uneven":
        bench_uneven(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    if args.workload == "pml":
        bench_pml(args)
        return

    import torch

    from paper_2603_16393_amd import FwiPlan, FwiW2Loss, guidance_step  # noqa: F401
    import fwi_inputs as fi

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    acq, v0hat, v_true, w = make_inputs()
    plan = FwiPlan(acq, max_batch=B, device=dev, timing=True)
    wt = torch.tensor(w, dtype=torch.float32, device=dev)
    dobs = plan.forward(torch.tensor(v_true[None], dtype=torch.float32, device=dev), wt, keep_for_adjoint=False)
    plan.set_obs(dobs[0].contiguous())
    v = torch.tensor(v0hat, dtype=torch.float32, device=dev)
    x0 = torch.tensor(fi.to_normalised(v0hat), dtype=torch.float32, device=dev)
    d = torch.empty((B, NS, acq.nr, NT), dtype=torch.float32, device=dev)
    J = torch.empty(B, dtype=torch.float64, device=dev)
    adj = torch.empty_like(d)
    g = torch.empty((B, NZ, NX), dtype=torch.float32, device=dev)
    vn = torch.empty_like(g)
    rho = torch.empty(B, dtype=torch.float32, device=dev)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    stage_ms = np.zeros(4)

    def step(record=False):
        if record:
            ev[0].record()
        plan.forward(v, wt, keep_for_adjoint=True, out=d)
        if record:
            ev[1].record()
        plan.w2_misfit(d, want_adjoint=True, J_out=J, adj_out=adj)
        if record:
            ev[2].record()
        plan.adjoint_gradient(v, adj, out=g)
        if record:
            ev[3].record()
        guidance_step(x0, g, g, x0, unit_scale=1500.0, out=vn, rho_out=rho)
        if record:
            ev[4].record()

    if args.copy_calibration:
        # before any sweep
        copy_calibration(dev)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.warmup:
        plan.sweep_ms()  # restart the per-sweep event averages at the timed region
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record()
    for _ in range(args.steps):
        step()
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    # mean device time of the forward and adjoint sweep kernels over the timed steps (HIP events the
    # library records on the stream it launches them on)
    fwd_sweep_ms, adj_sweep_ms = plan.sweep_ms()
    # per-stage durations (HIP events on the stream the kernels run on), averaged over a few more steps
    reps = max(3, min(args.steps, 10))
    for _ in range(reps):
        step(record=True)
        torch.cuda.synchronize()
        stage_ms += np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(4)])
    stage_ms /= reps
    if plan.status() != 0:
        print("device-side check failed", file=sys.stderr)
        sys.exit(1)

    ms_per_step = total_ms / args.steps
    value = B * args.steps / (total_ms / 1e3)
    nzp, nxp = acq.padded_shape
    npts = nzp * nxp
    updates = B * NS * (NT - 1) * npts  # per sweep
    # algorithmic bytes per sweep: read u^n, u^{n-1}, K and write u^{n+1} (16 B) per point-update,
    # plus 4 B per model-region point for the forward history (written forward, read by the adjoint)
    alg_bytes = 16.0 * updates + 4.0 * B * NS * (NT - 1) * NZ * NX
    adj_dominant = adj_sweep_ms >= fwd_sweep_ms
    dom_ms = max(fwd_sweep_ms, adj_sweep_ms)
    split = plan.info.get("lds_split", 1) > 1
    kname = "k_wave_split" if split else "k_wave_lds"
    dom = f"{kname}<ADJ> (adjoint sweep)" if adj_dominant else f"{kname} (forward sweep)"
    achieved = alg_bytes / (dom_ms / 1e3) / 1e9
    traffic = measured_traffic("split", "adjoint" if adj_dominant else "forward")
    # after the timed region; not in counter runs, whose calibration dispatches are the only copies
    copy_gbps = None if args.copy_calibration else copy_rate_gbps(dev)
    ddpm_us = None if args.copy_calibration else ddpm_step_us(dev, v)
    out = {
        "metric": "guidance grads/s (70x70, 5 shots, 1k steps) plain vs surrogate @cos>=0.95",
        "value": round(value, 2),
        "unit": "grads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plain-solver guidance gradient: 16 faulted 70x70 models (dx=10 m, 1500-4500 m/s), 5 surface "
                        "shots x 70 receivers, 1000 samples at dt=1 ms, 15 Hz Ricker, 40-cell sponge, W2 misfit, "
                        "adjoint gradient, preconditioned update",
            "batch": B,
            "padded_grid": [nzp, nxp],
            "path": ("lds-resident" if plan.info["path"] == 0 else "tiled") +
                    (f", {plan.info['lds_split']} workgroups per field" if split else ""),
            "tile": [plan.info["lds_tile_x"], plan.info["lds_tile_z"]],
        },
        "stage_ms": {"forward": round(stage_ms[0], 4), "w2_misfit": round(stage_ms[1], 4),
                     "adjoint_gradient": round(stage_ms[2], 4), "guidance": round(stage_ms[3], 4)},
        "gpts_per_s": round(2 * updates / (ms_per_step / 1e3) / 1e9, 2),
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "launch_ms": round(dom_ms, 4),
            # beside the published peak: the measured copy rate; above 1 because the field stays in LDS
            "copy_GBps_measured": round(copy_gbps, 1) if copy_gbps else None,
            "frac_of_copy": round(achieved / copy_gbps, 4) if copy_gbps else None,
            # `achieved` is the effective rate on algorithmic bytes (the field never leaves the chip); the HBM
            # bytes the counters measured, per launch over the same duration, and what limits the kernel instead
            "achieved_kind": "effective (algorithmic bytes / launch time)",
            "measured_traffic_GBps": round(traffic / (dom_ms / 1e3) / 1e9, 1) if traffic else None,
            "measured_traffic_frac": round(traffic / (dom_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
            "limiter": "VALU issue and halo-exchange latency (the field is LDS-resident)",
        },
        "sweep_ms": {"forward": round(fwd_sweep_ms, 4), "adjoint": round(adj_sweep_ms, 4)},
        # reverse DDPM step of Algorithm 2 (clean estimator from a score, posterior mean + noise) on the batch
        "ddpm_step_us": ddpm_us,
        "variants": None,
        "operators": None,
        "surrogate": None,
        "cpu_baseline": None,
    }
    if not args.no_variants:
        out["variants"] = comparison_variants(plan, acq, wt, dobs[0].contiguous(), v, x0)
        out["operators"] = perturbed_operators(v0hat, v_true, x0)
        out["pml"] = pml_guidance(acq, v0hat, v_true, x0, w)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_guidance(plan, wt, v_true)
        out["reverse_loop"] = reverse_loop(plan, wt, v_true)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(acq, v0hat, v_true, w)
    print(json.dumps(out))
    plan.close()


if __name__ == "__main__":
    main()
