"""Uneven batches in one persistent launch (fwi_batch_*) vs the FP64 oracle
and vs the per-geometry plan, through the C ABI (HBM-swept fields that
outlast the batch's share per compute unit run as row parts in lockstep).

Bars: seismograms and gradients relative L2 <= 1e-4 against the oracle (the
FP32-stencil target); against the plan's own sweep for the same geometry the
arithmetic per point is the same, so traces must agree bitwise (LDS-resident
units vs the LDS path, HBM-swept units vs the tiled path).  Gradients against
the plan agree to 1e-6 (the injection and imaging sums are the same
operations, the checkpoint schedules differ only in which steps are
recomputed, which is exact).
"""
import dataclasses
import sys

import numpy as np
import pytest

import fwi_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.linalg.norm(b))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _small_requests():
    """Five requests: LDS-resident sizes, a buried receiver row, receivers on two
    rows (swept from HBM), a grid too large for the LDS, a sponge on top."""
    reqs = []
    a0 = fi.surface_acquisition(24, 30, ns=2, nt=300, nb=8)
    reqs.append((a0, fi.faulted_model(24, 30, 1)))
    a1 = fi.surface_acquisition(40, 40, ns=3, nt=257, nb=10, rec_row=5)
    reqs.append((a1, fi.layered_model(40, 40, 2, depth_range=(5, 35))))
    a2 = fi.surface_acquisition(30, 36, ns=2, nt=211, nb=6)
    a2 = dataclasses.replace(a2, rec_iz=np.where(np.arange(a2.nr) % 2 == 0, 0, 3).astype(np.int32))
    reqs.append((a2, fi.faulted_model(30, 36, 3)))
    a3 = fi.surface_acquisition(100, 120, ns=2, nt=180, nb=20)
    reqs.append((a3, fi.faulted_model(100, 120, 4)))
    a4 = fi.surface_acquisition(20, 26, ns=1, nt=150, nb=8, free_surface=False, src_row=3, rec_row=2)
    reqs.append((a4, fi.layered_model(20, 26, 5, depth_range=(4, 16))))
    return [(a, v, fi.ricker(a.nt, a.dt, a.f_peak)) for a, v in reqs]


@pytest.mark.parametrize("autotune", [True, False])
def test_small_uneven_batch_vs_oracle_and_plans(dev, autotune):
    import oracle
    from paper_2603_16393_amd import FwiPlan
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = _small_requests()
    b = FwiBatch([a for a, _, _ in reqs], autotune=autotune, device=dev)
    kinds = [i["kind"] for i in b.info]
    parts = [i["parts"] for i in b.info]
    _say(f"kinds {kinds} tiles {[(i['tile_x'], i['tile_z'], i['tuned']) for i in b.info]} parts {parts}")
    # receivers on two rows: swept from HBM; the 100 x 120 field, too large for one workgroup's LDS, runs as
    # LDS-resident row bands on several workgroups
    assert kinds[0] == 0 and kinds[1] == 0 and kinds[2] == 1 and kinds[3] == 2
    assert parts[3] >= 2
    v = b.pack_velocity([m for _, m, _ in reqs])
    w = b.pack_wavelets([x for _, _, x in reqs])
    tr = b.forward(v, w)
    tr2 = b.forward(v, w)
    torch.cuda.synchronize()
    assert b.status() == 0
    assert torch.equal(tr, tr2)
    for r, (a, m, wav) in enumerate(reqs):
        got = b.traces_of(tr, r).cpu().numpy()
        ref = oracle.forward(a, np.asarray(m, np.float32).astype(np.float64),
                             np.asarray(wav, np.float32).astype(np.float64))
        err = _rel(got, ref)
        _say(f"request {r} kind {kinds[r]}: traces rel L2 vs oracle {err:.2e}")
        assert err <= 1e-4
        assert np.all(got[:, :, 0] == 0.0)
        # the plan's sweep of the same family rounds identically: LDS-resident (kind 0) vs the plan's LDS
        # sweep, HBM-swept (kind 1) vs its tiled sweep; row bands (kind 2, the LDS family's arithmetic) have no
        # plan counterpart at a size that does not fit one workgroup, so they are held to the tiled sweep at
        # FP32 rounding level
        plan = FwiPlan(a, max_batch=1, device=dev, force_path=-1 if kinds[r] == 0 else 1)
        assert plan.info["path"] == (0 if kinds[r] == 0 else 1)
        d = plan.forward(torch.tensor(np.asarray(m, np.float32)[None], device=dev),
                         torch.tensor(np.asarray(wav, np.float32), device=dev), keep_for_adjoint=False)
        torch.cuda.synchronize()
        ref_plan = d[0].cpu().numpy()
        if kinds[r] == 2:
            e = _rel(got, ref_plan)
            _say(f"request {r}: row bands vs the plan's tiled sweep rel L2 {e:.2e}")
            assert e <= 1e-5
        else:
            assert np.array_equal(ref_plan, got), f"request {r}: batch and plan sweeps differ"
        plan.close()
    b.close()


def test_row_bands_agree_with_the_hbm_sweep(dev):
    """The 140 x 140 and 256 x 256 requests of the uneven workload (one of each, all shots): as LDS-resident row
    bands (kind 2) and as HBM-swept fields (bands switched off: kind 1), forward traces and, in gradient batches,
    gradients.  The two evaluate the Laplacian in different FMA orders (the LDS family's and the tiled family's),
    so they agree to FP32 rounding, not bit for bit; each is reproducible bit for bit."""
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = fi.uneven_requests()
    pick = []
    for size in (140, 256):
        pick.append(next(r for r in range(len(reqs)) if reqs[r][0].nz == size))
    sel = [reqs[r] for r in pick]
    out, grad = {}, {}
    for bands in (True, False):
        b = FwiBatch([a for a, _, _ in sel], autotune=False, device=dev, gradients=True, bands=bands)
        kinds = [i["kind"] for i in b.info]
        _say(f"bands={bands}: kinds {kinds} parts {[i['parts'] for i in b.info]} "
             f"tiles {[(i['tile_x'], i['tile_z']) for i in b.info]}")
        assert kinds == ([2, 2] if bands else [1, 1])
        v = b.pack_velocity([m for _, m, _ in sel])
        w = b.pack_wavelets([x for _, _, x in sel])
        adj = b.pack_traces([_adjoint_sources(a, 70 + i) for i, (a, _, _) in enumerate(sel)])
        out[bands] = b.forward(v, w).cpu().numpy()
        again = b.forward(v, w).cpu().numpy()
        grad[bands] = b.gradient(v, w, adj).cpu().numpy()
        grad_again = b.gradient(v, w, adj).cpu().numpy()
        torch.cuda.synchronize()
        assert b.status() == 0
        assert np.array_equal(out[bands], again)
        assert np.array_equal(grad[bands], grad_again)
        b.close()
    e = _rel(out[True], out[False])
    eg = _rel(grad[True], grad[False])
    _say(f"row bands vs HBM sweep: traces rel L2 {e:.2e}, gradients rel L2 {eg:.2e}")
    assert e <= 1e-5
    assert eg <= 1e-5


def test_invalid_velocity_flag(dev):
    from paper_2603_16393_amd import _lib
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = _small_requests()[:2]
    b = FwiBatch([a for a, _, _ in reqs], autotune=False, device=dev)
    models = [m.copy() for _, m, _ in reqs]
    models[1][3, 4] = 5000.0  # above v_max
    b.forward(b.pack_velocity(models), b.pack_wavelets([x for _, _, x in reqs]))
    assert b.status() == _lib.FWI_EDEVICE
    assert b.status() == 0
    b.close()


def test_uneven_64_requests_sampled_vs_oracle(dev):
    """The 64-request mixed batch (70/140/256 grids, 1000/1500/2500 steps,
    5-10 shots) in the launch configuration the benchmark times; one shot of
    one request per size class checked against the oracle."""
    import oracle
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = fi.uneven_requests()
    b = FwiBatch([a for a, _, _ in reqs], autotune=True, device=dev)
    v = b.pack_velocity([m for _, m, _ in reqs])
    w = b.pack_wavelets([x for _, _, x in reqs])
    tr = b.forward(v, w)
    torch.cuda.synchronize()
    assert b.status() == 0
    assert bool(torch.isfinite(tr).all())
    seen = set()
    for r, (a, m, wav) in enumerate(reqs):
        if a.nz in seen:
            continue
        seen.add(a.nz)
        s = a.ns - 1
        sub = a.subset_shots([s])
        ref = oracle.forward(sub, np.asarray(m, np.float32).astype(np.float64),
                             np.asarray(wav, np.float32).astype(np.float64))[0]
        got = b.traces_of(tr, r)[s].cpu().numpy()
        err = _rel(got, ref)
        _say(f"request {r} ({a.nz}x{a.nx}, nt {a.nt}, shot {s}/{a.ns}, kind {b.info[r]['kind']}): rel L2 {err:.2e}")
        assert err <= 1e-4
    assert seen == {70, 140, 256}
    b.close()


def _adjoint_sources(acq, seed):
    """Band-limited adjoint sources [ns][nr][nt] (white noise filtered by the
    request's Ricker wavelet); the gradient is linear in them."""
    rng = np.random.default_rng(seed)
    wav = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    k = wav[: min(acq.nt, int(np.argmax(np.abs(wav))) * 2 + 1)]
    noise = rng.standard_normal((acq.ns, acq.nr, acq.nt))
    out = np.apply_along_axis(lambda t: np.convolve(t, k, mode="same"), 2, noise)
    return (out / np.abs(out).max()).astype(np.float32)


@pytest.mark.parametrize("autotune", [True, False])
def test_small_uneven_batch_gradient_vs_oracle_and_plans(dev, autotune):
    import oracle
    from paper_2603_16393_amd import FwiPlan
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = _small_requests()
    b = FwiBatch([a for a, _, _ in reqs], autotune=autotune, device=dev, gradients=True)
    kinds = [i["kind"] for i in b.info]
    _say(f"gradient batch: kinds {kinds} tiles {[(i['tile_x'], i['tile_z']) for i in b.info]}")
    v = b.pack_velocity([m for _, m, _ in reqs])
    w = b.pack_wavelets([x for _, _, x in reqs])
    adjs = [_adjoint_sources(a, 10 + r) for r, (a, _, _) in enumerate(reqs)]
    adj = b.pack_traces(adjs)
    tr = b.forward(v, w)
    g1 = b.gradient(v, w, adj)
    g2 = b.gradient(v, w, adj)
    tr2 = b.forward(v, w)
    torch.cuda.synchronize()
    assert b.status() == 0
    assert torch.equal(g1, g2), "gradient not reproducible"
    assert torch.equal(tr, tr2), "forward changed by a gradient call"
    for r, (a, m, wav) in enumerate(reqs):
        got = b.model_of(g1, r).cpu().numpy()
        m32 = np.asarray(m, np.float32)
        ref = oracle.gradient(a, m32.astype(np.float64), np.asarray(wav, np.float32).astype(np.float64),
                              adjs[r].astype(np.float64))
        err = _rel(got, ref)
        plan = FwiPlan(a, max_batch=1, device=dev, force_path=-1 if kinds[r] == 0 else 1)
        vt = torch.tensor(m32[None], device=dev)
        plan.forward(vt, torch.tensor(np.asarray(wav, np.float32), device=dev), keep_for_adjoint=True)
        gp = plan.adjoint_gradient(vt, torch.tensor(adjs[r][None], device=dev))[0].cpu().numpy()
        plan.close()
        ep = _rel(got, gp)
        _say(f"request {r} kind {kinds[r]}: gradient rel L2 vs oracle {err:.2e}, vs plan {ep:.2e}")
        assert err <= 1e-4
        if kinds[r] == 2:
            # row bands evaluate the Laplacian in the LDS family's order, the plan's tiled sweep in the tiled
            # family's: FP32 rounding apart
            assert ep <= 1e-5, f"request {r}: batch and plan gradients differ"
        else:
            assert np.array_equal(got, gp), f"request {r}: batch and plan gradients differ"
    b.close()


def test_gradient_needs_the_option(dev):
    from paper_2603_16393_amd import _lib
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = _small_requests()[:1]
    b = FwiBatch([a for a, _, _ in reqs], autotune=False, device=dev)
    v = b.pack_velocity([reqs[0][1]])
    w = b.pack_wavelets([reqs[0][2]])
    adj = torch.zeros(b.trace_elems, dtype=torch.float32, device=dev)
    with pytest.raises(_lib.FwiError) as e:
        b.gradient(v, w, adj)
    assert e.value.code == _lib.FWI_ESTATE
    b.close()


def test_uneven_64_requests_gradient_sampled_vs_oracle(dev):
    """Gradients of the 64-request mixed batch in one launch: every request
    gets band-limited adjoint sources, except that for one request per size
    class (the shortest record) they are zero on all shots but the last, so
    its gradient is that one shot's, which the oracle computes."""
    import oracle
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = fi.uneven_requests()
    picked = {}
    for r, (a, _, _) in enumerate(reqs):
        if a.nz not in picked or a.nt < reqs[picked[a.nz]][0].nt:
            picked[a.nz] = r
    b = FwiBatch([a for a, _, _ in reqs], autotune=True, device=dev, gradients=True)
    v = b.pack_velocity([m for _, m, _ in reqs])
    w = b.pack_wavelets([x for _, _, x in reqs])
    adjs = []
    for r, (a, _, _) in enumerate(reqs):
        x = _adjoint_sources(a, 100 + r)
        if r in picked.values():
            x[:-1] = 0.0
        adjs.append(x)
    g = b.gradient(v, w, b.pack_traces(adjs))
    torch.cuda.synchronize()
    assert b.status() == 0
    assert bool(torch.isfinite(g).all())
    for nz, r in sorted(picked.items()):
        a, m, wav = reqs[r]
        s = a.ns - 1
        sub = a.subset_shots([s])
        ref = oracle.gradient(sub, np.asarray(m, np.float32).astype(np.float64),
                              np.asarray(wav, np.float32).astype(np.float64), adjs[r][s:].astype(np.float64))
        got = b.model_of(g, r).cpu().numpy()
        err = _rel(got, ref)
        _say(f"request {r} ({a.nz}x{a.nx}, nt {a.nt}, shot {s}/{a.ns}, kind {b.info[r]['kind']}): "
             f"gradient rel L2 {err:.2e}")
        assert err <= 1e-4
    assert set(picked) == {70, 140, 256}
    b.close()


def test_batch_launches_replay_from_a_captured_graph(dev):
    """fwi_batch_forward / fwi_batch_gradient issue only kernels on the
    caller's stream (the work-queue counter is cleared by a kernel), so a
    caller can capture them into a graph; every replay, with eager calls in
    between, matches the eager result bit for bit."""
    from paper_2603_16393_amd.batch import FwiBatch

    reqs = _small_requests()
    b = FwiBatch([a for a, _, _ in reqs], autotune=False, device=dev, gradients=True)
    v = b.pack_velocity([m for _, m, _ in reqs])
    w = b.pack_wavelets([x for _, _, x in reqs])
    adj = b.pack_traces([_adjoint_sources(a, 40 + r) for r, (a, _, _) in enumerate(reqs)])
    tr_ref = b.forward(v, w).clone()
    g_ref = b.gradient(v, w, adj).clone()
    torch.cuda.synchronize()
    tr = torch.zeros_like(tr_ref)
    g = torch.zeros_like(g_ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.forward(v, w, out=tr)  # warm-up on the capture stream
        b.gradient(v, w, adj, out=g)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            b.forward(v, w, out=tr)
            b.gradient(v, w, adj, out=g)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        tr.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(tr, tr_ref), f"replay {rep}: traces differ"
        assert torch.equal(g, g_ref), f"replay {rep}: gradient differs"
        b.forward(v, w)  # eager work between replays
        torch.cuda.synchronize()
    assert b.status() == 0
    del graph
    b.close()
