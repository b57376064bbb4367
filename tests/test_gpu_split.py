"""Split LDS-resident sweep (several workgroups per field, 4-row halos
exchanged every step) through the C ABI.

The per-point arithmetic is the same as the one-workgroup-per-field sweep,
so traces and gradients must equal it bit for bit; each comparison is made
on several calls to catch a halo read from the wrong time level.  The
oracle bars are those of the plain path (rel L2 <= 1e-4).
"""
import dataclasses
import sys

import numpy as np
import pytest

import fwi_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _run(plan, v, w, adj, reps):
    outs = []
    for _ in range(reps):
        d = plan.forward(v, w, keep_for_adjoint=True)
        g = plan.adjoint_gradient(v, adj)
        torch.cuda.synchronize()
        outs.append((d.clone(), g.clone()))
    assert plan.status() == 0
    return outs


def _adjoint_sources(shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    k = np.exp(-0.5 * (np.arange(-30, 31) / 8.0) ** 2)
    x = np.apply_along_axis(lambda t: np.convolve(t, k, mode="same"), -1, x)
    return (x / np.abs(x).max()).astype(np.float32)


CASES = {
    # the guidance batch: 16 samples x 5 shots -> 3 workgroups per field
    "b16_70x70": dict(nz=70, nx=70, ns=5, nt=1000, nb=40, B=16, kw={}),
    # one field -> the finest split
    "b1_70x70_1shot": dict(nz=70, nx=70, ns=1, nt=600, nb=40, B=1, kw={}),
    # sponge on top, buried source and receiver rows, ragged tiles in x and z
    "b3_46x61_sponge_top": dict(nz=46, nx=61, ns=2, nt=400, nb=17, B=3,
                                kw=dict(free_surface=False, src_row=5, rec_row=9)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_split_equals_whole_field_sweep(dev, case):
    from paper_2603_16393_amd import FwiPlan

    c = CASES[case]
    acq = fi.surface_acquisition(c["nz"], c["nx"], ns=c["ns"], nt=c["nt"], nb=c["nb"], **c["kw"])
    B = c["B"]
    force = 1 if case != "b16_70x70" else 0
    ps = FwiPlan(acq, max_batch=B, device=dev, split=force)
    pw = FwiPlan(acq, max_batch=B, device=dev, split=-1)
    _say(f"{case}: split plan {ps.info}, whole-field tile {(pw.info['lds_tile_x'], pw.info['lds_tile_z'])}")
    assert ps.info["path"] == 0 and pw.info["path"] == 0
    assert ps.info["lds_split"] >= 2 and pw.info["lds_split"] == 1
    v = torch.tensor(np.stack([fi.faulted_model(c["nz"], c["nx"], 50 + b) for b in range(B)]).astype(np.float32),
                     device=dev)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    adj = torch.tensor(_adjoint_sources((B, acq.ns, acq.nr, acq.nt), 3), device=dev)
    ref = _run(pw, v, w, adj, 1)[0]
    for i, (d, g) in enumerate(_run(ps, v, w, adj, 3)):
        assert torch.equal(d, ref[0]), f"call {i}: traces differ (max {float((d - ref[0]).abs().max()):.3e})"
        assert torch.equal(g, ref[1]), f"call {i}: gradients differ (max {float((g - ref[1]).abs().max()):.3e})"
    ps.close()
    pw.close()


@pytest.mark.parametrize("ns,nt", [(17, 1000), (20, 500)])
def test_tail_split_equals_whole_field_sweep(dev, ns, nt):
    """More fields than CUs (16 samples x 17 or 20 shots): full rounds of the
    whole-field sweep, then the partial last round split over the idle CUs in
    a second launch; bit for bit the whole-field sweep's results, on three
    calls and for a smaller batch that has no partial round."""
    from paper_2603_16393_amd import FwiPlan

    acq = fi.surface_acquisition(70, 70, ns=ns, nt=nt, nb=40)
    B = 16
    ps = FwiPlan(acq, max_batch=B, device=dev)
    pw = FwiPlan(acq, max_batch=B, device=dev, split=-1)
    _say(f"{ns} shots: {B * ns} fields, plan {ps.info}")
    assert ps.info["lds_split"] == 1 and pw.info["lds_split"] == 1
    v = torch.tensor(np.stack([fi.faulted_model(70, 70, 80 + b) for b in range(B)]).astype(np.float32), device=dev)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    adj = torch.tensor(_adjoint_sources((B, acq.ns, acq.nr, acq.nt), 5), device=dev)
    for nb_ in (B, 4):
        ref = _run(pw, v[:nb_], w, adj[:nb_], 1)[0]
        for i, (d, g) in enumerate(_run(ps, v[:nb_], w, adj[:nb_], 3 if nb_ == B else 1)):
            assert torch.equal(d, ref[0]), f"B={nb_} call {i}: traces differ"
            assert torch.equal(g, ref[1]), f"B={nb_} call {i}: gradients differ"
    ps.close()
    pw.close()


def test_sources_and_receivers_on_band_boundaries(dev):
    """Receiver row and source on the published rows of a middle band (their
    corrections must precede the publication); split vs whole field bitwise,
    and vs the oracle."""
    import math

    import oracle
    from paper_2603_16393_amd import FwiPlan

    nz, nx, nb = 100, 60, 20
    probe = fi.surface_acquisition(nz, nx, ns=2, nt=300, nb=nb, free_surface=False)
    p0 = FwiPlan(probe, max_batch=2, device=dev, split=1)
    G, PI = p0.info["lds_split"], p0.info["lds_tile_z"]
    nzp = p0.info["nzp"]
    p0.close()
    H = 8 + max(1, math.ceil((math.ceil(nzp / G) - 8) / PI)) * PI
    assert G >= 3, (G, H)
    rec_pad, src_pad = H + 1, 2 * H - 2  # band 1: second row, next-to-last row
    acq = fi.surface_acquisition(nz, nx, ns=2, nt=300, nb=nb, free_surface=False, rec_row=rec_pad - nb,
                                 src_row=src_pad - nb)
    ps = FwiPlan(acq, max_batch=2, device=dev, split=1)
    pw = FwiPlan(acq, max_batch=2, device=dev, split=-1)
    assert (ps.info["lds_split"], ps.info["lds_tile_z"]) == (G, PI)
    _say(f"bands of {H} rows x {G}, receivers on padded row {rec_pad}, sources on row {src_pad}")
    models = np.stack([fi.faulted_model(nz, nx, 70 + b) for b in range(2)]).astype(np.float32)
    v = torch.tensor(models, device=dev)
    wav = fi.ricker(acq.nt, acq.dt, acq.f_peak).astype(np.float32)
    w = torch.tensor(wav, device=dev)
    adj_np = _adjoint_sources((2, acq.ns, acq.nr, acq.nt), 5)
    adj = torch.tensor(adj_np, device=dev)
    ref = _run(pw, v, w, adj, 1)[0]
    for i, (d, g) in enumerate(_run(ps, v, w, adj, 2)):
        assert torch.equal(d, ref[0]), f"call {i}: traces differ"
        assert torch.equal(g, ref[1]), f"call {i}: gradients differ"
    dref = oracle.forward(acq, models[0].astype(np.float64), wav.astype(np.float64))
    gref = oracle.gradient(acq, models[0].astype(np.float64), wav.astype(np.float64), adj_np[0].astype(np.float64))
    et, eg = _rel(ref[0][0].cpu().numpy(), dref), _rel(ref[1][0].cpu().numpy(), gref)
    _say(f"vs oracle: traces {et:.2e}, gradient {eg:.2e}")
    assert et <= 1e-4 and eg <= 1e-4
    ps.close()
    pw.close()


def test_split_vs_oracle_one_shot(dev):
    import oracle
    from paper_2603_16393_amd import FwiPlan

    acq = fi.surface_acquisition(70, 70, ns=1, nt=500, nb=40)
    plan = FwiPlan(acq, max_batch=1, device=dev, split=1)
    assert plan.info["lds_split"] >= 2
    m = fi.layered_model(70, 70, 3).astype(np.float32)
    wav = fi.ricker(acq.nt, acq.dt, acq.f_peak).astype(np.float32)
    adj = _adjoint_sources((1, acq.ns, acq.nr, acq.nt), 4)
    vt = torch.tensor(m[None], device=dev)
    d = plan.forward(vt, torch.tensor(wav, device=dev), keep_for_adjoint=True)
    g = plan.adjoint_gradient(vt, torch.tensor(adj, device=dev))
    torch.cuda.synchronize()
    assert plan.status() == 0
    dref = oracle.forward(acq, m.astype(np.float64), wav.astype(np.float64))
    gref = oracle.gradient(acq, m.astype(np.float64), wav.astype(np.float64), adj[0].astype(np.float64))
    et, eg = _rel(d[0].cpu().numpy(), dref), _rel(g[0].cpu().numpy(), gref)
    _say(f"split one-shot: traces rel L2 {et:.2e}, gradient rel L2 {eg:.2e}")
    assert et <= 1e-4 and eg <= 1e-4
    plan.close()


def test_split_option_errors(dev):
    from paper_2603_16393_amd import FwiPlan, _lib

    acq = fi.surface_acquisition(70, 70, ns=5, nt=100, nb=40)
    with pytest.raises(_lib.FwiError) as e:
        FwiPlan(acq, max_batch=64, device=dev, split=1)  # 320 fields: no CU left to share
    assert e.value.code == _lib.FWI_EINVAL
    with pytest.raises(_lib.FwiError):
        FwiPlan(acq, max_batch=1, device=dev, force_path=1, split=1)  # the tiled path does not split
    p = FwiPlan(acq, max_batch=1, device=dev, lds_tile=(3, 11))
    assert p.info["lds_split"] == 1  # an explicit tile keeps one workgroup per field
    p.close()


def test_split_plan_under_graph_capture(dev):
    """A plan that splits its fields runs the whole-field kernels while the
    caller's stream is capturing (a cooperative launch is not recorded); the
    captured forward + misfit + adjoint replays equal the eager (split) calls
    bit for bit."""
    from paper_2603_16393_amd import FwiPlan

    acq = fi.surface_acquisition(70, 70, ns=2, nt=300, nb=40)
    plan = FwiPlan(acq, max_batch=2, device=dev)
    assert plan.info["lds_split"] >= 2
    vt = torch.tensor(fi.faulted_model(70, 70, 9)[None].astype(np.float32), device=dev)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    plan.set_obs(plan.forward(vt, w, keep_for_adjoint=False)[0].contiguous())
    v = torch.tensor(np.stack([fi.faulted_model(70, 70, 80 + b) for b in range(2)]).astype(np.float32), device=dev)
    d = torch.empty((2, acq.ns, acq.nr, acq.nt), dtype=torch.float32, device=dev)
    J = torch.empty(2, dtype=torch.float64, device=dev)
    adj = torch.empty_like(d)
    g = torch.empty((2, 70, 70), dtype=torch.float32, device=dev)

    def step():
        plan.forward(v, w, keep_for_adjoint=True, out=d)
        plan.w2_misfit(d, J_out=J, adj_out=adj)
        plan.adjoint_gradient(v, adj, out=g)

    step()
    torch.cuda.synchronize()
    ref = (d.clone(), J.clone(), g.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        step()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            step()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        d.zero_()
        g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(d, ref[0]) and torch.equal(J, ref[1]) and torch.equal(g, ref[2]), f"replay {rep}"
        step()  # eager (split) work between replays
        torch.cuda.synchronize()
    assert plan.status() == 0
    del graph
    plan.close()
