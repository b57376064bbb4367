"""Pins of the oracle's perfectly matched layer (Sec. 2.1: absorbing boundary
on the non-reflecting sides; Sec. 6.1: a PML of 6 grid points on the left,
right and bottom).  The paper gives no PML equations; the oracle follows the
unsplit second-order PML obtained from a complex coordinate stretch, and
these checks tie it to what such a layer must do, independently of its own
code:

* without a layer (nb = 0) it is the pinned sponge-free leapfrog, bit for bit;
* inside the model it reproduces the solution of an unbounded domain (the
  same model with its edges extended far enough that nothing returns within
  the record, computed by the pinned sponge scheme) to about 1e-3, which a
  damping sponge of the same width (about 0.4) and a rigid edge (about 1)
  do not;
* thickening the layer reduces the error (the discrete layer converges);
* after the source stops, the field decays (no growing mode at 0.95 of the
  CFL limit and the largest damping);
* left-right symmetry of a symmetric experiment (index and sign errors in
  the x-direction terms break it);
* the reverse-mode gradient equals central finite differences of the
  forward map on tiny grids, with and without the reflecting top (every
  transpose, including the mirrored ones, against the forward).
"""
import dataclasses

import numpy as np
import pytest

import fwi_inputs as fi
import oracle


def _shot(acq, s):
    return acq.subset_shots([s])


def test_pml_without_layer_is_the_leapfrog():
    acq = dataclasses.replace(_shot(fi.operator_acquisition("Init"), 5), nb=0, nt=300)
    v = fi.faulted_model(70, 70, 3)
    w = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    d_plain = oracle.forward(acq, v, w)
    d_pml = oracle.forward(dataclasses.replace(acq, pml=True), v, w)
    assert np.array_equal(d_plain, d_pml)
    rng = np.random.default_rng(2)
    a = rng.standard_normal(d_plain.shape)
    g_plain = oracle.gradient(acq, v, w, a)
    g_pml = oracle.gradient(dataclasses.replace(acq, pml=True), v, w, a)
    assert np.max(np.abs(g_pml - g_plain)) <= 1e-12 * np.max(np.abs(g_plain))


def _unbounded_error(nb_list, nt=800, ext=260):
    """Relative L2 error of the surface traces against an unbounded-domain
    reference: the model padded by `ext` edge-replicated cells on the sides
    and bottom (waves need 2 ext cells = 520 > 4500 m/s * 0.8 s / 10 m = 360
    cells to come back), run without any layer."""
    base = dataclasses.replace(_shot(fi.operator_acquisition("Init"), 3), nt=nt)
    v = fi.faulted_model(70, 70, 1000)
    w = fi.ricker(nt, base.dt, base.f_peak)
    ref_acq = dataclasses.replace(base, nz=70 + ext, nx=70 + 2 * ext, src_ix=base.src_ix + ext,
                                  rec_ix=base.rec_ix + ext, nb=0)
    d_ref = oracle.forward(ref_acq, np.pad(v, ((0, ext), (ext, ext)), mode="edge"), w)
    out = {}
    for key in nb_list:
        nb, pml = key
        d = oracle.forward(dataclasses.replace(base, nb=nb, pml=pml), v, w)
        out[key] = float(np.linalg.norm(d - d_ref) / np.linalg.norm(d_ref))
    return out


def test_pml_reproduces_the_unbounded_domain():
    e = _unbounded_error([(6, True), (10, True), (6, False), (0, False)])
    assert e[(6, True)] < 3e-3
    assert e[(10, True)] < 0.5 * e[(6, True)]
    assert e[(6, False)] > 0.1       # a sponge this thin reflects
    assert e[(0, False)] > 0.5       # a rigid edge reflects everything


@pytest.mark.parametrize("fs", [True, False])
def test_pml_field_decays_after_the_source(fs):
    acq = dataclasses.replace(_shot(fi.operator_acquisition("Init"), 5), nb=6, pml=True, free_surface=fs, nt=4000)
    # time step at 0.95 of the stability limit for v_max
    dt = 0.95 * acq.dt / oracle.cfl_number(acq.v_max, acq.dt, acq.dz, acq.dx)
    acq = dataclasses.replace(acq, dt=dt)
    v = np.full((70, 70), acq.v_max)
    d = oracle.forward(acq, v, fi.ricker(acq.nt, dt, acq.f_peak))[0]
    assert np.max(np.abs(d[..., -500:])) < 1e-5 * np.max(np.abs(d))


def test_pml_symmetric_experiment_gives_symmetric_traces():
    nx = 41
    acq = fi.Acquisition(nz=30, nx=nx, dz=10.0, dx=10.0, dt=0.001, nt=600, nb=6, free_surface=True, v_max=3000.0,
                         src_iz=np.array([3], np.int32), src_ix=np.array([nx // 2], np.int32),
                         rec_iz=np.zeros(nx, np.int32), rec_ix=np.arange(nx, dtype=np.int32), pml=True)
    v = np.tile(np.linspace(2000.0, 3000.0, 30)[:, None], (1, nx))
    d = oracle.forward(acq, v, fi.ricker(acq.nt, acq.dt, 15.0))[0]  # [receiver][sample]
    assert np.max(np.abs(d - d[::-1])) <= 1e-12 * np.max(np.abs(d))


@pytest.mark.parametrize("fs", [True, False])
def test_pml_gradient_matches_finite_differences(fs):
    rng = np.random.default_rng(5 + int(fs))
    nz, nx = 9, 11
    acq = fi.Acquisition(nz=nz, nx=nx, dz=10.0, dx=12.0, dt=0.001, nt=140, nb=6, free_surface=fs, v_max=4000.0,
                         src_iz=np.array([1, 3], np.int32), src_ix=np.array([2, 8], np.int32),
                         rec_iz=np.full(nx, 0 if fs else 1, np.int32), rec_ix=np.arange(nx, dtype=np.int32),
                         f_peak=25.0, pml=True)
    v = 2000.0 + 1500.0 * rng.random((nz, nx))
    w = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    a = rng.standard_normal((acq.ns, acq.nr, acq.nt))
    g = oracle.gradient(acq, v, w, a)

    def J(vv):
        return float(np.sum(a * oracle.forward(acq, vv, w)))

    # corners, edges (whose gradient collects the layer's cells) and the interior
    for iz, ix in [(0, 0), (0, nx - 1), (nz - 1, 0), (nz - 1, nx - 1), (4, 5), (0, 5), (nz - 1, 5), (3, 0)]:
        h = 1e-4 * v[iz, ix]
        vp, vm = v.copy(), v.copy()
        vp[iz, ix] += h
        vm[iz, ix] -= h
        fd = (J(vp) - J(vm)) / (2 * h)
        assert abs(fd - g[iz, ix]) <= 1e-6 * np.max(np.abs(g)), (iz, ix, fd, g[iz, ix])
