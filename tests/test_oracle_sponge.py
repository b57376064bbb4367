"""Behavioural pins of the oracle's damping sponge (the absorbing layer of the
workloads; the paper's own layer type, the PML of Sec. 6.1, has its pins in
test_oracle_pml.py).

The paper specifies no sponge.  The oracle's reading is the damped wave
equation u_tt + eta u_t = v^2 (Lap u + s) inside an nb-cell layer, with the
quadratic profile eta = 3 v_max ln(1/R) / (2 nb h) (delta/nb)^2, R = 1e-3,
stepped as a damped discrete velocity: per axis the factor
a = (1 - eta dt/2)/(1 + eta dt/2) multiplies u^n - u^{n-1}, and a node in a
corner takes the product of its two axis factors.  These checks tie that
reading to what the physics fixes, independently of the oracle's code:

* the echo from the layer's outer (rigid) edge comes back attenuated by the
  WKB amplitude factor of the damped wave equation, exp(-(1/v) int eta dz)
  = R^(v_max / (2 v)) for a normally incident plane wave (1 - 2 eta dt for
  eta dt, a profile that is not quadratic, or a missing 1/2 in the factor
  each move it by an order of magnitude or more);
* the total returned signal falls as the layer widens (a gradual layer
  reflects less), and 40 cells return under 3 % of a rigid wall's echo;
* with a 40-cell layer on the sides and bottom, surface traces of a faulted
  model reproduce an unbounded-domain reference to under 3 % (the corners'
  product factors are exercised here);
* nb = 0 is the plain leapfrog (test_oracle_pml.py).

The plane wave comes from reciprocity, which the oracle satisfies exactly for
surface pairs (test_oracle_stencil.py): the sum over all surface receivers of
one centre shot equals the response at the centre to a line source along the
surface, a downgoing plane wave until its ends are felt.
"""
import math

import numpy as np
import pytest

import fwi_inputs as fi
import oracle

from test_oracle_pml import _unbounded_error

R_TARGET = 1e-3
V = 2000.0
D = 20          # model rows above the layer
NX = 400        # surface line of 4 km: its ends are felt at the centre after 1 s
DT = 1e-3
F_PEAK = 15.0


def _plane_response(nz, nb, v_max, nt):
    acq = fi.Acquisition(nz=nz, nx=NX, dz=10.0, dx=10.0, dt=DT, nt=nt, nb=nb, free_surface=True, v_max=v_max,
                         src_iz=np.array([0], np.int32), src_ix=np.array([NX // 2], np.int32),
                         rec_iz=np.zeros(NX, np.int32), rec_ix=np.arange(NX, dtype=np.int32), f_peak=F_PEAK)
    d = oracle.forward(acq, np.full((nz, NX), V), fi.ricker(nt, DT, F_PEAK))[0]
    return d.sum(axis=0)


def _echo_ratios(L, v_max, nt=1200):
    """(high-passed echo of the outer edge, whole return) of an L-cell layer under D model rows, each relative to
    the echo of a rigid wall at the same place (D + L model rows, no layer)."""
    a = _plane_response(D, L, v_max, nt)
    b = _plane_response(D + L, 0, v_max, nt)
    t = np.arange(nt) * DT
    t_echo = 2.0 * (D + L) * 10.0 / V + 1.1 / F_PEAK
    win = (t > t_echo - 0.1) & (t < t_echo + 0.1)
    assert t_echo + 0.1 < 1.0  # before the ends of the line source are felt
    # second time difference: keeps the 15 Hz echo, suppresses the layer's low-frequency onset reflection
    ha, hb = np.diff(a, 2), np.diff(b, 2)
    wh = win[1:-1]
    echo = np.max(np.abs(ha[wh])) / np.max(np.abs(hb[wh]))
    after_direct = (t > 0.18) & (t < t_echo + 0.1)
    whole = np.max(np.abs(a[after_direct])) / np.max(np.abs(b[win]))
    return echo, whole


@pytest.mark.parametrize("L,v_max", [(40, 2000.0), (40, 3000.0), (60, 4000.0)])
def test_outer_edge_echo_follows_damped_wave_attenuation(L, v_max):
    echo, _ = _echo_ratios(L, v_max)
    predicted = R_TARGET ** (v_max / (2.0 * V))
    assert 0.8 < echo / predicted < 1.25, (echo, predicted)


def test_return_falls_with_layer_width():
    whole = [_echo_ratios(L, 4000.0)[1] for L in (10, 20, 40, 60)]
    assert all(b < a for a, b in zip(whole, whole[1:])), whole
    assert whole[2] < 0.03, whole


def test_forty_cell_sponge_reproduces_the_unbounded_domain():
    e = _unbounded_error([(40, False), (20, False), (0, False)])
    assert e[(40, False)] < 0.03, e
    assert e[(40, False)] < 0.5 * e[(20, False)], e
    assert e[(0, False)] > 0.5, e
