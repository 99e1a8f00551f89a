"""Pins of the oracle's obliquely incident plane wave (a plane-wave source with a direction k).

The model problem's source (eq. model1 with eq. f) is the boundary condition d_n E = P(t) on
the top face: a wave entering normally.  A wave travelling along a unit direction k (k_z < 0)
reaches top-face node i at the delay tau_i = k . (x_i - x_ref), x_ref the top-face node it
reaches first, so there d_n E = P(t - tau_i) (the reading this repository takes).  In eps = 1
the continuous solution is then the plane wave E = pol Q(t - k . (x - x_ref)) / cos(theta),
Q = int_0^t P, cos(theta) = -k_z: its normal derivative on the face is -k_z P / cos(theta) = P.
The box's Neumann sides do not carry that wave: the data beyond a side differ from it, and the
difference travels inward at speed one, so near the face centre the closed form holds until
the distance to the nearest side has elapsed.  A wave in the x-z plane is independent of y,
which a thin slab with Neumann y-faces carries exactly.

Pinned here: second-order convergence of the top-face traces to that closed form inside its
window, the same for a wave in the y-z plane (the other delay axis), bit-for-bit equality of
k = -e_z with normal incidence, the refused upward direction, and planted mistakes (delay sign,
reference node, an extra cos(theta) in the forcing) that fail the pin.
"""

import math

import numpy as np
import pytest
from scipy.integrate import cumulative_simpson

import synth
from oracle import solver as osolver
from oracle.discretization import Discretization
from synth.configs import FACE_BOTTOM, FACE_TOP, SRC_GAUSS_SINE, ProblemDesc, Source

THETA = math.radians(25.0)
LONG, DEPTH = 4.0, 1.0       # slab length along the delay axis and depth
TP = 0.4                     # pulse period
X_C = LONG / 2
T_END = X_C - 0.3            # before the sides' influence reaches the observed nodes


def _q_of(src):
    """Q(s) = int_0^s P on a fine table (composite Simpson), linear in between."""
    sup = 2.0 * src.t0
    ts = np.linspace(0.0, sup, 40001)
    pv = np.array([osolver.source_time_function(src, s) for s in ts])
    tab = cumulative_simpson(pv, x=ts, initial=0.0)
    return lambda s: np.interp(np.clip(s, 0.0, sup), ts, tab)


def _oblique_error(h, axis=0):
    """Rel L2 error of the top-face traces (component of pol) near the face centre against
    pol Q(t - tau) / cos(theta), for a wave tilted along `axis` (0: x, 1: y)."""
    n_long = int(round(LONG / h)) + 1
    nz = int(round(DEPTH / h)) + 1
    dims = [5, 5, nz]
    dims[axis] = n_long
    dt = 0.5 * h / math.sqrt(3.0)
    nt = int(T_END / dt)
    desc = ProblemDesc(n_outer=tuple(dims), h=h, origin=(0.0, 0.0, 0.0), fem_lo=(1, 1, 1), fem_cells=(2, 2, 2),
                       dt=dt, n_steps=nt, ckpt_every=nt, detector_faces=FACE_TOP, absorbing_faces=FACE_BOTTOM,
                       t_switch=1e9)
    k = np.zeros(3)
    k[axis] = math.sin(THETA)
    k[2] = -math.cos(THETA)
    pol = [0.0, 0.0, 0.0]
    pol[1 - axis] = 1.0
    src = Source(kind=SRC_GAUSS_SINE, omega=2 * math.pi / TP, t0=1.5 * TP, width=0.5 * TP, pol=tuple(pol),
                 dir=tuple(k))
    d = Discretization(desc, fd_only=True).set_coefficients(np.ones(27), np.zeros(27))
    tr = osolver.forward(d, src)["traces"][:, :, 1 - axis]
    xd = d.x[d.det]
    sel = (np.abs(xd[:, 1 - axis] - 2 * h) < 1e-9) & (np.abs(xd[:, axis] - X_C) <= 0.25 + 1e-9)
    g = xd[:, axis] * 8.0
    sel &= np.abs(g - np.round(g)) < 1e-9
    tn = dt * np.arange(1, nt + 1)
    Q = _q_of(src)
    tau = xd[sel, axis] * k[axis]
    exact = np.stack([Q(tn - ti) for ti in tau], axis=1) / math.cos(THETA)
    return float(np.linalg.norm(tr[:, sel] - exact) / np.linalg.norm(exact))


_ERR = {}


def _err(h, axis=0):
    if (h, axis) not in _ERR:
        _ERR[(h, axis)] = _oblique_error(h, axis)
    return _ERR[(h, axis)]


def test_oblique_plane_wave_second_order():
    errs = [_err(h) for h in (1 / 20, 1 / 40, 1 / 80)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 <= r1 <= 4.8 and 3.6 <= r2 <= 4.5, errs
    assert errs[2] < 5e-3, errs


def test_oblique_wave_along_y_is_the_mirror_case():
    """The same wave tilted along y on the transposed slab: the same error to rounding."""
    assert abs(_err(1 / 40, axis=1) - _err(1 / 40, axis=0)) <= 1e-9 * _err(1 / 40, axis=0)


def test_straight_down_equals_normal_incidence():
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    base = w.sources[0]
    ref = osolver.forward(d, base)["traces"]
    assert np.abs(ref).max() > 0
    for v in ((0.0, 0.0, -1.0), (0.0, 0.0, -2.5)):
        s = Source(kind=base.kind, omega=base.omega, t0=base.t0, width=base.width, amp=base.amp, pol=base.pol, dir=v)
        assert np.array_equal(osolver.forward(d, s)["traces"], ref)


def test_upward_direction_is_refused():
    src = Source(kind=SRC_GAUSS_SINE, omega=1.0, t0=1.0, width=0.5, dir=(0.3, 0.0, 0.1))
    with pytest.raises(ValueError):
        osolver.incidence(src)


@pytest.mark.parametrize("mutation", ["delay_sign", "reference", "cos_factor"])
def test_oblique_mutations_are_caught(monkeypatch, mutation):
    base = _err(1 / 40)
    if mutation == "delay_sign":
        orig = osolver.arrival_delays
        monkeypatch.setattr(osolver, "arrival_delays", lambda d, k: (lambda t: (t[0], -t[1]))(orig(d, k)))
    elif mutation == "reference":
        orig = osolver.arrival_delays
        monkeypatch.setattr(osolver, "arrival_delays", lambda d, k: (lambda t: (t[0], t[1].max() - t[1]))(orig(d, k)))
    else:
        orig = osolver.forcing
        monkeypatch.setattr(osolver, "forcing", lambda d, s, n: math.cos(THETA) * orig(d, s, n))
    bad = _oblique_error(1 / 40)
    assert bad > 3.0 * base and bad > 0.05, (mutation, base, bad)
