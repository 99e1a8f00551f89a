"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each test perturbs one plausible detail of the oracle -- a dropped factor, a
sign, a shifted time index, a dropped gradient term -- and checks that the
corresponding pin's metric moves far outside its tolerance.
"""

import math

import numpy as np

import synth
from oracle import solver as osolver
from oracle.discretization import Discretization


def _dot_residual(d, nt=20, seed=1):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((nt, d.N, 3))
    fw = osolver.forward(d, force=lambda k: F[k], n_steps=nt)
    R = rng.standard_normal((nt, len(d.det), 3))
    ag = osolver.adjoint_gradient(d, R, fw, keep_lambda=True)
    lhs = np.sum(R * fw["traces"])
    return abs(lhs + np.sum(ag["lambda"] * F)) / abs(lhs)


def test_dropped_eps_minus_one_in_transpose_is_caught():
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    assert _dot_residual(d) < 1e-12
    orig = d.divdiv_T
    d.divdiv_T = lambda L: orig(L) / np.where(d.eps > 1, d.eps - 1.0, 1.0)[:, None] * d.eps[:, None]
    assert _dot_residual(d) > 1e-6


def test_shifted_damping_index_in_adjoint_is_caught():
    w = synth.small("tiny")
    w.desc.t_switch = 8.5 * w.desc.dt
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    rng = np.random.default_rng(2)
    nt = 20
    F = rng.standard_normal((nt, d.N, 3))
    fw = osolver.forward(d, force=lambda k: F[k], n_steps=nt)
    R = rng.standard_normal((nt, len(d.det), 3))
    orig = d.damping
    d.damping = lambda n: orig(n + 1)          # adjoint uses S^k instead of S^{k-1}
    ag = osolver.adjoint_gradient(d, R, fw, keep_lambda=True)
    lhs = np.sum(R * fw["traces"])
    assert abs(lhs + np.sum(ag["lambda"] * F)) / abs(lhs) > 1e-8


def test_source_sign_is_caught_by_plane_wave(monkeypatch):
    from tests.test_oracle_invariants import _plane_wave_error
    src = synth.gauss_sine(2 * math.pi)
    assert _plane_wave_error(0.05, src) < 2e-2
    orig = osolver.forcing
    monkeypatch.setattr(osolver, "forcing", lambda d, s, n: -orig(d, s, n))
    assert _plane_wave_error(0.05, src) > 1.5


def test_dropped_divdiv_gradient_term_is_caught():
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = osolver.forward(d, src)["traces"] * 0.9
    fw = osolver.forward(d, src)
    _, cot = osolver.loss_and_cotangent(fw["traces"], eobs)
    ag = osolver.adjoint_gradient(d, cot, fw)
    i = int(np.nonzero(d.fem_free)[0][0])
    delta = 1e-5
    e = w.eps.copy()
    e[i] += delta
    jp = osolver.loss_and_cotangent(osolver.forward(Discretization(w.desc).set_coefficients(e, w.sigma), src)["traces"], eobs)[0]
    e[i] -= 2 * delta
    jm = osolver.loss_and_cotangent(osolver.forward(Discretization(w.desc).set_coefficients(e, w.sigma), src)["traces"], eobs)[0]
    fd = (jp - jm) / (2 * delta)
    assert abs(ag["g_eps"][i] - fd) <= 1e-4 * abs(fd)
    assert abs(ag["g_mass"][i] - fd) > 1e-2 * abs(fd)      # mass term alone is wrong
