"""Pins of the oracle's general initial data (eq. forward_initial_cond: E(0) = f_0,
dE/dt(0) = f_1), taken as the starting levels E^0 = f_0, E^{-1} = f_0 - dt f_1.

* Closed form: with eps = 1, sigma = 0 and every face Neumann (mirror weights), a product of
  cosines cos(pi m_x i / (N_x - 1)) ... is an eigenvector of the lumped-mass 7-point operator
  with eigenvalue mu = sum_a (2 - 2 cos(pi m_a / (N_a - 1))) / h^2, so the three-level
  recursion moves its amplitude as a^n = A cos(n phi) + B sin(n phi), cos(phi) = 1 - dt^2 mu / 2,
  with a^0 = A (f_0) and a^{-1} = A - dt b (f_1 = b times the mode).  The traces equal that
  amplitude times the mode on every detector node.
* Invariant: the energy W^{n+1/2} is conserved from the starting pair on (W^{-1/2} included)
  and the balance identity holds with damping and a source.
* Brute force: the eps / sigma gradient matches central differences of J on a tiny grid with
  f_0, f_1 != 0 (both div-div forms); this is what pins the n = 0 rows, among them the
  -lambda(x, 0) f_1 term of eq. gradeps.
* Identity: the mass term equals its summation-by-parts form with the boundary term
  -m lambda^0 . V^0 / dt^2, which is a material part of it here.
* Zero initial data gives the start from rest bit for bit.
"""

import math

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle import solver as osolver
from oracle.solver import forward, loss_and_cotangent


def _closed_box(name="tiny", n_steps=120):
    w = synth.with_steps(synth.small(name), n_steps)
    w.desc.absorbing_faces = 0
    n = w.desc.n_fem_nodes()
    d = Discretization(w.desc).set_coefficients(np.ones(n), np.zeros(n))
    return w, d


def cosine_mode_errors(solver=None):
    """(max trace error / scale, energy spread / max, balance / max) of the closed-form case."""
    solver = solver or osolver
    w, d = _closed_box()
    desc = w.desc
    nx, ny, nz = desc.n_outer
    m = (2, 1, 3)
    lz, ly, lx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mode = (np.cos(np.pi * m[0] * lx / (nx - 1)) * np.cos(np.pi * m[1] * ly / (ny - 1))
            * np.cos(np.pi * m[2] * lz / (nz - 1))).ravel()
    A, b = np.array([0.7, -1.2, 0.4]), np.array([3.0, 0.5, -2.0])
    f0 = mode[:, None] * A[None, :]
    f1 = mode[:, None] * b[None, :]
    mu = sum((2.0 - 2.0 * math.cos(math.pi * m[a] / (desc.n_outer[a] - 1))) for a in range(3)) / desc.h ** 2
    dt = desc.dt
    phi = math.acos(1.0 - 0.5 * dt * dt * mu)
    B = (A * math.cos(phi) - (A - dt * b)) / math.sin(phi)
    fw = solver.forward(d, force=lambda n: np.zeros((d.N, 3)), initial=(f0, f1))
    n = np.arange(1, desc.n_steps + 1)
    amp = np.cos(n * phi)[:, None] * A[None, :] + np.sin(n * phi)[:, None] * B[None, :]
    expect = mode[d.det][None, :, None] * amp[:, None, :]
    scale = np.abs(expect).max()
    assert scale > 0.1
    W = fw["energy"]
    return (float(np.abs(fw["traces"] - expect).max() / scale), float((W.max() - W.min()) / W.max()),
            float(np.abs(fw["balance"]).max() / W.max()))


def test_cosine_mode_closed_form():
    tr, spread, bal = cosine_mode_errors()
    assert tr <= 1e-11
    # the energy of the starting pair is carried unchanged
    assert spread <= 1e-12 and bal <= 1e-12


def test_energy_balance_with_initial_data_damping_and_source():
    w = synth.with_steps(synth.small("ragged"), 200)
    n = w.desc.n_fem_nodes()
    d = Discretization(w.desc)
    sig = np.where(d.fem_free, 0.8, 0.0)
    d.set_coefficients(np.ones(n), sig)
    f0, f1 = synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 61)
    fw = forward(d, w.sources[0], initial=(f0, f1))
    assert np.abs(fw["balance"]).max() <= 1e-12 * np.abs(fw["energy"]).max()
    assert fw["energy"][-1] < 0.95 * fw["energy"][0]


def test_zero_initial_data_is_start_from_rest():
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    z = np.zeros((d.N, 3))
    a = forward(d, w.sources[0])
    b = forward(d, w.sources[0], initial=(z, z))
    for k in ("traces", "energy", "balance", "fem_hist"):
        np.testing.assert_array_equal(a[k], b[k])


def gradient_fd_errors(form, solver=None):
    """Worst relative error of g_eps, g_sigma against central differences of J (tiny grid,
    f_0, f_1 != 0), over a fifth of the free nodes."""
    solver = solver or osolver
    w = synth.small("tiny")
    src = w.sources[0]
    init = synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 62)
    d = Discretization(w.desc, divdiv_form=form).set_coefficients(w.eps, w.sigma)
    eobs = 0.8 * solver.forward(d, src)["traces"]          # data of the problem started from rest
    fw = solver.forward(d, src, initial=init)
    _, cot = loss_and_cotangent(fw["traces"], eobs)
    ag = solver.adjoint_gradient(d, cot, fw)

    def J(eps, sig):
        dd = Discretization(w.desc, divdiv_form=form).set_coefficients(eps, sig)
        return loss_and_cotangent(solver.forward(dd, src, initial=init)["traces"], eobs)[0]

    worst = 0.0
    free = np.nonzero(d.fem_free)[0]
    for i in free[:: max(1, len(free) // 5)]:
        for which in ("eps", "sig"):
            e, s = w.eps.copy(), w.sigma.copy()
            c = e if which == "eps" else s
            c[i] += 1e-5
            jp = J(e, s)
            c[i] -= 2e-5
            fd = (jp - J(e, s)) / 2e-5
            g = ag["g_eps" if which == "eps" else "g_sigma"][i]
            worst = max(worst, abs(g - fd) / abs(fd))
    return worst


@pytest.mark.parametrize("form", ["R1", "R2"])
def test_gradient_with_initial_data_matches_central_differences(form):
    assert gradient_fd_errors(form) <= 1e-4


def sbp_errors(solver=None):
    """(|g_mass - g_mass_sbp| / scale, boundary term / scale) with f_0, f_1 != 0."""
    solver = solver or osolver
    w = synth.small("ragged")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    init = synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 63)
    fw = solver.forward(d, w.sources[0], initial=init)
    cot = synth.noise(fw["traces"].shape, 7) * 1e-3
    ag = solver.adjoint_gradient(d, cot, fw, keep_lambda=True)
    scale = np.abs(ag["g_mass"]).max()
    lam0 = ag["lambda"][0][d.fem_grid]
    V0 = w.desc.dt * init[1][d.fem_grid]
    bt = np.where(d.fem_free, d.m[d.fem_grid] * np.sum(lam0 * V0, axis=1) / w.desc.dt ** 2, 0.0)
    ss = np.abs(ag["g_sigma"]).max()
    assert np.abs(ag["g_sigma"] - ag["g_sigma_sbp"]).max() <= 1e-12 * ss   # with its lambda^0 . V^0 row
    return float(np.abs(ag["g_mass"] - ag["g_mass_sbp"]).max() / scale), float(np.abs(bt).max() / scale)


def test_mass_term_summation_by_parts_with_boundary_term():
    err, bt = sbp_errors()
    assert err <= 1e-12
    # the boundary term -m lambda^0 . V^0 / dt^2 is not negligible here
    assert bt >= 1e-3
