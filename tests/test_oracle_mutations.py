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


def _cga_scalar_run(gamma0=1.0, n_iter=3):
    from oracle.cga import cga_loop
    w = np.array([1.0])
    prm = dict(gamma_eps=gamma0, gamma_sig=1.0, p=0.5, alpha_eps=0.25, alpha_sig=0.25, eps_max=10.0, sig_max=5.0)
    grad = lambda e, s: (w * (e - 3.0), np.zeros_like(s), 0.0)  # noqa: E731
    return [h["eps"]["coef"][0] for h in cga_loop(grad, np.array([1.0]), np.array([0.0]), w, np.array([True]), prm, n_iter)]


# hand-derived iterates of the scalar quadratic (tests/test_oracle_cga.py): gamma^0 = 1 and 2
CGA_CLOSED_FORMS = {1.0: [1.5, 3.0, 5.0 - 2.0 * math.sqrt(2.0) / 3.0], 2.0: [1.5, 29.0 / 16.0]}


def _cga_pins_hold():
    return all(np.allclose(_cga_scalar_run(g0, len(x)), x, rtol=1e-12, atol=0) for g0, x in CGA_CLOSED_FORMS.items())


def test_cga_mutations_are_caught_by_the_closed_form(monkeypatch):
    from oracle import cga as ocga
    assert _cga_pins_hold()
    alpha = ocga.next_alpha
    mutations = {
        "beta without the squares": ("fletcher_reeves_beta",
                                     lambda gn2, prev, m: math.sqrt(gn2 / prev) if m > 0 and prev > 0 else 0.0),
        "inverted beta": ("fletcher_reeves_beta", lambda gn2, prev, m: prev / gn2 if m > 0 and gn2 > 0 else 0.0),
        "direction sign": ("direction", lambda g, beta, d: g + beta * d),
        "alpha sign": ("next_alpha", lambda w, g, d, gamma, a: -alpha(w, g, d, gamma, a)),
        "alpha without gamma": ("next_alpha", lambda w, g, d, gamma, a: gamma * alpha(w, g, d, gamma, a)),
        "gamma index": ("next_gamma", lambda g0, m, p: g0 / float(m + 2) ** p),
        "gamma not decayed": ("next_gamma", lambda g0, m, p: g0),
    }
    for name, (fn, bad) in mutations.items():
        with monkeypatch.context() as mp:
            mp.setattr(ocga, fn, bad)
            assert not _cga_pins_hold(), name


def test_cga_unscaled_gradient_is_caught(monkeypatch):
    from oracle import cga as ocga
    from tests.test_oracle_cga import test_weighted_vector_quadratic_reduces_to_scalar as pin
    pin()
    orig = ocga.gradient_function
    monkeypatch.setattr(ocga, "gradient_function",
                        lambda dJ, w, c, c0, gamma, free: orig(dJ * w, w, c, c0, gamma, free))
    try:
        pin()
    except AssertionError:
        return
    raise AssertionError("an unscaled nodal derivative passed the weighted-quadratic pin")


def test_cga_termination_grouping_mutation_is_caught(monkeypatch):
    from oracle import cga as ocga
    from tests.test_oracle_cga import test_termination_grouping as pin
    pin()
    monkeypatch.setattr(ocga, "stop_test", lambda step, gn, prm: (step["eps"] < prm.get("eta1_eps", 0.0)
                                                                 and gn["eps"] < prm.get("eta2_eps", 0.0))
                        or (step["sig"] < prm.get("eta1_sig", 0.0) and gn["sig"] < prm.get("eta2_sig", 0.0)))
    try:
        pin()
    except AssertionError:
        return
    raise AssertionError("the per-field grouping of the stop test passed the termination pin")


# ---- general initial data: mistakes planted in the oracle's source text ---------------------

_INIT_MUTATIONS = {
    # E^{-1} = f_0 + dt f_1 (sign of the one-sided difference)
    "sign of the starting increment": ("E_prev = E_cur - V0", "E_prev = E_cur + V0"),
    # f_1 taken as the increment itself
    "dt missing from V^0": ("V0 = dt * np.asarray", "V0 = np.asarray"),
    # level -1 of the FEM history left at rest
    "level -1 not stored": ("fem_hist[0] = E_prev[d.fem_grid]", "fem_hist[0] = 0.0 * E_prev[d.fem_grid]"),
    # W^{-1/2} without its stiffness half
    "starting energy": ("/ dt ** 2 + 0.5 * np.sum(E_cur * d.apply_A(E_prev))", "/ dt ** 2"),
    # summation by parts without its boundary row
    "boundary row dropped": ("g_mass_sbp -= m * np.sum(lam_f[0]", "g_mass_sbp -= 0.0 * m * np.sum(lam_f[0]"),
}


def _mutated_solver(old, new):
    import types
    src = open(osolver.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle_solver_mutant")
    exec(compile(src.replace(old, new), "oracle_solver_mutant", "exec"), mod.__dict__)
    return mod


def test_initial_data_mutations_are_caught():
    from tests.test_oracle_initial_data import cosine_mode_errors, gradient_fd_errors, sbp_errors
    assert max(cosine_mode_errors()) < 1e-11 and sbp_errors()[0] < 1e-12
    for name, (old, new) in _INIT_MUTATIONS.items():
        m = _mutated_solver(old, new)
        caught = max(cosine_mode_errors(m)) > 1e-6 or sbp_errors(m)[0] > 1e-6
        if not caught:
            caught = gradient_fd_errors("R1", m) > 1e-3
        assert caught, name
