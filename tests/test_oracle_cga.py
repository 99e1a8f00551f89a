"""Pins of the CGA oracle (box "CGA", eq. tikhonov_functional, eq. gradeps).

* Closed form: on the quadratic Phi(x) = c/2 |x - x*|^2 + gamma/2 |x - x^0|^2 the CGA's
  iterates stay on the line through x^0 and x*, so the whole run reduces to scalars.
  With c = 1, gamma^0 = 1, p = 1/2, alpha^0 = 1/4, x^0 = 1, x* = 3 the paper's steps give
  by hand:
      m = 0: g = -2, d = 2, x^1 = 3/2, alpha^1 = -(g, d) / (gamma^0 (d, d)) = 1, gamma^1 = 1;
      m = 1: g = -1, beta = 1/4, d = 3/2, x^2 = 3, alpha^2 = 2/3, gamma^2 = 1/sqrt(2);
      m = 2: g = sqrt(2), beta = 2, d = 3 - sqrt(2), x^3 = 5 - 2 sqrt(2)/3,
             alpha^3 = -2 / (3 - sqrt(2)), gamma^3 = 1/sqrt(3).
  A dropped square in beta, a sign of d or alpha, an unlagged alpha or an off-by-one in
  the gamma schedule changes these numbers.  With gamma^0 = 2 (the rest as above):
      m = 0: g = -2, d = 2, x^1 = 3/2, alpha^1 = 1/2;
      m = 1: g = -1/2, beta = 1/16, d = 5/8, x^2 = 29/16, alpha^2 = 2/5.  The same run on nodes of unequal lumped mass
  (x^0, x* vectors) must give x^m = x^0 + t_m (x* - x^0) with the scalar t_m: this pins the
  division of the nodal derivative by the mass and the mass-weighted inner products.
* The box of eq. epsilon_sigma_constraint: an update past eps_max stops at eps_max.
* The termination test's grouping (either step test, and either gradient test).
* Brute force: the gradient function is the L2 representative of the derivative of the
  discrete Tikhonov functional: central differences of Phi along a direction v equal
  (g, v) with lumped-mass weights, on a tiny hybrid problem.
* Descent: the first iteration with a small alpha^0 lowers Phi on a tiny problem, keeps
  the box and leaves nodes of layers 0 and 1 at eps = 1, sigma = 0.
"""

import math

import numpy as np
import pytest

import synth
from oracle.cga import cga, cga_loop, gradient_function, inner, solve_gradient, tikhonov_value
from oracle.discretization import Discretization
from oracle.solver import forward, loss_and_cotangent

PARAMS = dict(gamma_eps=1.0, gamma_sig=1.0, p=0.5, alpha_eps=0.25, alpha_sig=0.25,
              eps_max=10.0, sig_max=5.0)


def _quadratic(w, xstar, c=1.0):
    """dJ/dx of J = c/2 sum_i w_i (x_i - x*_i)^2 (sigma part: J does not depend on sigma)."""
    def grad_fn(eps, sig):
        return w * c * (eps - xstar), np.zeros_like(sig), 0.5 * c * float(np.sum(w * (eps - xstar) ** 2))
    return grad_fn


def test_scalar_quadratic_closed_form():
    w = np.array([1.0])
    hist = cga_loop(_quadratic(w, np.array([3.0])), np.array([1.0]), np.array([0.0]), w,
                    np.array([True]), PARAMS, 3)
    s2 = math.sqrt(2.0)
    x = [h["eps"]["coef"][0] for h in hist]
    assert x == pytest.approx([1.5, 3.0, 5.0 - 2.0 * s2 / 3.0], rel=1e-15, abs=0)
    assert [h["eps"]["grad_norm"] for h in hist] == pytest.approx([2.0, 1.0, s2], rel=1e-15)
    assert [h["eps"]["beta"] for h in hist] == pytest.approx([0.0, 0.25, 2.0], rel=1e-15)
    assert [h["eps"]["alpha_used"] for h in hist] == pytest.approx([0.25, 1.0, 2.0 / 3.0], rel=1e-15)
    assert hist[2]["eps"]["alpha_next"] == pytest.approx(-2.0 / (3.0 - s2), rel=1e-14)
    assert [h["eps"]["gamma_next"] for h in hist] == pytest.approx([1.0, 1.0 / s2, 1.0 / math.sqrt(3.0)], rel=1e-15)
    # sigma has a zero gradient throughout: no movement, beta guarded, no NaN
    assert all(h["sig"]["coef"][0] == 0.0 and h["sig"]["grad_norm"] == 0.0 for h in hist)
    assert not any(h["converged"] for h in hist)


def test_scalar_quadratic_closed_form_gamma2():
    w = np.array([1.0])
    hist = cga_loop(_quadratic(w, np.array([3.0])), np.array([1.0]), np.array([0.0]), w,
                    np.array([True]), dict(PARAMS, gamma_eps=2.0), 2)
    assert [h["eps"]["coef"][0] for h in hist] == pytest.approx([1.5, 29.0 / 16.0], rel=1e-15, abs=0)
    assert [h["eps"]["beta"] for h in hist] == pytest.approx([0.0, 1.0 / 16.0], rel=1e-15)
    assert [h["eps"]["alpha_next"] for h in hist] == pytest.approx([0.5, 0.4], rel=1e-15)


def test_weighted_vector_quadratic_reduces_to_scalar():
    rng = np.random.default_rng(5)
    n = 7
    w = rng.uniform(0.3, 3.0, n) * 1e-3
    free = np.ones(n, dtype=bool)
    free[[0, 4]] = False
    x0 = np.where(free, rng.uniform(1.0, 2.0, n), 1.0)
    xs = np.where(free, x0 + rng.uniform(0.5, 1.5, n), 1.0)
    hist = cga_loop(_quadratic(w, xs), x0, np.zeros(n), w, free, PARAMS, 3)
    # scalar run: x^0 = 1, x* = 3 -> t_m = (x^m - 1) / 2
    t = np.array([0.25, 1.0, (4.0 - 2.0 * math.sqrt(2.0) / 3.0) / 2.0])
    # the line x^0 + t (x* - x^0) scales |g| by |x* - x^0| / 2 (weighted norm)
    scale = math.sqrt(inner(w, xs - x0, xs - x0)) / 2.0
    for h, tm in zip(hist, t):
        np.testing.assert_allclose(h["eps"]["coef"], x0 + tm * (xs - x0), rtol=1e-14, atol=0)
    assert [h["eps"]["grad_norm"] for h in hist] == pytest.approx([2 * scale, scale, math.sqrt(2) * scale], rel=1e-13)


def test_box_projection():
    w = np.array([1.0])
    prm = dict(PARAMS, eps_max=4.0)
    hist = cga_loop(_quadratic(w, np.array([3.0])), np.array([1.0]), np.array([0.0]), w, np.array([True]), prm, 3)
    assert hist[2]["eps"]["coef"][0] == 4.0                 # 5 - 2 sqrt(2)/3 > 4 is cut at eps_max
    assert hist[2]["eps"]["step_norm"] == pytest.approx(1.0, rel=1e-15)
    # below the lower bound: a large step toward eps < 1 stops at 1
    hist = cga_loop(_quadratic(w, np.array([-5.0])), np.array([1.0]), np.array([0.0]), w, np.array([True]),
                    dict(PARAMS, alpha_eps=10.0), 1)
    assert hist[0]["eps"]["coef"][0] == 1.0 and hist[0]["eps"]["step_norm"] == 0.0


def test_termination_grouping():
    w = np.array([1.0])
    run = lambda **eta: cga_loop(_quadratic(w, np.array([3.0])), np.array([1.0]), np.array([0.0]), w,  # noqa: E731
                                 np.array([True]), dict(PARAMS, **eta), 6)
    # steps 0.5, 1.5, ...; gradient norms 2, 1, ...: both eps tests hold first at m = 1
    assert len(run(eta1_eps=1.6, eta2_eps=1.5)) == 2
    # the step test alone (gradient test never met) never stops the run
    assert len(run(eta1_eps=10.0)) == 6
    # sigma never moves: its step test holds at once; with the eps gradient test at m = 0 -> one iteration
    assert len(run(eta1_sig=1e-12, eta2_eps=2.5)) == 1
    # sigma's zero gradient meets the gradient test at once; the eps step test decides:
    # the first step (0.5) is under 1.6; steps 0.5, 1.5, 1.057 all exceed 0.4
    assert len(run(eta2_sig=1e-12, eta1_eps=1.6)) == 1
    assert len(run(eta2_sig=1e-12, eta1_eps=0.4)) >= 3


def _tiny_problem():
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    eps0 = np.ones(d.n_fem)
    sig0 = np.zeros(d.n_fem)
    return w, d, src, eobs, eps0, sig0


def test_lumped_mass_weights_on_free_nodes():
    w, d, *_ = _tiny_problem()
    wt = d.m[d.fem_grid]
    h = w.desc.h
    n_free = int(np.prod([c - 3 for c in w.desc.fem_cells]))
    assert d.fem_free.sum() == n_free
    assert np.all(wt[d.fem_free] == pytest.approx(h ** 3, rel=1e-14))


def test_gradient_function_is_l2_representative():
    w, d, src, eobs, eps0, sig0 = _tiny_problem()
    wt = d.m[d.fem_grid]
    free = d.fem_free
    rng = np.random.default_rng(2)
    eps = np.where(free, 1.0 + rng.uniform(0.2, 1.5, d.n_fem), 1.0)
    sig = np.where(free, rng.uniform(0.05, 0.5, d.n_fem), 0.0)
    ge_, gs_, _ = solve_gradient(d, [src], eobs)(eps, sig)
    gam_e, gam_s = 3e3, 7e2
    g_e = gradient_function(ge_, wt, eps, eps0, gam_e, free)
    g_s = gradient_function(gs_, wt, sig, sig0, gam_s, free)

    def phi(e, s):
        dd = Discretization(w.desc).set_coefficients(e, s)
        J = loss_and_cotangent(forward(dd, src)["traces"], eobs[0])[0]
        return tikhonov_value(J, wt, e, s, eps0, sig0, gam_e, gam_s)

    v = np.where(free, rng.standard_normal(d.n_fem), 0.0)
    t = 1e-5
    fd_e = (phi(eps + t * v, sig) - phi(eps - t * v, sig)) / (2 * t)
    fd_s = (phi(eps, sig + t * v) - phi(eps, sig - t * v)) / (2 * t)
    assert inner(wt, g_e, v) == pytest.approx(fd_e, rel=1e-6)
    assert inner(wt, g_s, v) == pytest.approx(fd_s, rel=1e-6)
    # the unscaled nodal derivative is off by 1 / h^3: the pin separates the two
    assert abs(float(np.sum(g_e * v)) - fd_e) > 0.5 * abs(fd_e)


def test_first_iteration_descends_and_keeps_the_box():
    w, d, src, eobs, eps0, sig0 = _tiny_problem()
    wt = d.m[d.fem_grid]
    prm = dict(gamma_eps=1e-2, gamma_sig=1e-2, p=0.5, alpha_eps=0.0, alpha_sig=0.0, eps_max=8.0, sig_max=2.0)
    # alpha^0 such that the first update moves eps by 0.05 at most
    ge_, gs_, J0 = solve_gradient(d, [src], eobs)(eps0, sig0)
    ge = gradient_function(ge_, wt, eps0, eps0, prm["gamma_eps"], d.fem_free)
    gs = gradient_function(gs_, wt, sig0, sig0, prm["gamma_sig"], d.fem_free)
    prm.update(alpha_eps=0.05 / np.abs(ge).max(), alpha_sig=0.05 / max(np.abs(gs).max(), 1e-30))
    hist = cga(d, [src], eobs, eps0, sig0, prm, 2)
    e1, s1 = hist[0]["eps"]["coef"], hist[0]["sig"]["coef"]
    assert hist[1]["J"] < hist[0]["J"] == pytest.approx(J0, rel=1e-14)
    for h in hist:
        e, s = h["eps"]["coef"], h["sig"]["coef"]
        assert np.all((e >= 1.0) & (e <= 8.0) & (s >= 0.0) & (s <= 2.0))
        assert np.all(e[~d.fem_free] == 1.0) and np.all(s[~d.fem_free] == 0.0)
    assert np.any(e1 != 1.0) and np.any(s1 != 0.0)
