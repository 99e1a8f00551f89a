"""Conjugate gradient reconstruction of eps and sigma (box "CGA"), FP64.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU baseline may use it; the HIP path shares no
code with it.

The CGA minimises the Tikhonov functional of eq. tikhonov_functional,
    Phi(eps, sigma) = J(eps, sigma) + gamma_eps/2 |eps - eps^0|^2 + gamma_sig/2 |sigma - sigma^0|^2,
where J is the discrete trace misfit 1/2 sum |E - E_obs|^2 of oracle.solver and
eps^0, sigma^0 are the initial guesses.  Iteration m (m = 0, 1, ...) takes the steps
of box "CGA" in the paper's order:

  1. forward and adjoint solves at (eps^m, sigma^m) and the gradient functions of
     eq. gradeps, g^m = (dJ/dc_i) / m_i + gamma^m (c_i - c^0_i) on free nodes
     (c = eps or sigma; zero elsewhere);
  2./3. beta^m = |g^m|^2 / |g^{m-1}|^2, d^m = -g^m + beta^m d^{m-1} (d^0 = -g^0),
     c^{m+1} = c^m + alpha^m d^m, kept in the box of eq. epsilon_sigma_constraint
     (1 <= eps <= eps_max, 0 <= sigma <= sig_max);
  4. alpha^{m+1} = -(g^m, d^m) / (gamma^m (d^m, d^m));
  5. gamma^{m+1} = gamma^0 / (m + 1)^p;
  6. stop if (|eps^{m+1} - eps^m| < eta1_eps or |sigma^{m+1} - sigma^m| < eta1_sig)
     and (|g_eps^m| < eta2_eps or |g_sig^m| < eta2_sig).

Readings where the paper leaves a choice:
  * (u, v) and |u| are the L2(Omega) inner product and norm of the nodal functions
    with lumped-mass quadrature, (u, v) = sum_i m_i u_i v_i over the FEM nodes
    (m_i = h^3 on every free node);
  * g is the L2 representative of the derivative of Phi: the nodal derivative of the
    discrete J divided by the lumped mass, plus the Tikhonov term with the current
    gamma^m; the Tikhonov centre is the initial guess;
  * alpha^m of step 2 is the value step 4 produced in the previous iteration (alpha^0
    is given); beta^m = 0 when |g^{m-1}| = 0; alpha^{m+1} = alpha^m when d^m = 0;
  * the projection onto the box after each update is how the constraint of the
    inverse problem is kept; nodes of layers 0 and 1 keep eps = 1, sigma = 0;
  * the termination test groups as (step test for eps or sigma) and (gradient test
    for eps or sigma); a run also ends after a given number of iterations.
"""

from __future__ import annotations

import math

import numpy as np

from .solver import adjoint_gradient, forward, loss_and_cotangent

FIELDS = ("eps", "sig")


def inner(w, u, v):
    """(u, v) = sum_i w_i u_i v_i: lumped-mass quadrature of the L2(Omega) inner product."""
    return float(np.sum(w * u * v))


def gradient_function(dJ, w, c, c0, gamma, free):
    """Step 1: the gradient function of eq. gradeps at the nodes (L2 representative)."""
    g = np.zeros_like(c)
    g[free] = dJ[free] / w[free] + gamma * (c[free] - c0[free])
    return g


def tikhonov_value(J, w, eps, sig, eps0, sig0, gamma_eps, gamma_sig):
    """Phi of eq. tikhonov_functional with the lumped-mass quadrature of the penalty terms."""
    return (J + 0.5 * gamma_eps * inner(w, eps - eps0, eps - eps0)
            + 0.5 * gamma_sig * inner(w, sig - sig0, sig - sig0))


class CGAState:
    """Scalars and the previous direction of each coefficient field."""

    def __init__(self, n, params):
        self.m = 0
        self.params = dict(params)
        self.gamma = {f: float(params["gamma_" + f]) for f in FIELDS}
        self.alpha = {f: float(params["alpha_" + f]) for f in FIELDS}
        self.d = {f: np.zeros(n) for f in FIELDS}
        self.gn2_prev = {f: 0.0 for f in FIELDS}


def fletcher_reeves_beta(gn2, gn2_prev, m):
    """Steps 2/3: beta^m = |g^m|^2 / |g^{m-1}|^2 (no previous direction at m = 0)."""
    return gn2 / gn2_prev if m > 0 and gn2_prev > 0 else 0.0


def direction(g, beta, d_prev):
    """Steps 2/3: d^m = -g^m + beta^m d^{m-1}."""
    return -g + beta * d_prev


def project(c, lo, hi):
    """The box of eq. epsilon_sigma_constraint."""
    return np.clip(c, lo, hi)


def next_alpha(w, g, d, gamma, alpha):
    """Step 4: alpha^{m+1} = -(g^m, d^m) / (gamma^m (d^m, d^m))."""
    dd = inner(w, d, d)
    return -inner(w, g, d) / (gamma * dd) if dd > 0 else alpha


def next_gamma(gamma0, m, p):
    """Step 5: gamma^{m+1} = gamma^0 / (m + 1)^p."""
    return gamma0 / float(m + 1) ** p


def stop_test(step, gnorm, prm):
    """Step 6: (step test for eps or sigma) and (gradient test for eps or sigma)."""
    small_step = step["eps"] < prm.get("eta1_eps", 0.0) or step["sig"] < prm.get("eta1_sig", 0.0)
    small_grad = gnorm["eps"] < prm.get("eta2_eps", 0.0) or gnorm["sig"] < prm.get("eta2_sig", 0.0)
    return bool(small_step and small_grad)


def cga_update(state, dJ, coef, coef0, w, free):
    """Steps 2-6 of one iteration.

    dJ, coef, coef0: dicts over FIELDS of nodal arrays (dJ/dc, c^m, c^0).  Returns
    (new coefficients, info); state advances to iteration m + 1.
    """
    prm = state.params
    bounds = {"eps": (1.0, float(prm["eps_max"])), "sig": (0.0, float(prm["sig_max"]))}
    new, info = {}, {"m": state.m}
    for f in FIELDS:
        gamma = state.gamma[f]
        g = gradient_function(dJ[f], w, coef[f], coef0[f], gamma, free)
        gn2 = inner(w, g, g)
        beta = fletcher_reeves_beta(gn2, state.gn2_prev[f], state.m)
        d = direction(g, beta, state.d[f])
        c = coef[f].copy()
        c[free] = project(coef[f][free] + state.alpha[f] * d[free], *bounds[f])
        alpha_next = next_alpha(w, g, d, gamma, state.alpha[f])
        step = c - coef[f]
        info[f] = dict(grad_norm=math.sqrt(gn2), beta=beta, alpha_used=state.alpha[f], alpha_next=alpha_next,
                       step_norm=math.sqrt(inner(w, step, step)), gamma_used=gamma,
                       change_norm=math.sqrt(inner(w, c - coef0[f], c - coef0[f])))
        new[f] = c
        state.d[f] = d
        state.gn2_prev[f] = gn2
        state.alpha[f] = alpha_next
    for f in FIELDS:
        state.gamma[f] = next_gamma(float(prm["gamma_" + f]), state.m, float(prm["p"]))
        info[f]["gamma_next"] = state.gamma[f]
    info["converged"] = stop_test({f: info[f]["step_norm"] for f in FIELDS},
                                  {f: info[f]["grad_norm"] for f in FIELDS}, prm)
    state.m += 1
    return new, info


def cga_loop(grad_fn, eps0, sig0, w, free, params, n_iter):
    """Run up to n_iter CGA iterations with grad_fn(eps, sig) -> (dJ/deps, dJ/dsig, J).

    Returns the list of per-iteration infos (each with the coefficients it produced and J at
    the coefficients it started from).
    """
    eps0 = np.asarray(eps0, dtype=np.float64)
    sig0 = np.asarray(sig0, dtype=np.float64)
    state = CGAState(len(eps0), params)
    coef = {"eps": eps0.copy(), "sig": sig0.copy()}
    c0 = {"eps": eps0, "sig": sig0}
    hist = []
    for _ in range(n_iter):
        ge, gs, J = grad_fn(coef["eps"], coef["sig"])
        coef, info = cga_update(state, {"eps": ge, "sig": gs}, coef, c0, w, free)
        info["J"] = J
        info["eps"]["coef"] = coef["eps"].copy()
        info["sig"]["coef"] = coef["sig"].copy()
        hist.append(info)
        if info["converged"]:
            break
    return hist


def solve_gradient(d, sources, eobs, z=None, initial=None):
    """Step 1 on the discrete scheme: gradient of J summed over sources, and J (z: the
    smoothing function of eq. tikhonov_functional at the trace rows, or None for z = 1;
    initial: (f_0, f_1) of eq. forward_initial_cond for every source, or None for rest)."""
    def grad_fn(eps, sig):
        d.set_coefficients(eps, sig)
        ge = np.zeros(d.n_fem)
        gs = np.zeros(d.n_fem)
        J = 0.0
        for s, src in enumerate(sources):
            fw = forward(d, src, initial=initial)
            Js, r = loss_and_cotangent(fw["traces"], eobs[s], z)
            ag = adjoint_gradient(d, r, fw)
            ge += ag["g_eps"]
            gs += ag["g_sigma"]
            J += Js
        return ge, gs, J
    return grad_fn


def cga(d, sources, eobs, eps0, sig0, params, n_iter, z=None, initial=None):
    """The CGA on the discretisation d: eobs is [n_src][n_steps][n_det][3]."""
    w = d.m[d.fem_grid]
    return cga_loop(solve_gradient(d, sources, eobs, z, initial), eps0, sig0, w, d.fem_free, params, n_iter)
