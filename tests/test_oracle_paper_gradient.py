"""Pins of the paper-formula gradient variant and the symmetric div-div form R2.

eq. gradeps writes the div-div part of g_eps as the time integral of div(lambda) div(E),
having dropped grad(eps~).E from div(eps~ E).  On the discrete scheme that is
    sum_n sum_{K ∋ i} (|K| / 4) div_K(lambda^n) div_K(E^n),
which is not the derivative of the R1 scheme (the nodal product inside the divergence) but is
exactly the derivative of the R2 scheme, whose div-div term carries the element mean of
eps - 1 outside the divergence.  So:

* R2 equals R1 when eps is constant (then (eps - 1) leaves the divergence in both);
* R2 is symmetric on fields supported on the FEM-owned nodes, and each form's transpose is
  its transpose (inner-product identity);
* the adjoint recursion stays the exact transpose under R2 (dot-product test);
* brute force: under R2 the paper formula matches central differences of J per free node
  (this is what pins the formula's code, weights |K|/4 and restriction included);
* under R1 the paper formula is a different vector from the exact gradient (it is reported
  against it, not used in its place).

The smoothing function z of eq. tikhonov_functional (the misfit weighted in time):
* the taper is 1 up to T - delta, 0 at T (the last trace row is time level N_t), monotone and
  C1 at both ends of its ramp;
* brute force: with z the adjoint source z_n r^n gives the gradient of the weighted J
  (central differences), and the unweighted source does not.
"""

import numpy as np

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward, loss_and_cotangent


def _tiny(form):
    w = synth.small("tiny")
    return w, Discretization(w.desc, divdiv_form=form).set_coefficients(w.eps, w.sigma)


def test_r2_equals_r1_for_constant_eps():
    w, d1 = _tiny("R1")
    _, d2 = _tiny("R2")
    rng = np.random.default_rng(1)
    E = rng.standard_normal((d1.N, 3))
    for d in (d1, d2):
        d.eps = np.full(d.n_fem, 2.7)       # operator identity only (not an admissible medium)
    np.testing.assert_allclose(d2.divdiv(E), d1.divdiv(E), rtol=1e-12, atol=1e-12 * np.abs(d1.divdiv(E)).max())
    np.testing.assert_allclose(d2.divdiv_T(E), d1.divdiv_T(E), rtol=1e-12, atol=1e-12 * np.abs(d1.divdiv_T(E)).max())


def test_transposes_and_r2_symmetry():
    rng = np.random.default_rng(2)
    for form in ("R1", "R2"):
        _, d = _tiny(form)
        E = rng.standard_normal((d.N, 3))
        L = rng.standard_normal((d.N, 3))
        lhs = np.sum(L[d.fem_grid] * d.divdiv(E))
        rhs = np.sum(E[d.fem_grid] * d.divdiv_T(L))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs), form
    # R2 is symmetric on fields supported on the FEM-owned nodes; R1 is not
    own = np.zeros(d.N, dtype=bool)
    own[d.fem_grid[d.fem_owned]] = True
    E[~own] = 0.0
    L[~own] = 0.0
    for form, sym in (("R2", True), ("R1", False)):
        _, d = _tiny(form)
        a = np.sum(L[d.fem_grid] * d.divdiv(E))
        b = np.sum(E[d.fem_grid] * d.divdiv(L))
        assert (abs(a - b) <= 1e-12 * abs(a)) == sym, form


def test_adjoint_dot_product_r2():
    _, d = _tiny("R2")
    rng = np.random.default_rng(3)
    nt = 20
    F = rng.standard_normal((nt, d.N, 3))
    fw = forward(d, force=lambda k: F[k], n_steps=nt)
    R = rng.standard_normal((nt, len(d.det), 3))
    ag = adjoint_gradient(d, R, fw, keep_lambda=True)
    lhs = np.sum(R * fw["traces"])
    assert abs(lhs + np.sum(ag["lambda"] * F)) <= 1e-12 * abs(lhs)


def _fd_check(form):
    w, d = _tiny(form)
    src = w.sources[0]
    eobs = forward(d, src)["traces"] * 0.9
    fw = forward(d, src)
    _, cot = loss_and_cotangent(fw["traces"], eobs)
    ag = adjoint_gradient(d, cot, fw)

    def J(eps):
        dd = Discretization(w.desc, divdiv_form=form).set_coefficients(eps, w.sigma)
        return loss_and_cotangent(forward(dd, src)["traces"], eobs)[0]

    fd = np.zeros(d.n_fem)
    for i in np.nonzero(d.fem_free)[0]:
        e = w.eps.copy()
        e[i] += 1e-5
        jp = J(e)
        e[i] -= 2e-5
        fd[i] = (jp - J(e)) / 2e-5
    return d, ag, fd


def test_paper_formula_is_the_exact_gradient_of_r2():
    d, ag, fd = _fd_check("R2")
    free = d.fem_free
    assert np.all(np.abs(ag["g_eps_paper"][free] - fd[free]) <= 1e-4 * np.abs(fd[free]))
    np.testing.assert_array_equal(ag["g_eps"], ag["g_eps_paper"])


def test_paper_formula_differs_from_the_exact_r1_gradient():
    d, ag, fd = _fd_check("R1")
    free = d.fem_free
    assert np.all(np.abs(ag["g_eps"][free] - fd[free]) <= 1e-4 * np.abs(fd[free]))
    rel = np.linalg.norm(ag["g_eps_paper"] - ag["g_eps"]) / np.linalg.norm(ag["g_eps"])
    assert rel > 1e-3


# ---- the smoothing function z of eq. tikhonov_functional -----------------------------------

def test_taper_shape():
    from oracle.solver import taper
    dt, nt, delta = 0.01, 200, 0.5
    z = taper(nt, dt, delta)
    t = dt * np.arange(1, nt + 1)
    T = nt * dt
    assert np.all(z[t <= T - delta + 1e-12] == 1.0) and z[-1] == 0.0
    assert np.all(np.diff(z) <= 0) and np.all((z >= 0) & (z <= 1))
    # C1 at both ends of the ramp: one-sided slopes vanish (second order in dt)
    assert abs(z[-1] - z[-2]) <= 2 * (np.pi / delta) ** 2 * dt ** 2
    k = int(np.searchsorted(t, T - delta + 1e-12))
    assert abs(z[k] - z[k - 1]) <= 2 * (np.pi / delta) ** 2 * dt ** 2
    np.testing.assert_array_equal(taper(nt, dt, 0.0), np.ones(nt))


def test_weighted_misfit_gradient_matches_central_differences():
    """With z the adjoint source is z_n r^n: the gradient matches differences of the weighted J."""
    from oracle.solver import taper
    w, d = _tiny("R1")
    src = w.sources[0]
    eobs = forward(d, src)["traces"] * 0.9
    z = taper(w.desc.n_steps, w.desc.dt, 0.4 * w.desc.n_steps * w.desc.dt)
    fw = forward(d, src)
    J0, cot = loss_and_cotangent(fw["traces"], eobs, z)
    J1, _ = loss_and_cotangent(fw["traces"], eobs)
    assert J0 < J1
    ag = adjoint_gradient(d, cot, fw)

    def J(eps):
        dd = Discretization(w.desc).set_coefficients(eps, w.sigma)
        return loss_and_cotangent(forward(dd, src)["traces"], eobs, z)[0]

    for i in np.nonzero(d.fem_free)[0][:3]:
        e = w.eps.copy()
        e[i] += 1e-5
        jp = J(e)
        e[i] -= 2e-5
        fd = (jp - J(e)) / 2e-5
        assert abs(ag["g_eps"][i] - fd) <= 1e-4 * abs(fd)
    # unweighted cotangent would not match the weighted J
    ag1 = adjoint_gradient(d, loss_and_cotangent(fw["traces"], eobs)[1], fw)
    assert np.linalg.norm(ag1["g_eps"] - ag["g_eps"]) > 1e-2 * np.linalg.norm(ag["g_eps"])
