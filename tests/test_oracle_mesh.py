"""Pins of the oracle on general (locally refined) FEM meshes.

The refined meshes are those of the paper's box "ACGA" after one refinement by eq. meshref on
the uniform starting mesh: marked cells get their centre as a node and their six Kuhn
tetrahedra bisected across the main diagonal (synth.refined_mesh).  Pinned here:

* special case: the Kuhn split passed as a general mesh is the default discretisation
  (operators, traces, gradient to rounding);
* invariants on a refined mesh: the adjoint dot-product test (exact transpose), conservation of
  the discrete energy for the symmetric form R2 with variable eps in a closed box, and the exact
  balance identity (R2) with conductivity, absorbing faces and a source;
* brute force: central differences of J on a tiny refined mesh at free lattice nodes and at
  inserted centres, per node <= 1e-4;
* the lumped mass of an inserted centre (|K|/4 over its twelve tetrahedra = h^3/4) and the
  fill of the box (volumes sum to it).
"""

import math

import numpy as np
import pytest

import synth
from oracle import solver as osolver
from oracle.discretization import Discretization


def _refined(name="tiny", beta=0.5, steps=None):
    w = synth.small(name)
    if steps:
        w.desc.n_steps = steps
    marks = synth.meshref_marks(w.desc, w.eps, beta)
    mesh = synth.refined_mesh(w.desc, marks)
    eps = synth.refined_values(w.desc, marks, w.eps)
    sig = synth.refined_values(w.desc, marks, w.sigma)
    return w, marks, mesh, eps, sig


def stable_dt(d, safety=0.8, iters=200, seed=0):
    """The explicit scheme's step limit 2 / sqrt(lambda_max(M_eps^-1 A)) (power iteration), times
    a safety factor, and never above the finite-difference region's 0.5 h / sqrt(3)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((d.N, 3))
    lam = 0.0
    for _ in range(iters):
        u = d.apply_A(v) / d.M_eps[:, None]
        lam = float(np.linalg.norm(u) / np.linalg.norm(v))
        v = u / np.linalg.norm(u)
    return min(safety * 2.0 / math.sqrt(lam), 0.5 * d.h / math.sqrt(3.0))


def test_kuhn_split_as_a_general_mesh_is_the_default():
    w = synth.small("ragged")
    none = np.zeros(int(np.prod(w.desc.fem_cells)), dtype=bool)
    mesh = synth.refined_mesh(w.desc, none)
    d0 = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    d1 = Discretization(w.desc, mesh=mesh).set_coefficients(w.eps, w.sigma)
    E = np.random.default_rng(1).standard_normal((d0.N, 3))
    a0, a1 = d0.apply_A(E), d1.apply_A(E)
    assert np.abs(a0 - a1).max() <= 1e-13 * np.abs(a0).max()
    assert np.abs(d0.apply_AT(E) - d1.apply_AT(E)).max() <= 1e-13 * np.abs(a0).max()
    f0 = osolver.forward(d0, w.sources[0], n_steps=40)
    f1 = osolver.forward(d1, w.sources[0], n_steps=40)
    assert np.abs(f0["traces"] - f1["traces"]).max() <= 1e-12 * np.abs(f0["traces"]).max()


def test_centres_masses_and_box_fill():
    w, marks, mesh, eps, sig = _refined()
    assert marks.sum() > 0
    d = Discretization(w.desc, mesh=mesh)
    centres = d.m_fem_lumped[d.n_fem - d.n_extra:]
    assert np.allclose(centres, w.desc.h ** 3 / 4, rtol=1e-13)
    assert abs(d.vol.sum() - np.prod(w.desc.fem_cells) * w.desc.h ** 3) <= 1e-12 * d.vol.sum()
    assert d.fem_free[d.n_fem - d.n_extra:].all()


def test_adjoint_dot_product_on_a_refined_mesh():
    w, marks, mesh, eps, sig = _refined()
    d = Discretization(w.desc, mesh=mesh).set_coefficients(eps, sig)
    w.desc.dt = stable_dt(d)
    d = Discretization(w.desc, mesh=mesh).set_coefficients(eps, sig)
    rng = np.random.default_rng(2)
    nt = 25
    F = rng.standard_normal((nt, d.N, 3))
    fw = osolver.forward(d, force=lambda k: F[k], n_steps=nt)
    R = rng.standard_normal((nt, len(d.det), 3))
    ag = osolver.adjoint_gradient(d, R, fw, keep_lambda=True)
    lhs = np.sum(R * fw["traces"])
    assert abs(lhs + np.sum(ag["lambda"] * F)) <= 1e-12 * abs(lhs)


def test_energy_conserved_and_balanced_on_a_refined_mesh():
    w, marks, mesh, eps, sig = _refined()
    w.desc.absorbing_faces = 0
    d = Discretization(w.desc, mesh=mesh, divdiv_form="R2").set_coefficients(eps, np.zeros_like(sig))
    w.desc.dt = stable_dt(d)
    d = Discretization(w.desc, mesh=mesh, divdiv_form="R2").set_coefficients(eps, np.zeros_like(sig))
    rng = np.random.default_rng(3)
    f0 = rng.standard_normal((d.N, 3))
    f1 = rng.standard_normal((d.N, 3))
    fw = osolver.forward(d, force=lambda k: np.zeros((d.N, 3)), n_steps=60, initial=(f0, f1))
    e = fw["energy"]
    assert np.abs(e - e[0]).max() <= 1e-12 * abs(e[0])
    # with conductivity, absorption and a source: the exact balance identity
    w.desc.absorbing_faces = synth.FACE_TOP | synth.FACE_BOTTOM
    d2 = Discretization(w.desc, mesh=mesh, divdiv_form="R2").set_coefficients(eps, sig)
    fb = osolver.forward(d2, w.sources[0], n_steps=60)
    assert np.abs(fb["balance"]).max() <= 1e-12 * np.abs(fb["energy"]).max()


def test_gradient_matches_central_differences_on_a_refined_mesh():
    w, marks, mesh, eps, sig = _refined()
    d = Discretization(w.desc, mesh=mesh).set_coefficients(eps, sig)
    w.desc.dt = stable_dt(d)
    src = w.sources[0]

    def solve(e, s):
        return osolver.forward(Discretization(w.desc, mesh=mesh).set_coefficients(e, s), src)

    eobs = solve(eps, sig)["traces"] * 0.9
    d = Discretization(w.desc, mesh=mesh).set_coefficients(eps, sig)
    fw = osolver.forward(d, src)
    _, cot = osolver.loss_and_cotangent(fw["traces"], eobs)
    ag = osolver.adjoint_gradient(d, cot, fw)
    free = np.nonzero(d.fem_free)[0]
    centres = free[free >= d.n_fem - d.n_extra]
    lattice = free[free < d.n_fem - d.n_extra]
    assert len(centres) > 0
    delta = 1e-5
    # the nodes of each kind where the gradient is largest (elsewhere the signal is at the level
    # of the finite differences' rounding)
    mag = np.abs(ag["g_eps"]) + np.abs(ag["g_sigma"])
    pick = list(lattice[np.argsort(-mag[lattice])[:2]]) + list(centres[np.argsort(-mag[centres])[:2]])
    for i in [int(v) for v in pick]:
        for which in ("eps", "sigma"):
            base = eps if which == "eps" else sig
            vals = []
            for sgn in (1, -1):
                c = base.copy()
                c[i] += sgn * delta
                t = solve(c, sig)["traces"] if which == "eps" else solve(eps, c)["traces"]
                vals.append(osolver.loss_and_cotangent(t, eobs)[0])
            fd = (vals[0] - vals[1]) / (2 * delta)
            g = ag["g_eps"][i] if which == "eps" else ag["g_sigma"][i]
            assert abs(g - fd) <= 1e-4 * max(abs(fd), 1e-12), (i, which, g, fd)


def test_meshes_that_do_not_fill_the_box_are_refused():
    w = synth.small("tiny")
    none = np.zeros(int(np.prod(w.desc.fem_cells)), dtype=bool)
    ex, tets = synth.refined_mesh(w.desc, none)
    with pytest.raises(ValueError):
        Discretization(w.desc, mesh=(ex, tets[:-1]))
