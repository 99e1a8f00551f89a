"""Pins of the oracle's spatial operators against closed forms and invariants.

* The P1 stiffness of the Kuhn split equals h times the 7-point stencil on
  every FEM-owned row (a textbook special case), and the lumped mass is h^3.
* Stiffness and div-div are second-order consistent with -Laplace(E) and
  -grad div((eps - 1) E) (the spatial part of the box "Forward problem",
  eq. forward_prob) on smooth fields: the error drops by 4 per halving of h.
* With a constant eps, M_eps^{-1} A moves longitudinal plane waves at speed 1 and
  transverse ones at 1/sqrt(eps) (closed form of eq. forward_prob), to second order, for
  both div-div forms: this also fixes the eps in the mass matrix.
* The transposed operator used by the adjoint is the exact transpose.
* Lumped masses and face masses add up to the box volume and face areas.
"""

import math

import numpy as np
import pytest
import sympy

import synth
from oracle.discretization import Discretization


def _desc(nc, h=None, n_outer=None):
    h = h or 2.0 / nc
    n_outer = n_outer or (nc + 4,) * 3
    return synth.ProblemDesc(n_outer=n_outer, h=h, origin=(-2 * h,) * 3, fem_lo=(2, 2, 2),
                             fem_cells=(nc,) * 3, dt=0.1 * h, n_steps=1)


def test_kuhn_stiffness_is_seven_point_on_fem_rows():
    d = Discretization(synth.small("ragged").desc)
    rows = d.fem_grid[d.fem_owned]
    diff = (d.K_fem - d.K_fd)[rows]
    assert abs(diff).max() <= 1e-13 * d.h
    # and the 7-point row has exactly 6 neighbours of weight -h
    r = d.K_fem[rows[len(rows) // 2]].toarray().ravel()
    nz = np.sort(r[np.abs(r) > 1e-12 * d.h])
    assert len(nz) == 7 and np.allclose(nz[:6], -d.h) and math.isclose(nz[6], 6 * d.h)


def test_lumped_masses():
    d = Discretization(synth.small("ragged").desc)
    own = d.fem_owned
    assert np.allclose(d.m_fem_lumped[own], d.h ** 3, rtol=1e-13)
    # Kuhn lumping on the FEM box's edges/corners is not the mirror lumping
    vals = set(np.round(d.m_fem_lumped[~own] / d.h ** 3, 9))
    assert {0.083333333, 0.166666667, 0.25, 0.333333333, 0.5} <= vals
    # the grid masses tile the outer box exactly
    vol = np.prod((d.nvec - 1) * d.h)
    assert math.isclose(d.m.sum(), vol, rel_tol=1e-12)
    assert math.isclose(d.vol.sum(), np.prod(np.array(d.desc.fem_cells) * d.h), rel_tol=1e-12)


def test_face_masses_tile_faces():
    d = Discretization(synth.small("ragged").desc)
    ext = (d.nvec - 1) * d.h
    for bit, (a, _s) in {1: (2, 1), 2: (2, 0), 4: (0, 0), 8: (0, 1), 16: (1, 0), 32: (1, 1)}.items():
        area = np.prod([ext[b] for b in range(3) if b != a])
        assert math.isclose(d.face_mass[bit].sum(), area, rel_tol=1e-12)


def _consistency_errors(nc):
    X, Y, Z = sympy.symbols("x y z")
    eps_s = 1 + 0.5 * sympy.sin(1.3 * X + 0.4) * sympy.cos(0.7 * Y - 0.2) * sympy.sin(0.9 * Z + 1.1)
    E_s = [sympy.cos(1.1 * X + 0.5 * Y - 0.3 * Z), sympy.sin(0.6 * X - 0.8 * Y + 0.4 * Z + 0.3),
           sympy.cos(0.2 * X + 0.9 * Y + 1.2 * Z)]
    div = sum(sympy.diff((eps_s - 1) * E_s[c], v) for c, v in enumerate((X, Y, Z)))
    graddiv = [-sympy.diff(div, v) for v in (X, Y, Z)]
    lap = [-sum(sympy.diff(E_s[c], v, 2) for v in (X, Y, Z)) for c in range(3)]
    f = lambda e: sympy.lambdify((X, Y, Z), e, "numpy")  # noqa: E731
    d = Discretization(_desc(nc))
    x = d.x
    xf = x[d.fem_grid]
    d.eps = f(eps_s)(xf[:, 0], xf[:, 1], xf[:, 2])   # operator-only test: no layer constraint
    E = np.stack([f(e)(x[:, 0], x[:, 1], x[:, 2]) for e in E_s], axis=1)
    sel = d.fem_layer >= 2
    xs = x[d.fem_grid[sel]]
    m = d.m_fem_lumped[sel][:, None]
    ref_dd = np.stack([f(e)(xs[:, 0], xs[:, 1], xs[:, 2]) for e in graddiv], axis=1) * m
    ref_k = np.stack([f(e)(xs[:, 0], xs[:, 1], xs[:, 2]) for e in lap], axis=1) * m
    dd = d.divdiv(E)[sel]
    kk = (d.K_fem @ E)[d.fem_grid[sel]]
    return (np.abs(dd - ref_dd).max() / np.abs(ref_dd).max(), np.abs(kk - ref_k).max() / np.abs(ref_k).max())


def test_second_order_consistency_of_stiffness_and_divdiv():
    e8 = _consistency_errors(8)
    e16 = _consistency_errors(16)
    for a, b in zip(e8, e16):
        assert 3.5 < a / b < 4.5, (a, b)
    assert e16[0] < 0.02 and e16[1] < 0.002


def test_transpose_operator_is_exact_transpose():
    w = synth.small("ragged")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((d.N, 3))
    y = rng.standard_normal((d.N, 3))
    lhs = np.sum(d.apply_A(x) * y)
    rhs = np.sum(x * d.apply_AT(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # non-trivially non-symmetric once eps varies
    assert abs(np.sum(d.apply_A(x) * y) - np.sum(d.apply_A(y) * x)) > 1e-6 * abs(lhs)


def test_detector_counts_and_order():
    d = Discretization(synth.c1().desc)
    assert len(d.det) == 25 ** 3 - 23 ** 3 == 3458
    assert np.all(np.diff(d.det) > 0)
    w = synth.small("ragged")
    d = Discretization(w.desc)
    nx, ny, nz = w.desc.n_outer
    ijk = d.ijk[d.det]
    on = (ijk[:, 2] == nz - 1) | (ijk[:, 0] == 0) | (ijk[:, 1] == ny - 1)
    assert on.all() and len(d.det) == nx * ny + (nz - 1) * (ny + nx - 1)


def test_coefficient_constraint_enforced():
    w = synth.small("tiny")
    d = Discretization(w.desc)
    bad = w.eps.copy()
    bad[d.fem_layer == 1] = 2.0
    with pytest.raises(ValueError):
        d.set_coefficients(bad, w.sigma)
    bad = w.eps.copy()
    bad[d.fem_free] = 0.5
    with pytest.raises(ValueError):
        d.set_coefficients(bad, w.sigma)


def _wave_speed_errors(nc, eps_c=4.0, form="R1"):
    """Closed form: in a constant medium eps, eps E_tt - Laplace E - (eps - 1) grad div E = 0 has
    longitudinal plane waves at speed 1 (omega^2 = |k|^2) and transverse ones at 1/sqrt(eps)
    (omega^2 = |k|^2 / eps).  On free FEM rows, M_eps^{-1} A applied to cos(k.x + 0.3) times
    the unit vector along k (or across it) must give omega^2 times the field."""
    d = Discretization(_desc(nc), divdiv_form=form)
    n = d.n_fem
    d.set_coefficients(np.ones(n), np.zeros(n))
    d.eps = np.full(n, eps_c)              # operator-only test: eps constant on every FEM node
    eg = np.ones(d.N)
    eg[d.fem_grid] = eps_c
    M = d.m * eg
    k = np.array([0.9, -0.5, 0.7])
    kk = float(k @ k)
    kh = k / math.sqrt(kk)
    t = np.cross(kh, [0.0, 0.0, 1.0])
    t /= np.linalg.norm(t)
    ph = np.cos(d.x @ k + 0.3)
    rows = d.fem_grid[d.fem_layer >= 2]
    out = []
    for u, w2 in ((ph[:, None] * kh[None, :], kk), (ph[:, None] * t[None, :], kk / eps_c)):
        r = d.apply_A(u)[rows] / M[rows][:, None]
        out.append(float(np.abs(r - w2 * u[rows]).max() / (w2 * np.abs(u[rows]).max())))
    return out


def test_longitudinal_and_transverse_wave_speeds():
    for form in ("R1", "R2"):
        e8, e16 = _wave_speed_errors(8, form=form), _wave_speed_errors(16, form=form)
        for a, b in zip(e8, e16):
            assert 3.6 < a / b < 4.4, (form, a, b)
        assert max(e16) < 3e-3, (form, e16)
