"""Pins of the oracle's refinement step of box "ACGA" (oracle/acga.py): marking by eq. meshref,
the refined mesh and the interpolation onto it.

* marks: brute force on hand-built media (a spike of eps at one free node marks exactly the
  cells around it; eps and sigma spikes at different nodes mark nothing, since both
  inequalities must hold; sigma = 0 leaves the sigma test vacuous), only cells with
  FEM-owned corners, beta = 0 marks every such cell;
* the mesh: nothing marked gives the Kuhn split (operators to 1e-13); a refined mesh is
  conforming (each interior triangle in exactly two tetrahedra, each boundary triangle once
  and on the box surface), non-degenerate, fills the box, and a marked cell's twelve
  tetrahedra have volume h^3/12 each;
* interpolation: exact (to rounding) for trilinear functions, whose value at a cell centre
  is the mean of the corners; old nodes keep their values;
* the loop's stitching: with nothing marked its second level is the CGA on the uniform mesh
  from the first level's result (the CGA itself is pinned in tests/test_oracle_cga.py, the
  solves on refined meshes in tests/test_oracle_mesh.py).
"""

import itertools

import numpy as np
import pytest

import synth
from oracle import acga
from oracle.discretization import Discretization


def _lat(desc):
    return tuple(int(c) + 1 for c in desc.fem_cells)


def _node(desc, i, j, k):
    nx, ny, _ = _lat(desc)
    return i + nx * (j + ny * k)


def test_marks_of_a_single_spike():
    w = synth.small("skinlet")
    n = int(np.prod(_lat(w.desc)))
    eps, sig = np.ones(n), np.zeros(n)
    i, j, k = 10, 11, 12
    eps[_node(w.desc, i, j, k)] = 5.0
    m = acga.marks(w.desc, eps, sig, 0.5, 0.5).reshape(tuple(int(c) for c in w.desc.fem_cells)[::-1])
    expect = np.zeros_like(m)
    for dk, dj, di in itertools.product((0, 1), repeat=3):
        expect[k - dk, j - dj, i - di] = True
    assert np.array_equal(m, expect)


def test_marks_need_both_inequalities():
    w = synth.small("skinlet")
    n = int(np.prod(_lat(w.desc)))
    eps, sig = np.ones(n), np.zeros(n)
    eps[_node(w.desc, 10, 11, 12)] = 5.0
    sig[_node(w.desc, 5, 6, 7)] = 2.0
    assert not acga.marks(w.desc, eps, sig, 0.5, 0.5).any()
    sig[_node(w.desc, 10, 11, 12)] = 2.0
    assert acga.marks(w.desc, eps, sig, 0.5, 0.5).sum() == 8


def test_marks_respect_the_overlap_layers():
    w = synth.small("ragged")
    n = int(np.prod(_lat(w.desc)))
    c = [int(v) for v in w.desc.fem_cells]
    m = acga.marks(w.desc, np.ones(n), np.zeros(n), 0.0, 0.0)
    assert m.sum() == (c[0] - 2) * (c[1] - 2) * (c[2] - 2)
    mm = m.reshape(c[::-1])
    assert not mm[0].any() and not mm[-1].any() and not mm[:, 0].any() and not mm[:, :, -1].any()


def test_nothing_marked_is_the_kuhn_split():
    w = synth.small("ragged")
    none = np.zeros(int(np.prod(w.desc.fem_cells)), dtype=bool)
    d0 = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    d1 = Discretization(w.desc, mesh=acga.refine(w.desc, none)).set_coefficients(w.eps, w.sigma)
    E = np.random.default_rng(3).standard_normal((d0.N, 3))
    a0 = d0.apply_A(E)
    assert np.abs(a0 - d1.apply_A(E)).max() <= 1e-13 * np.abs(a0).max()


def test_refined_mesh_is_conforming_and_fills_the_box():
    w = synth.small("skinlet")
    m = acga.marks(w.desc, w.eps, w.sigma, 0.3, 0.0)
    assert 0 < m.sum() < m.size
    xyz, tets = acga.refine(w.desc, m)
    h = w.desc.h
    nx, ny, nz = _lat(w.desc)
    lat = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    lat = lat.transpose(2, 1, 0, 3).reshape(-1, 3).astype(np.float64)
    pts = np.concatenate([lat, (xyz - np.asarray(w.desc.origin)) / h - np.asarray(w.desc.fem_lo)])
    P = pts[tets]
    vol = np.abs(np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6.0
    assert vol.min() > 1e-9
    assert abs(vol.sum() - np.prod(w.desc.fem_cells)) <= 1e-9 * vol.sum()
    # in units of h: a Kuhn tetrahedron has volume 1/6, each of its halves 1/12
    assert np.all(np.isclose(vol, 1 / 6) | np.isclose(vol, 1 / 12))
    assert np.isclose(vol, 1 / 12).sum() == 12 * m.sum()
    faces = {}
    for t in tets:
        for f in itertools.combinations(sorted(int(v) for v in t), 3):
            faces[f] = faces.get(f, 0) + 1
    cells = np.asarray(w.desc.fem_cells, dtype=np.float64)
    for f, cnt in faces.items():
        assert cnt in (1, 2)
        if cnt == 1:   # a boundary triangle lies in a face of the box
            q = pts[list(f)]
            assert any(np.allclose(q[:, a], 0.0) or np.allclose(q[:, a], cells[a]) for a in range(3))


def test_interpolation_is_exact_for_trilinear_functions():
    w = synth.small("ragged")
    m = acga.marks(w.desc, w.eps, w.sigma, 0.4, 0.0)
    nx, ny, nz = _lat(w.desc)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = lambda x, y, z: 0.3 + 1.1 * x - 0.7 * y + 0.2 * z + 0.05 * x * y - 0.03 * y * z + 0.02 * x * z + 0.01 * x * y * z
    vals = f(x, y, z).reshape(-1)
    out = acga.interpolate(w.desc, m, vals)
    assert np.array_equal(out[:vals.size], vals)
    cz, cy, cx = np.nonzero(m.reshape(tuple(int(c) for c in w.desc.fem_cells)[::-1]))
    exact = f(cx + 0.5, cy + 0.5, cz + 0.5)
    assert np.abs(out[vals.size:] - exact).max() <= 1e-12 * np.abs(exact).max()


def test_loop_with_nothing_marked_continues_on_the_uniform_mesh():
    """The stitching of the loop: with beta_eps > 1 no cell is marked, so the second level must
    be the CGA on the (uniform) mesh started from, and centred on, the first level's result,
    with the same observations."""
    from oracle.cga import cga
    from oracle.solver import forward
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    n = d.n_fem
    prm = dict(gamma_eps=0.5, gamma_sig=0.5, p=0.5, alpha_eps=0.5, alpha_sig=0.05, eps_max=8.0, sig_max=2.0)
    r = acga.acga(w.desc, [src], eobs, np.ones(n), np.zeros(n), prm, 2, 1.5, 0.0)
    assert not r["marks"].any() and len(r["mesh"][0]) == 0
    h1 = cga(Discretization(w.desc), [src], eobs, r["eps_coarse"], r["sig_coarse"], prm, 2)
    assert r["eps_coarse"] is not None and np.any(r["eps_coarse"] != 1.0)
    for a, b in zip(r["fine"], h1):
        for f in ("eps", "sig"):
            assert a[f]["grad_norm"] == pytest.approx(b[f]["grad_norm"], rel=1e-12)
            assert np.allclose(a[f]["coef"], b[f]["coef"], rtol=1e-12, atol=1e-14)
