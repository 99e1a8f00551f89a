"""Pins of the oracle's box "ACGA" (oracle/acga.py): marking by eq. meshref, the refined
meshes, the interpolation onto them and the loop.

* marks: brute force on hand-built media on K_h^0 (a spike of eps at one free node marks
  exactly the elements around it, and refines the eight cells around it; eps and sigma spikes
  at different nodes mark nothing, since both inequalities must hold; sigma = 0 leaves the
  sigma test vacuous); beta = 0 refines every cell with FEM-owned corners and none in the
  overlap layers; on a refined mesh a constant field marks exactly the elements whose diameter
  h_K is within beta of the largest (the mesh function of eq. meshfunction enters);
* the first refinement of K_h^0 is the cell-centre rule of the mesh generator synth.refined_mesh
  (an independent implementation), element for element;
* nothing marked gives the Kuhn split (operators to 1e-13);
* three successive refinements: conforming (each interior triangle in exactly two elements,
  each boundary triangle once and on the box surface), filling the box, every split halving an
  element's volume, elements that do not degenerate, midpoints strictly inside, elements with
  a vertex in layer 0 never split;
* interpolation: the refined mesh carries the same piecewise-linear function (evaluated at
  random points on both meshes, to 1e-12), old nodes keep their values;
* the loop: with nothing marked the second level is the CGA on the uniform mesh from the
  first level's result (the CGA itself is pinned in tests/test_oracle_cga.py, the solves on
  refined meshes in tests/test_oracle_mesh.py); the stop test's grouping; a loop with loose
  tolerances stops after its first refinement.
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


def _cells(desc):
    return tuple(int(c) for c in desc.fem_cells)


def _cell_of_centres(desc, ref):
    """Cells whose centres the refinement inserted (first refinement of K_h^0)."""
    P = acga.node_coords(desc, ref["mesh"][0])[ref["n_old"]:]
    c = np.floor(P).astype(np.int64)
    assert np.allclose(P - c, 0.5)
    cx, cy, _ = _cells(desc)
    return c[:, 0] + cx * (c[:, 1] + cy * c[:, 2])


def test_marks_of_a_single_spike():
    w = synth.small("skinlet")
    n = int(np.prod(_lat(w.desc)))
    eps, sig = np.ones(n), np.zeros(n)
    i, j, k = 10, 11, 12
    v = _node(w.desc, i, j, k)
    eps[v] = 5.0
    m = acga.marks(w.desc, None, eps, sig, 0.5, 0.5)
    _, tets = acga.kuhn_mesh(w.desc)
    assert np.array_equal(m, (tets == v).any(axis=1))
    ref = acga.refine(w.desc, None, m)
    cx, cy, _ = _cells(w.desc)
    got = sorted(int(c) for c in _cell_of_centres(w.desc, ref))
    want = sorted((i - di) + cx * ((j - dj) + cy * (k - dk)) for di, dj, dk in itertools.product((0, 1), repeat=3))
    assert got == want


def test_marks_need_both_inequalities():
    w = synth.small("skinlet")
    n = int(np.prod(_lat(w.desc)))
    eps, sig = np.ones(n), np.zeros(n)
    eps[_node(w.desc, 10, 11, 12)] = 5.0
    sig[_node(w.desc, 5, 6, 7)] = 2.0
    assert not acga.marks(w.desc, None, eps, sig, 0.5, 0.5).any()
    sig[_node(w.desc, 10, 11, 12)] = 2.0
    m = acga.marks(w.desc, None, eps, sig, 0.5, 0.5)
    assert m.sum() == 24      # the elements around an interior lattice node
    assert len(acga.refine(w.desc, None, m)["edges"]) == 8


def test_refinement_respects_the_overlap_layers():
    w = synth.small("ragged")
    n = int(np.prod(_lat(w.desc)))
    c = _cells(w.desc)
    m = acga.marks(w.desc, None, np.ones(n), np.zeros(n), 0.0, 0.0)
    assert m.all()
    ref = acga.refine(w.desc, None, m)
    cells = _cell_of_centres(w.desc, ref)
    assert len(cells) == (c[0] - 2) * (c[1] - 2) * (c[2] - 2)
    ci, cj, ck = cells % c[0], (cells // c[0]) % c[1], cells // (c[0] * c[1])
    assert ci.min() == 1 and ci.max() == c[0] - 2 and cj.min() == 1 and ck.max() == c[2] - 2


def test_marks_use_the_element_diameter():
    """After one refinement the halves of a refined cell's elements have diameter sqrt(2) h
    against sqrt(3) h for the untouched Kuhn elements: with a constant field, beta = 0.9 marks
    exactly the untouched elements and beta = 0.8 (< sqrt(2/3)) marks all."""
    w = synth.small("tiny")
    n = int(np.prod(_lat(w.desc)))
    m0 = acga.marks(w.desc, None, np.ones(n), np.zeros(n), 0.0, 0.0)
    ref = acga.refine(w.desc, None, m0)
    ext, tets = ref["mesh"]
    f = np.full(n + len(ext), 2.0)
    hk = acga.diameters(acga.node_coords(w.desc, ext), tets)
    assert np.allclose(np.unique(np.round(hk, 12)), [np.sqrt(2.0), np.sqrt(3.0)])
    m = acga.marks(w.desc, ref["mesh"], f, f, 0.9, 0.0)
    assert np.array_equal(m, np.isclose(hk, np.sqrt(3.0)))
    assert acga.marks(w.desc, ref["mesh"], f, f, 0.8, 0.0).all()


def test_first_refinement_is_the_cell_centre_rule():
    w = synth.small("ragged")
    rng = np.random.default_rng(5)
    _, tets = acga.kuhn_mesh(w.desc)
    m = rng.random(len(tets)) < 0.05
    ref = acga.refine(w.desc, None, m)
    cells = np.zeros(int(np.prod(_cells(w.desc))), dtype=bool)
    cells[_cell_of_centres(w.desc, ref)] = True
    # the cells that hold a marked element and have all their corners FEM-owned
    lay = acga.node_layers(w.desc, int(np.prod(_lat(w.desc))))
    want = np.zeros_like(cells)
    want[np.nonzero(m)[0] // 6] = True
    for cid in np.nonzero(want)[0]:
        corners = set(int(v) for v in tets[6 * cid:6 * cid + 6].reshape(-1))
        want[cid] = all(lay[v] >= 1 for v in corners)
    assert np.array_equal(cells, want)
    ext, tt = synth.refined_mesh(w.desc, cells)
    assert np.array_equal(ref["mesh"][1], tt.astype(np.int64))
    assert np.abs(ref["mesh"][0] - ext).max() <= 1e-14 * max(1.0, np.abs(ext).max())


def test_nothing_marked_is_the_kuhn_split():
    w = synth.small("ragged")
    ref = acga.refine(w.desc, None, np.zeros(6 * int(np.prod(_cells(w.desc))), dtype=bool))
    assert len(ref["edges"]) == 0
    d0 = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    d1 = Discretization(w.desc, mesh=ref["mesh"]).set_coefficients(w.eps, w.sigma)
    E = np.random.default_rng(3).standard_normal((d0.N, 3))
    a0 = d0.apply_A(E)
    assert np.abs(a0 - d1.apply_A(E)).max() <= 1e-13 * np.abs(a0).max()


def _three_refinements(name="tiny"):
    """Three successive refinements driven by a smooth bump (the elements near its peak)."""
    w = synth.small(name)
    mesh = None
    out = []
    c = np.asarray(_cells(w.desc), dtype=np.float64)
    for _ in range(3):
        ext = np.zeros((0, 3)) if mesh is None else mesh[0]
        P = acga.node_coords(w.desc, ext)
        f = np.exp(-np.sum((P - 0.45 * c) ** 2, axis=1) / (0.08 * c.min() ** 2))
        m = acga.marks(w.desc, mesh, f, f, 0.5, 0.0)
        ref = acga.refine(w.desc, mesh, m)
        out.append((mesh, m, ref))
        mesh = ref["mesh"]
    return w, out


def _faces(tets):
    faces = {}
    for t in tets:
        for f in itertools.combinations(sorted(int(v) for v in t), 3):
            faces[f] = faces.get(f, 0) + 1
    return faces


def _volumes(P, tets):
    return np.abs(np.einsum("ij,ij->i", P[tets[:, 1]] - P[tets[:, 0]],
                            np.cross(P[tets[:, 2]] - P[tets[:, 0]], P[tets[:, 3]] - P[tets[:, 0]]))) / 6.0


def test_successive_refinements_are_conforming_and_fill_the_box():
    w, levels = _three_refinements()
    cells = np.asarray(_cells(w.desc), dtype=np.float64)
    n_lat = int(np.prod(_lat(w.desc)))
    lay = acga.node_layers(w.desc, n_lat)
    for mesh, m, ref in levels:
        old_ext, old_tets = acga.kuhn_mesh(w.desc) if mesh is None else mesh
        ext, tets = ref["mesh"]
        assert len(ref["edges"]) > 0 and len(tets) > len(old_tets)
        P = acga.node_coords(w.desc, ext)
        assert np.all(P[n_lat:] > 0) and np.all(P[n_lat:] < cells)
        vol = _volumes(P, tets)
        assert abs(vol.sum() - np.prod(cells)) <= 1e-9 * vol.sum()
        # no element degenerates: volume against the cube of the diameter stays bounded below
        assert np.min(vol / acga.diameters(P, tets) ** 3) > 0.025
        # every split halves an element: the new volumes are old ones over powers of two
        vold = _volumes(acga.node_coords(w.desc, old_ext), old_tets)
        allowed = np.round(np.concatenate([vold / 2 ** k for k in range(4)]), 12)
        assert np.all(np.isin(np.round(vol, 12), allowed))
        # elements with a vertex in layer 0 are untouched
        touch0 = sorted(tuple(t) for t in old_tets.tolist() if any(v < n_lat and lay[v] == 0 for v in t))
        now0 = sorted(tuple(t) for t in tets.tolist() if any(v < n_lat and lay[v] == 0 for v in t))
        assert touch0 == now0
        for f, cnt in _faces(tets).items():
            assert cnt in (1, 2)
            if cnt == 1:
                q = P[list(f)]
                assert any(np.allclose(q[:, a], 0.0) or np.allclose(q[:, a], cells[a]) for a in range(3))


def _p1_eval(P, tets, values, pts):
    """The P1 function of (P, tets, values) at points: locate each point's element by its
    barycentric coordinates and combine the vertex values."""
    A = P[tets[:, 1:]] - P[tets[:, :1]]                       # rows: edge vectors from vertex 0
    inv = np.linalg.inv(np.transpose(A, (0, 2, 1)))           # maps x - p0 to (l1, l2, l3)
    out = np.empty(len(pts))
    for q, x in enumerate(pts):
        lam = np.einsum("tij,tj->ti", inv, x - P[tets[:, 0]])
        full = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
        t = int(np.argmax(full.min(axis=1)))
        assert full[t].min() >= -1e-12
        out[q] = float(full[t] @ values[tets[t]])
    return out


def test_interpolation_keeps_the_piecewise_linear_function():
    w, levels = _three_refinements()
    rng = np.random.default_rng(8)
    cells = np.asarray(_cells(w.desc), dtype=np.float64)
    pts = rng.random((150, 3)) * cells
    for mesh, m, ref in levels:
        old_ext, old_tets = acga.kuhn_mesh(w.desc) if mesh is None else mesh
        vals = rng.standard_normal(ref["n_old"])
        new = acga.interpolate(ref, vals)
        assert np.array_equal(new[:ref["n_old"]], vals)
        a = _p1_eval(acga.node_coords(w.desc, old_ext), old_tets, vals, pts)
        b = _p1_eval(acga.node_coords(w.desc, ref["mesh"][0]), ref["mesh"][1], new, pts)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def _loop_inputs():
    from oracle.solver import forward
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    prm = dict(gamma_eps=0.5, gamma_sig=0.5, p=0.5, alpha_eps=0.5, alpha_sig=0.05, eps_max=8.0, sig_max=2.0)
    return w, src, eobs, d.n_fem, prm


def test_loop_with_nothing_marked_continues_on_the_uniform_mesh():
    """With beta_eps > 1 no element is marked, so the second level must be the CGA on the
    (uniform) mesh started from, and centred on, the first level's result, with the same
    observations."""
    from oracle.cga import cga
    w, src, eobs, n, prm = _loop_inputs()
    r = acga.acga(w.desc, [src], eobs, np.ones(n), np.zeros(n), prm, 2, 1.5, 0.0, n_refine=1)
    l0, l1 = r["levels"]
    assert not l0["marks"].any() and len(l1["mesh"][0]) == 0
    assert np.any(l0["eps"] != 1.0)
    h1 = cga(Discretization(w.desc), [src], eobs, l0["eps"], l0["sigma"], prm, 2)
    for a, b in zip(l1["history"], h1):
        for f in ("eps", "sig"):
            assert a[f]["grad_norm"] == pytest.approx(b[f]["grad_norm"], rel=1e-12)
            assert np.allclose(a[f]["coef"], b[f]["coef"], rtol=1e-12, atol=1e-14)


def test_stop_test_grouping():
    th = dict(theta1_eps=1.0, theta1_sig=1.0, theta2_eps=1.0, theta2_sig=1.0)
    small, big = 0.5, 2.0
    assert acga.stop_test({"eps": small, "sig": big}, {"eps": big, "sig": small}, th)
    assert not acga.stop_test({"eps": big, "sig": big}, {"eps": small, "sig": small}, th)
    assert not acga.stop_test({"eps": small, "sig": small}, {"eps": big, "sig": big}, th)
    assert not acga.stop_test({"eps": small, "sig": small}, {"eps": small, "sig": small}, {})


def test_loop_stops_after_the_first_refinement_with_loose_tolerances():
    w, src, eobs, n, prm = _loop_inputs()
    th = dict(theta1_eps=1e9, theta1_sig=1e9, theta2_eps=1e9, theta2_sig=1e9)
    r = acga.acga(w.desc, [src], eobs, np.ones(n), np.zeros(n), prm, 1, 0.5, 0.0, n_refine=3, theta=th)
    assert len(r["levels"]) == 2 and r["levels"][1]["stop"]
    r = acga.acga(w.desc, [src], eobs, np.ones(n), np.zeros(n), prm, 1, 0.5, 0.0, n_refine=2)
    assert len(r["levels"]) == 3 and not r["levels"][2]["stop"]
    assert len(r["levels"][2]["mesh"][0]) > len(r["levels"][1]["mesh"][0]) > 0
