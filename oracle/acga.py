"""Adaptive conjugate gradient reconstruction (box "ACGA"), FP64.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the smoke check
and the benchmark's CPU baseline may use it; the HIP path shares no code with it.

Box "ACGA", for the meshes K_h^i, i = 0, 1, ...:
  1. the CGA on K_h^i (oracle.cga);
  2. mark the elements where eq. meshref holds for the reconstruction;
  3. refine them into K_h^{i+1}, interpolate eps_h, sigma_h (and E_obs) onto it;
  4. stop, or repeat from 1 on K_h^{i+1}.

Readings (where the paper leaves a choice):
  * K_h^0 is the uniform Kuhn split of the FEM box (six tetrahedra per cell);
  * step 2: h_K of eq. meshfunction is the element's diameter (its longest edge), and
    eps_h, sigma_h are nodal (P1) functions; an element K is marked when at one of its
    vertices v both h_K |eps(v)| >= beta_eps M_eps and h_K |sigma(v)| >= beta_sig M_sig hold,
    where M_f is the largest h_K' |f(v')| over all elements K' and their vertices v'.  On
    K_h^0 every h_K is the same and cancels;
  * step 3, longest-edge bisection with propagation: a marked element is bisected at its
    longest edge (among edges within 1e-9 of the longest, the one with the smaller (smaller,
    larger) pair of node indices), and so is every element around that edge, at the edge's
    midpoint, so the mesh stays conforming; before that, every element around the edge whose
    own longest edge is another one is bisected first, in the same way (recursively, in
    increasing element id), so that every element is always split at its longest edge, which
    keeps the elements from degenerating.  An edge is bisected only when every element
    around it has all its vertices FEM-owned (lattice layer >= 1), so the two overlap layers
    keep their lattice elements; a marked element whose propagation meets another edge stays
    as it is.  The marked elements are taken in element order (one already split is skipped);
    the k-th bisection's midpoint becomes node n + k (n: the nodes of K_h^i); an element
    split at edge (a, b), a < b, is replaced in the element list by its half with b replaced by
    the midpoint, then its half with a replaced by it (children get ids after all existing
    ones).  On K_h^0 the longest edge of every element is its cell's main diagonal, which lies
    in the cell's six elements only, so a cell is refined by inserting its centre and bisecting
    its six elements, exactly when one of its corners meets the rule;
  * step 3's interpolation: eps_h, sigma_h keep their values at the old nodes and take the
    mean of the bisected edge's endpoints at its midpoint (in bisection order: an endpoint
    may be an earlier midpoint), so the refined mesh carries the
    same piecewise-linear functions; E_obs lives on the outer grid's detectors, which the
    refinement of the FEM box does not touch, so its interpolation is the identity;
  * step 1 on K_h^{i+1} starts from the interpolated reconstruction, which is also its
    Tikhonov centre (the CGA's centre is its initial guess);
  * step 4 compares the CGA's result on K_h^{i+1} with the interpolated result of K_h^i
    (the same nodal functions would give a zero difference): stop when
    (|eps_{i+1} - eps_i| < theta1_eps or |sigma_{i+1} - sigma_i| < theta1_sig) and
    (|g_eps| < theta2_eps or |g_sig| < theta2_sig), with the lumped-mass L2 norms of
    K_h^{i+1} and g the last CGA gradients there; otherwise refine again, up to a given
    number of refinements.  The time step stays the same on every mesh (the paper refines in
    space only); the caller picks it below the finest mesh's limit.
"""

from __future__ import annotations

import math
from collections import defaultdict

import numpy as np

from .cga import cga
from .discretization import Discretization

# The six Kuhn tetrahedra of a cell: vertex 0 is the lowest corner, each following vertex one
# unit step along the next axis of the permutation, vertex 3 the highest corner.
PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
TIE = 1e-9


def kuhn_mesh(desc):
    """K_h^0: no extra nodes; per cell (lexicographic, x fastest) its six tetrahedra in PERMS
    order, in FEM-node indices (lattice nodes lexicographic)."""
    cells = [int(c) for c in desc.fem_cells]
    nx, ny = cells[0] + 1, cells[1] + 1
    tets = []
    for k in range(cells[2]):
        for j in range(cells[1]):
            for i in range(cells[0]):
                for perm in PERMS:
                    v = [np.array((i, j, k))]
                    for ax in perm:
                        step = np.zeros(3, dtype=np.int64)
                        step[ax] = 1
                        v.append(v[-1] + step)
                    tets.append([int(p[0] + nx * (p[1] + ny * p[2])) for p in v])
    return np.zeros((0, 3)), np.asarray(tets, dtype=np.int64)


def _mesh(desc, mesh):
    if mesh is None:
        return kuhn_mesh(desc)
    return np.asarray(mesh[0], dtype=np.float64).reshape(-1, 3), np.asarray(mesh[1], dtype=np.int64).reshape(-1, 4)


def node_coords(desc, extra):
    """Node positions in units of h from the FEM box's lower corner: lattice nodes, then the
    extra nodes."""
    s = np.asarray(desc.fem_cells, dtype=np.int64) + 1
    k, j, i = np.meshgrid(np.arange(s[2]), np.arange(s[1]), np.arange(s[0]), indexing="ij")
    lat = np.stack([i.reshape(-1), j.reshape(-1), k.reshape(-1)], axis=1).astype(np.float64)
    ext = (np.asarray(extra, dtype=np.float64).reshape(-1, 3) - np.asarray(desc.origin)) / desc.h \
        - np.asarray(desc.fem_lo, dtype=np.float64)
    return np.concatenate([lat, ext])


def node_layers(desc, n_nodes):
    """Lattice layer of each node (min over axes of the distance to the box's faces, in
    cells); extra nodes lie strictly inside and count as free."""
    c = np.asarray(desc.fem_cells, dtype=np.int64)
    s = c + 1
    k, j, i = np.meshgrid(np.arange(s[2]), np.arange(s[1]), np.arange(s[0]), indexing="ij")
    lat = np.stack([i.reshape(-1), j.reshape(-1), k.reshape(-1)], axis=1)
    lay = np.minimum(lat, c - lat).min(axis=1)
    return np.concatenate([lay, np.full(n_nodes - len(lay), int(c.max()))])


def _edges(t):
    return [(min(t[a], t[b]), max(t[a], t[b])) for a in range(4) for b in range(a + 1, 4)]


def diameters(P, tets):
    """h_K: the longest edge of each element, in units of h."""
    d2 = np.zeros(len(tets))
    for a in range(4):
        for b in range(a + 1, 4):
            d2 = np.maximum(d2, np.sum((P[tets[:, a]] - P[tets[:, b]]) ** 2, axis=1))
    return np.sqrt(d2)


def longest_edge(P, t):
    """The edge step 3 bisects in element t (ties: the smaller index pair)."""
    es = _edges([int(v) for v in t])
    l2 = [float(np.sum((P[a] - P[b]) ** 2)) for a, b in es]
    top = max(l2)
    return min(e for e, l in zip(es, l2) if l >= (1.0 - TIE) * top)


def marks(desc, mesh, eps, sig, beta_eps, beta_sig):
    """Step 2: the marked elements of the mesh (None: K_h^0), boolean per element."""
    extra, tets = _mesh(desc, mesh)
    P = node_coords(desc, extra)
    hk = diameters(P, tets)[:, None]
    e = hk * np.abs(np.asarray(eps, dtype=np.float64))[tets]
    s = hk * np.abs(np.asarray(sig, dtype=np.float64))[tets]
    return ((e >= beta_eps * e.max()) & (s >= beta_sig * s.max())).any(axis=1)


def refine(desc, mesh, elem_marks):
    """Step 3's mesh.  Returns dict(mesh=(extra_xyz, tets), edges=[(a, b), ...] in bisection
    order, n_old=the old mesh's FEM nodes)."""
    extra, tets = _mesh(desc, mesh)
    P = [p for p in node_coords(desc, extra)]
    n_lat = int(np.prod(np.asarray(desc.fem_cells) + 1))
    n_old = n_lat + len(extra)
    layer = list(node_layers(desc, n_old))
    # the refinement forest: element id -> vertices; leaves are the current mesh
    verts = {t: tuple(int(x) for x in v) for t, v in enumerate(tets)}
    kids = {}
    around = defaultdict(set)          # edge -> current elements that contain it
    for t, v in verts.items():
        for e in _edges(v):
            around[e].add(t)
    split = []
    new_xyz = []

    def eligible(e):
        return all(layer[v] >= 1 for u in around[e] for v in verts[u])

    def longest(t):
        return longest_edge(P, verts[t])

    def bisect(e):
        a, b = e
        m = len(P)
        q = 0.5 * (P[a] + P[b])
        P.append(q)
        layer.append(1 << 30)              # a midpoint lies strictly inside: free
        new_xyz.append(np.asarray(desc.origin) + desc.h * (np.asarray(desc.fem_lo, dtype=np.float64) + q))
        split.append(e)
        for t in sorted(around.pop(e)):
            v = verts[t]
            for f in _edges(v):
                if f != e:
                    around[f].discard(t)
            ids = []
            for half in (tuple(m if x == b else x for x in v), tuple(m if x == a else x for x in v)):
                c = len(verts)
                verts[c] = half
                ids.append(c)
                for f in _edges(half):
                    around[f].add(c)
            kids[t] = ids

    def refine_element(t):
        """Bisect leaf t at its longest edge, after bisecting first every element around that
        edge whose own longest edge is another one (so that every element is split at its
        longest edge); False if an edge on the way may not be bisected."""
        while t not in kids:
            e = longest(t)
            if not eligible(e):
                return False
            others = sorted(u for u in around[e] if longest(u) != e)
            if not others:
                bisect(e)
                return True
            for u in others:
                if u not in kids and not refine_element(u):
                    return False
        return True

    for t in np.nonzero(np.asarray(elem_marks, dtype=bool))[0]:
        if int(t) not in kids:
            refine_element(int(t))
    out = []

    def emit(t):
        if t in kids:
            for c in kids[t]:
                emit(c)
        else:
            out.append(verts[t])

    for t in range(len(tets)):
        emit(t)
    ext = np.concatenate([extra, np.asarray(new_xyz, dtype=np.float64).reshape(-1, 3)])
    return {"mesh": (ext, np.asarray(out, dtype=np.int64)), "edges": split, "n_old": n_old}


def interpolate(ref, values):
    """Step 3's nodal values on the refined mesh: the old values, then at each midpoint, in
    bisection order, the mean of its edge's endpoints (an endpoint may be an earlier midpoint)."""
    v = np.asarray(values, dtype=np.float64)
    if len(v) != ref["n_old"]:
        raise ValueError("values must live on the mesh that was refined")
    out = list(v)
    for a, b in ref["edges"]:
        out.append(0.5 * (out[a] + out[b]))
    return np.asarray(out, dtype=np.float64)


def change_norm(d, a, b):
    """|a - b| in the lumped-mass L2 norm over the free nodes of discretisation d."""
    w = d.m_fem_lumped[d.fem_free]
    diff = (np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))[d.fem_free]
    return math.sqrt(float(np.sum(w * diff * diff)))


def stop_test(change, gnorm, theta):
    """Step 4: (change test for eps or sigma) and (gradient test for eps or sigma)."""
    small = change["eps"] < theta.get("theta1_eps", 0.0) or change["sig"] < theta.get("theta1_sig", 0.0)
    grad = gnorm["eps"] < theta.get("theta2_eps", 0.0) or gnorm["sig"] < theta.get("theta2_sig", 0.0)
    return bool(small and grad)


def _per_level(x, i):
    return x[i] if isinstance(x, (list, tuple)) else x


def acga(desc, sources, eobs, eps0, sig0, params, n_iter, beta_eps, beta_sig, n_refine=1, theta=None):
    """The ACGA from K_h^0 with up to n_refine refinements.  params, beta_eps, beta_sig: one
    value for every level or a list per level; theta: the tolerances of step 4 (None: no early
    stop).  Returns dict(levels=[...], eps, sigma, mesh): per level its mesh (None for K_h^0),
    its start (the interpolated coefficients), its CGA history and result, and (if it was
    refined) its element marks and refinement; and, from level 1 on, the changes and the stop
    test of step 4."""
    mesh = None
    eps, sig = np.asarray(eps0, dtype=np.float64), np.asarray(sig0, dtype=np.float64)
    levels = []
    for i in range(n_refine + 1):
        d = Discretization(desc, mesh=mesh)
        hist = cga(d, sources, eobs, eps, sig, _per_level(params, i), n_iter)
        lv = {"mesh": mesh, "start": (eps, sig), "history": hist,
              "eps": hist[-1]["eps"]["coef"], "sigma": hist[-1]["sig"]["coef"]}
        levels.append(lv)
        if i > 0:
            lv["change"] = {"eps": change_norm(d, lv["eps"], eps), "sig": change_norm(d, lv["sigma"], sig)}
            lv["stop"] = theta is not None and stop_test(
                lv["change"], {f: hist[-1][f]["grad_norm"] for f in ("eps", "sig")}, theta)
            if lv["stop"]:
                break
        if i == n_refine:
            break
        lv["marks"] = marks(desc, mesh, lv["eps"], lv["sigma"], _per_level(beta_eps, i), _per_level(beta_sig, i))
        lv["refinement"] = refine(desc, mesh, lv["marks"])
        mesh = lv["refinement"]["mesh"]
        eps = interpolate(lv["refinement"], lv["eps"])
        sig = interpolate(lv["refinement"], lv["sigma"])
    return {"levels": levels, "eps": levels[-1]["eps"], "sigma": levels[-1]["sigma"], "mesh": levels[-1]["mesh"]}
