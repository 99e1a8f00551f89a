"""Adaptive conjugate gradient reconstruction (box "ACGA"), FP64, one refinement level.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the smoke check
and the benchmark's CPU baseline may use it; the HIP path shares no code with it.

Steps (box "ACGA"):
  1. the CGA on the current mesh (oracle.cga);
  2. refine the elements where eq. meshref holds for the reconstruction:
     |h eps_h| >= beta_eps max |h eps_h| and |h sigma_h| >= beta_sig max |h sigma_h|;
  3. build the new mesh, interpolate eps_h, sigma_h (and E_obs) onto it;
  4. stop, or repeat from 1 on the new mesh.

Readings (where the paper leaves a choice):
  * the starting mesh is the uniform Kuhn split of the FEM box, where the mesh function h of
    eq. meshfunction is the same on every element and cancels from both inequalities;
  * the inequalities are tested at the FEM nodes (eps_h, sigma_h are nodal functions) and an
    element is refined when both hold at one of its vertices; the maxima run over the whole FEM
    lattice; only cells whose eight corners are FEM-owned (layer >= 1) are refined, so that the
    two overlap layers keep their lattice elements;
  * refining a cell: its centre becomes a node, and each of its six Kuhn tetrahedra (which all
    contain the cell's main diagonal as an edge) is bisected at the midpoint of that edge, which
    is the centre.  No face of the cell is split, so the mesh stays conforming without
    propagating the refinement;
  * interpolation: the nodal functions keep their values at the old nodes and take the value of
    their trilinear interpolant (the mean of the cell's eight corners) at a centre; E_obs lives
    on the outer grid's detectors, which the refinement does not touch, so its interpolation is
    the identity;
  * the CGA on the refined mesh starts from the interpolated reconstruction, which is also its
    Tikhonov centre (the CGA's centre is its initial guess); one refinement level is taken, so
    the test of step 4 is not needed to stop.
"""

from __future__ import annotations

import numpy as np

from .cga import cga
from .discretization import Discretization

# The six Kuhn tetrahedra of a cell: vertex 0 is the lowest corner, each following vertex one
# unit step along the next axis of the permutation, vertex 3 the highest corner.
PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _corner_offsets():
    return np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)])


def marks(desc, eps, sig, beta_eps, beta_sig):
    """Step 2's cells (boolean per cell, lexicographic, x fastest)."""
    cells = np.asarray(desc.fem_cells, dtype=np.int64)
    shape = cells + 1
    e = np.abs(np.asarray(eps, dtype=np.float64)).reshape(shape[::-1])   # [z][y][x]
    s = np.abs(np.asarray(sig, dtype=np.float64)).reshape(shape[::-1])
    flag = (e >= beta_eps * e.max()) & (s >= beta_sig * s.max())
    out = np.zeros(cells[::-1], dtype=bool)
    for dx, dy, dz in _corner_offsets():
        out |= flag[dz:dz + cells[2], dy:dy + cells[1], dx:dx + cells[0]]
    # only cells whose corners are all FEM-owned: 1 <= corner index <= cells - 1 on every axis
    kk, jj, ii = np.meshgrid(np.arange(cells[2]), np.arange(cells[1]), np.arange(cells[0]), indexing="ij")
    owned = (ii >= 1) & (ii + 1 <= cells[0] - 1) & (jj >= 1) & (jj + 1 <= cells[1] - 1) & (kk >= 1) & \
        (kk + 1 <= cells[2] - 1)
    return (out & owned).reshape(-1)


def refine(desc, cell_marks):
    """Step 3's mesh: (extra_xyz [n_marked][3], tets [n][4]) in FEM-node indices (lattice nodes
    lexicographic, then the centres in cell order); per cell its six tetrahedra in PERMS order,
    those of a marked cell each replaced by its two halves (v0, v1, v2, centre), (centre, v1,
    v2, v3)."""
    cells = [int(c) for c in desc.fem_cells]
    nx, ny = cells[0] + 1, cells[1] + 1
    n_lat = nx * ny * (cells[2] + 1)
    h = float(desc.h)
    extra, tets = [], []
    for k in range(cells[2]):
        for j in range(cells[1]):
            for i in range(cells[0]):
                marked = bool(cell_marks[i + cells[0] * (j + cells[1] * k)])
                if marked:
                    centre = n_lat + len(extra)
                    extra.append([desc.origin[a] + h * (desc.fem_lo[a] + (i, j, k)[a] + 0.5) for a in range(3)])
                for perm in PERMS:
                    v = [np.array((i, j, k))]
                    for ax in perm:
                        step = np.zeros(3, dtype=np.int64)
                        step[ax] = 1
                        v.append(v[-1] + step)
                    ids = [int(p[0] + nx * (p[1] + ny * p[2])) for p in v]
                    if marked:
                        tets.append([ids[0], ids[1], ids[2], centre])
                        tets.append([centre, ids[1], ids[2], ids[3]])
                    else:
                        tets.append(ids)
    return np.asarray(extra, dtype=np.float64).reshape(-1, 3), np.asarray(tets, dtype=np.int64)


def interpolate(desc, cell_marks, values):
    """Step 3's nodal values: the old values, then the trilinear interpolant at each centre."""
    cells = np.asarray(desc.fem_cells, dtype=np.int64)
    v = np.asarray(values, dtype=np.float64)
    grid = v.reshape((cells + 1)[::-1])
    centre = np.zeros(cells[::-1])
    for dx, dy, dz in _corner_offsets():
        centre += grid[dz:dz + cells[2], dy:dy + cells[1], dx:dx + cells[0]]
    centre /= 8.0
    return np.concatenate([v, centre.reshape(-1)[np.asarray(cell_marks, dtype=bool)]])


def acga(desc, sources, eobs, eps0, sig0, params, n_iter, beta_eps, beta_sig, params_fine=None):
    """The CGA on the uniform mesh, one refinement, the CGA on the refined mesh.  Returns the
    two levels' CGA histories, the marks, the mesh and the final coefficients."""
    d0 = Discretization(desc)
    h0 = cga(d0, sources, eobs, eps0, sig0, params, n_iter)
    eps_c, sig_c = h0[-1]["eps"]["coef"], h0[-1]["sig"]["coef"]
    m = marks(desc, eps_c, sig_c, beta_eps, beta_sig)
    mesh = refine(desc, m)
    eps_f, sig_f = interpolate(desc, m, eps_c), interpolate(desc, m, sig_c)
    d1 = Discretization(desc, mesh=mesh)
    h1 = cga(d1, sources, eobs, eps_f, sig_f, params if params_fine is None else params_fine, n_iter)
    return {"coarse": h0, "fine": h1, "marks": m, "mesh": mesh, "eps_coarse": eps_c, "sig_coarse": sig_c,
            "eps": h1[-1]["eps"]["coef"], "sigma": h1[-1]["sig"]["coef"]}
