"""Oracle discretisation: outer structured grid + Kuhn-tetrahedral FEM box, FP64.

The paper splits the domain into a finite-difference part and a finite-element
part whose boundary lies inside the finite-difference part (section "The
mathematical model", domain decomposition paragraph), with eps = 1, sigma = 0 on
the finite-difference part (eq. epsilon_sigma_constraint) and a tetrahedral
mesh of the inner cube (section "Numerical results").  The paper does not print
the discrete scheme; this module writes out the reading used throughout:

* every outer node carries E in R^3; finite-difference rows use the 7-point
  Laplacian with mirror (Neumann) edge weights w_ij = h * (cells around the
  edge inside the box) / 4 and lumped mass h^3 * 2^-(boundary coordinates);
* the FEM box's hex cells are split into 6 Kuhn tetrahedra (one per axis
  permutation); FEM rows (nodes of layer >= 1) use the assembled P1 stiffness
  and lumped P1 mass, plus the div-div stabiliser of eq. lagrangian_weak with
  the nodal product (eps - 1) E inside the divergence;
* layer-0 FEM nodes belong to the finite-difference rows, layer-1 nodes to the
  FEM rows, so the coupling is a two-node overlap;
* first-order absorbing faces (eq. forward_absorbing_bc / model1) use the
  lumped face mass h^2 * 2^-(in-face boundary coordinates).

A general (e.g. locally refined) mesh of the FEM box can replace the Kuhn split: its
nodes are the box's lattice nodes plus extra nodes strictly inside the box, its
tetrahedra any conforming set that covers the box (``mesh=(extra_xyz, tets)``, tets in
FEM-node indices: lattice nodes first, lexicographic, then the extra nodes).  Extra
nodes are free FEM-owned nodes; the ownership rules of the lattice nodes are unchanged.
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

# face bit -> (normal axis, side); side 0 = min, 1 = max.  The top face is the
# paper's backscatter boundary (d_1 Omega), the bottom face d_2 Omega and the
# four sides d_3 Omega (section "Numerical results").
FACES = {1: (2, 1), 2: (2, 0), 4: (0, 0), 8: (0, 1), 16: (1, 0), 32: (1, 1)}
TOP = 1


class Discretization:
    def __init__(self, desc, fd_only: bool = False, divdiv_form: str = "R1", mesh=None):
        """divdiv_form: "R1" (the scheme: the nodal product (eps - 1) E inside the element
        divergence, eq. forward_prob) or "R2" (the element mean of eps - 1 outside it, a
        symmetric variant for which eq. gradeps' div-div term is the exact gradient).
        mesh: None (the Kuhn split of the box) or (extra_xyz (n_extra, 3), tets (n_tets, 4)) in
        FEM-node indices, lattice nodes first; every lattice node must be a vertex."""
        if divdiv_form not in ("R1", "R2"):
            raise ValueError("divdiv_form must be R1 or R2")
        self.desc = desc
        self.fd_only = fd_only
        self.divdiv_form = divdiv_form
        nvec = np.array([int(v) for v in desc.n_outer])
        self.nvec = nvec
        self.N_grid = int(np.prod(nvec))
        extra = np.zeros((0, 3)) if mesh is None else np.asarray(mesh[0], dtype=np.float64).reshape(-1, 3)
        self.n_extra = len(extra)
        self.N = self.N_grid + self.n_extra          # grid nodes, then the mesh's extra nodes
        h = float(desc.h)
        self.h = h
        self.dt = float(desc.dt)
        k, j, i = np.meshgrid(np.arange(nvec[2]), np.arange(nvec[1]), np.arange(nvec[0]), indexing="ij")
        ijk = np.stack([i, j, k], axis=-1).reshape(-1, 3)
        self.ijk = ijk
        self.x = np.concatenate([np.asarray(desc.origin, dtype=np.float64) + h * ijk, extra])
        on_bnd = (ijk == 0) | (ijk == nvec - 1)
        self.bcount = np.concatenate([on_bnd.sum(axis=1), np.zeros(self.n_extra, dtype=np.int64)])

        # ---- FEM lattice and layers --------------------------------------------------
        lo = np.array([int(v) for v in desc.fem_lo])
        cells = np.array([int(v) for v in desc.fem_cells])
        fshape = cells + 1
        lz, ly, lx = np.meshgrid(np.arange(fshape[2]), np.arange(fshape[1]), np.arange(fshape[0]), indexing="ij")
        lat = np.stack([lx, ly, lz], axis=-1).reshape(-1, 3)
        g = lat + lo
        n_lat = len(lat)
        # FEM node -> global node: lattice nodes to their grid node, extra nodes after the grid
        self.fem_grid = np.concatenate([g[:, 0] + nvec[0] * (g[:, 1] + nvec[1] * g[:, 2]),
                                        self.N_grid + np.arange(self.n_extra)])
        big = int(cells.max())           # extra nodes lie strictly inside: layer >= 2 (free)
        self.fem_layer = np.concatenate([np.minimum(lat, cells - lat).min(axis=1), np.full(self.n_extra, big)])
        self.n_fem = len(self.fem_grid)
        self.fem_owned = self.fem_layer >= 1
        self.fem_free = self.fem_layer >= 2
        owned_grid = np.zeros(self.N, dtype=bool)
        if not fd_only:
            owned_grid[self.fem_grid[self.fem_owned]] = True
        self.owned_grid = owned_grid

        # ---- Kuhn tetrahedra: v0 = cell corner, v_k = v_{k-1} + e_{pi(k)} --------------
        cz, cy, cx = np.meshgrid(np.arange(cells[2]), np.arange(cells[1]), np.arange(cells[0]), indexing="ij")
        corner = np.stack([cx, cy, cz], axis=-1).reshape(-1, 3)

        def lat_index(p):
            return p[:, 0] + fshape[0] * (p[:, 1] + fshape[1] * p[:, 2])

        if mesh is None:
            tets = []
            eye = np.eye(3, dtype=np.int64)
            for perm in itertools.permutations(range(3)):
                v = [corner]
                for a in perm:
                    v.append(v[-1] + eye[a])
                tets.append(np.stack([lat_index(p) for p in v], axis=1))
            self.tets = np.concatenate(tets, axis=0)
        else:
            self.tets = np.asarray(mesh[1], dtype=np.int64).reshape(-1, 4)
            if self.tets.min() < 0 or self.tets.max() >= self.n_fem:
                raise ValueError("mesh tetrahedra reference a node that does not exist")
            if n_lat != int(np.prod(fshape)):
                raise ValueError("lattice size mismatch")
        X = self.x[self.fem_grid][self.tets]                       # (T, 4, 3)
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)
        self.vol = np.abs(np.linalg.det(J)) / 6.0
        if not np.all(self.vol > 0):
            raise ValueError("degenerate tetrahedron")
        box = float(np.prod(cells)) * h ** 3
        if abs(self.vol.sum() - box) > 1e-9 * box:
            raise ValueError("the tetrahedra do not fill the FEM box")
        Jinv = np.linalg.inv(J)                                     # row k = grad of barycentric k
        G = np.empty((len(self.tets), 4, 3))
        G[:, 1:, :] = Jinv
        G[:, 0, :] = -Jinv.sum(axis=1)
        self.grad = G

        # ---- lumped masses -----------------------------------------------------------
        m_fem = np.bincount(self.tets.ravel(), weights=np.repeat(self.vol / 4.0, 4), minlength=self.n_fem)
        self.m_fem_lumped = m_fem
        m = h ** 3 * 2.0 ** (-self.bcount.astype(np.float64))
        m[self.N_grid:] = 0.0
        if np.any(m_fem[self.fem_layer >= 1] <= 0):
            raise ValueError("a FEM-owned node lies on no tetrahedron")
        if not fd_only:
            own = self.fem_owned
            m[self.fem_grid[own]] = m_fem[own]
        self.m = m

        # ---- stiffness -----------------------------------------------------------------
        rows, cols, vals = [], [], []
        for a in range(3):
            sel = ijk[:, a] < nvec[a] - 1   # grid nodes only (the first N_grid global indices)
            p = np.nonzero(sel)[0]
            q = p + int(np.prod(nvec[:a]))
            cnt = np.ones(len(p))
            for b in range(3):
                if b == a:
                    continue
                cnt = cnt * ((ijk[p, b] >= 1).astype(float) + (ijk[p, b] <= nvec[b] - 2).astype(float))
            w = h * cnt / 4.0
            rows += [p, q, p, q]
            cols += [p, q, q, p]
            vals += [w, w, -w, -w]
        K_fd = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.N, self.N)).tocsr()
        self.K_fd = K_fd
        Kloc = self.vol[:, None, None] * np.einsum("tac,tbc->tab", G, G)
        gi = self.fem_grid[self.tets]
        K_fem = sp.coo_matrix((Kloc.ravel(), (np.repeat(gi, 4, axis=1).ravel(), np.tile(gi, (1, 4)).ravel())),
                              shape=(self.N, self.N)).tocsr()
        self.K_fem = K_fem
        r_fd = sp.diags((~owned_grid).astype(np.float64))
        r_fem = sp.diags(owned_grid.astype(np.float64))
        self.K = (r_fd @ K_fd + r_fem @ K_fem).tocsr()
        self.KT = self.K.T.tocsr()

        # ---- faces: lumped face masses, detectors ----------------------------------------
        self.face_mass = {}
        for bit, (a, s) in FACES.items():
            on = np.zeros(self.N, dtype=bool)
            on[:self.N_grid] = ijk[:, a] == (0 if s == 0 else nvec[a] - 1)
            fm = np.zeros(self.N)
            fm[on] = h ** 2 * 2.0 ** (-(self.bcount[on] - 1).astype(np.float64))
            self.face_mass[bit] = fm
        det_mask = np.zeros(self.N, dtype=bool)
        for bit, (a, s) in FACES.items():
            if int(desc.detector_faces) & bit:
                det_mask[:self.N_grid] |= ijk[:, a] == (0 if s == 0 else nvec[a] - 1)
        self.det = np.nonzero(det_mask)[0]          # lexicographic order
        self.eps = None

    # ---- coefficients (eq. epsilon_sigma_constraint) ------------------------------------------
    def set_coefficients(self, eps, sigma):
        eps = np.asarray(eps, dtype=np.float64).reshape(-1)
        sigma = np.asarray(sigma, dtype=np.float64).reshape(-1)
        if eps.shape != (self.n_fem,) or sigma.shape != (self.n_fem,):
            raise ValueError("eps / sigma must have one value per FEM node")
        fixed = ~self.fem_free
        if np.any(eps[fixed] != 1.0) or np.any(sigma[fixed] != 0.0):
            raise ValueError("eps must be 1 and sigma 0 on FEM layers 0 and 1")
        if np.any(eps < 1.0) or np.any(sigma < 0.0):
            raise ValueError("eps >= 1 and sigma >= 0 required")
        if self.fd_only and (np.any(eps != 1.0) or np.any(sigma != 0.0)):
            raise ValueError("the pure finite-difference discretisation needs eps = 1, sigma = 0")
        self.eps = eps
        self.sigma = sigma
        eg = np.ones(self.N)
        sg = np.zeros(self.N)
        eg[self.fem_grid] = eps
        sg[self.fem_grid] = sigma
        self.M_eps = self.m * eg
        self.M_sig = self.m * sg
        return self

    # ---- operators ------------------------------------------------------------------------------
    def _scatter(self, contrib):
        out = np.empty((self.n_fem, 3))
        idx = self.tets.ravel()
        for c in range(3):
            out[:, c] = np.bincount(idx, weights=contrib[:, :, c].ravel(), minlength=self.n_fem)
        return out

    def element_mean_eps_minus_one(self):
        """(eps - 1) averaged over the four vertices of each tetrahedron (form R2)."""
        return (self.eps - 1.0)[self.tets].mean(axis=1)

    def divdiv(self, E):
        """FEM-owned rows only.  R1: (A_dd E)_i = sum_K |K| grad(phi_i) div_K((eps - 1) E);
        R2: (A_dd E)_i = sum_K |K| (mean_K eps - 1) grad(phi_i) div_K(E)."""
        if self.divdiv_form == "R1":
            w = (self.eps - 1.0)[:, None] * E[self.fem_grid]
            div = np.einsum("tac,tac->t", self.grad, w[self.tets])
        else:
            div = self.element_mean_eps_minus_one() * np.einsum("tac,tac->t", self.grad, E[self.fem_grid][self.tets])
        acc = self._scatter((self.vol * div)[:, None, None] * self.grad)
        acc[~self.fem_owned] = 0.0
        return acc

    def divdiv_T(self, L):
        """Transpose of divdiv (L restricted to the FEM rows).  R1: (eps_j - 1) sum_K |K|
        grad(phi_j) div_K(L); R2: sum_K |K| (mean_K eps - 1) grad(phi_j) div_K(L)."""
        Lf = L[self.fem_grid].copy()
        Lf[~self.fem_owned] = 0.0
        div = np.einsum("tac,tac->t", self.grad, Lf[self.tets])
        if self.divdiv_form == "R1":
            acc = self._scatter((self.vol * div)[:, None, None] * self.grad)
            return (self.eps - 1.0)[:, None] * acc
        div = self.element_mean_eps_minus_one() * div
        return self._scatter((self.vol * div)[:, None, None] * self.grad)

    def apply_A(self, E):
        out = self.K @ E
        if not self.fd_only:
            out[self.fem_grid] += self.divdiv(E)
        return out

    def apply_AT(self, L):
        out = self.KT @ L
        if not self.fd_only:
            out[self.fem_grid] += self.divdiv_T(L)
        return out

    # ---- time-dependent boundary data -----------------------------------------------------------
    def top_absorbs(self, n):
        return n * self.dt > float(self.desc.t_switch)

    def damping(self, n):
        """S^n: lumped absorbing-face masses active at step n (the top face only after t_switch)."""
        s = np.zeros(self.N)
        for bit, fm in self.face_mass.items():
            if int(self.desc.absorbing_faces) & bit:
                if bit == TOP and not self.top_absorbs(n):
                    continue
                s = s + fm
        return s
