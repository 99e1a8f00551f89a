"""Adaptive conjugate gradient reconstruction (box "ACGA") with one refinement level.

Level 0 runs the CGA on the uniform Kuhn split of the FEM box.  The elements where eq. meshref
holds for the reconstructed eps and sigma are then refined (dd_meshref_marks / dd_meshref_mesh:
a marked cell gets its centre as a node and its tetrahedra bisected), eps and sigma are
interpolated onto the new nodes (dd_meshref_values), and level 1 runs the CGA on the refined
mesh (dd_create_mesh) from the interpolated coefficients, which are also its Tikhonov centre.
The observations live on the outer grid's detectors, which the refinement of the FEM box does
not touch, so their interpolation is the identity.

Only argument marshalling happens here: the refinement runs in the library's host code, the
solves and the updates in its kernels.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from .cga import CGA
from .solver import Problem


def _host_f32(x, n):
    a = x.detach().to("cpu").numpy() if isinstance(x, torch.Tensor) else np.asarray(x)
    a = np.ascontiguousarray(a.reshape(-1)[:n], dtype=np.float32)
    if a.size != n:
        raise ValueError(f"need {n} FEM-lattice values")
    return a


def meshref(desc, eps, sigma, beta_eps, beta_sig):
    """Cells marked by eq. meshref for the lattice values eps, sigma (host or device), and the
    refined mesh (extra_xyz, tets) for Problem(desc, mesh=...)."""
    lib = _lib.load()
    cd = _lib.make_desc(desc)
    cells = [int(c) for c in desc.fem_cells]
    n_lat = int(np.prod(np.asarray(cells) + 1))
    e, s = _host_f32(eps, n_lat), _host_f32(sigma, n_lat)
    marks = np.zeros(int(np.prod(cells)), dtype=np.uint8)
    n = lib.dd_meshref_marks(ctypes.byref(cd), e.ctypes.data, s.ctypes.data, float(beta_eps), float(beta_sig),
                             marks.ctypes.data)
    if n < 0:
        raise _lib.DDError(int(n), _lib.ERRORS.get(int(n), "error"))
    xyz = np.zeros((int(n), 3), dtype=np.float64)
    tets = np.zeros((6 * marks.size + 6 * int(n), 4), dtype=np.int32)
    _lib.check(lib.dd_meshref_mesh(ctypes.byref(cd), marks.ctypes.data, xyz.ctypes.data if n else None,
                                   tets.ctypes.data))
    return marks, (xyz, tets)


def interpolate(desc, marks, lattice_values):
    """A FEM-lattice array on the refined mesh's nodes (float32, host)."""
    n_lat = int(np.prod(np.asarray(desc.fem_cells) + 1))
    v = _host_f32(lattice_values, n_lat)
    out = np.zeros(n_lat + int(np.count_nonzero(marks)), dtype=np.float32)
    m = np.ascontiguousarray(marks, dtype=np.uint8)
    _lib.check(_lib.load().dd_meshref_values(ctypes.byref(_lib.make_desc(desc)), m.ctypes.data, v.ctypes.data,
                                             out.ctypes.data))
    return out


def acga(desc, sources, obs, eps0, sig0, params, n_iter, beta_eps, beta_sig, levels=1):
    """Run the ACGA: `levels` = 0 (the CGA on the uniform mesh) or 1 (then refine and continue).

    params: a CGAParams for every level, or a callable (level, problem, eps, sigma) -> CGAParams.
    obs: the observations [n_src][n_steps][n_det][3] (float32 CUDA tensor), the same on every
    level.  Returns a dict with the final eps and sigma (CUDA tensors over the final mesh's FEM
    nodes), the refined mesh and its marks (None at level 0), and each level's CGA infos."""
    if levels not in (0, 1):
        raise ValueError("one refinement level is supported (levels = 0 or 1)")
    dev = torch.device("cuda", torch.cuda.current_device())
    eps = torch.as_tensor(eps0, dtype=torch.float32, device=dev).contiguous()
    sig = torch.as_tensor(sig0, dtype=torch.float32, device=dev).contiguous()
    mesh = marks = None
    history = []
    for level in range(levels + 1):
        p = Problem(desc, mesh=mesh)
        prm = params(level, p, eps, sig) if callable(params) else params
        run = CGA(p, sources, obs, eps, sig, prm)
        history.append(run.run(n_iter))
        eps, sig = run.eps.clone(), run.sigma.clone()
        run.close()
        p.close()
        if level == levels:
            break
        marks, mesh = meshref(desc, eps, sig, beta_eps, beta_sig)
        eps = torch.tensor(interpolate(desc, marks, eps), device=dev)
        sig = torch.tensor(interpolate(desc, marks, sig), device=dev)
    return {"eps": eps, "sigma": sig, "mesh": mesh, "marks": marks, "history": history}
