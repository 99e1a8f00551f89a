"""Adaptive conjugate gradient reconstruction (box "ACGA").

Level 0 runs the CGA on the uniform Kuhn split of the FEM box.  After each level the elements
where eq. meshref holds for the reconstructed eps and sigma are refined by longest-edge
bisection (dd_meshref_create: marks, propagation, the new mesh), eps and sigma are
interpolated onto the new nodes (dd_meshref_interpolate), and the next level runs the CGA on
the refined mesh (dd_create_mesh) from the interpolated coefficients, which are also its
Tikhonov centre.  The observations live on the outer grid's detectors, which the refinement of
the FEM box does not touch, so their interpolation is the identity.  Step 4's stop test
compares, on the refined mesh, the CGA's result with its start (the distance the device CGA
reports) and the last gradient norms with the tolerances.

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
    a = np.ascontiguousarray(a.reshape(-1), dtype=np.float32)
    if a.size != n:
        raise ValueError(f"need {n} values, one per FEM node of the mesh")
    return a


class Refinement:
    """One application of steps 2 and 3 to a mesh (None: the Kuhn split) for the nodal values
    eps, sigma (host or device): marks, the refined mesh (extra_xyz, tets) for
    Problem(desc, mesh=...), and interpolate() for nodal functions."""

    def __init__(self, desc, mesh, eps, sigma, beta_eps, beta_sig):
        lib = _lib.load()
        self._desc = _lib.make_desc(desc)
        n_lat = int(np.prod(np.asarray(desc.fem_cells) + 1))
        if mesh is None:
            xyz, tets = np.zeros((0, 3)), np.zeros((0, 4), dtype=np.int32)
        else:
            xyz = np.ascontiguousarray(mesh[0], dtype=np.float64).reshape(-1, 3)
            tets = np.ascontiguousarray(mesh[1], dtype=np.int32).reshape(-1, 4)
        self.n_old = n_lat + len(xyz)
        e, s = _host_f32(eps, self.n_old), _host_f32(sigma, self.n_old)
        h = ctypes.c_void_p()
        _lib.check(lib.dd_meshref_create(ctypes.byref(self._desc), len(xyz), xyz.ctypes.data if len(xyz) else None,
                                         len(tets), tets.ctypes.data if len(tets) else None, e.ctypes.data,
                                         s.ctypes.data, float(beta_eps), float(beta_sig), ctypes.byref(h)))
        self._h = h
        n = [ctypes.c_int64() for _ in range(4)]
        _lib.check(lib.dd_meshref_sizes(h, *[ctypes.byref(v) for v in n]))
        self.n_marked, self.n_bisected, n_extra, n_tets = (int(v.value) for v in n)
        n_in = len(tets) if len(tets) else 6 * int(np.prod(desc.fem_cells))
        self.marks = np.zeros(n_in, dtype=np.uint8)
        out_xyz = np.zeros((n_extra, 3), dtype=np.float64)
        out_tets = np.zeros((n_tets, 4), dtype=np.int32)
        _lib.check(lib.dd_meshref_result(h, self.marks.ctypes.data, out_xyz.ctypes.data if n_extra else None,
                                         out_tets.ctypes.data))
        self.mesh = (out_xyz, out_tets)

    def interpolate(self, values):
        """A nodal function of the old mesh (host or device) on the refined mesh (float32, host)."""
        v = _host_f32(values, self.n_old)
        out = np.zeros(self.n_old + self.n_bisected, dtype=np.float32)
        _lib.check(_lib.load().dd_meshref_interpolate(self._h, v.ctypes.data, out.ctypes.data))
        return out

    def close(self):
        if self._h:
            _lib.load().dd_meshref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _per_level(x, i):
    return x[i] if isinstance(x, (list, tuple)) else x


def acga(desc, sources, obs, eps0, sig0, params, n_iter, beta_eps, beta_sig, n_refine=1, theta=None):
    """Run the ACGA with up to n_refine refinements.

    params: a CGAParams (every level), a list per level, or a callable (level, problem, eps,
    sigma) -> CGAParams; beta_eps, beta_sig: one value or a list per level; theta: dict of
    step 4's tolerances theta1_eps, theta1_sig, theta2_eps, theta2_sig (None: no early stop).
    obs: the observations [n_src][n_steps][n_det][3] (float32 CUDA tensor), the same on every
    level.  Returns a dict with the final eps and sigma (CUDA tensors over the final mesh's FEM
    nodes) and mesh, and per level its mesh, CGA infos, marks and sizes of its refinement,
    and (from level 1) the distance of its result from its start and the stop test."""
    dev = torch.device("cuda", torch.cuda.current_device())
    eps = torch.as_tensor(eps0, dtype=torch.float32, device=dev).contiguous()
    sig = torch.as_tensor(sig0, dtype=torch.float32, device=dev).contiguous()
    mesh = None
    levels = []
    for i in range(n_refine + 1):
        p = Problem(desc, mesh=mesh)
        prm = params(i, p, eps, sig) if callable(params) else _per_level(params, i)
        run = CGA(p, sources, obs, eps, sig, prm)
        hist = run.run(n_iter)
        eps, sig = run.eps.clone(), run.sigma.clone()
        run.close()
        p.close()
        lv = {"mesh": mesh, "history": hist}
        levels.append(lv)
        if i > 0:
            last = hist[-1]
            lv["change"] = dict(last["change_norm"])
            small = lv["change"]["eps"] < (theta or {}).get("theta1_eps", 0.0) or \
                lv["change"]["sig"] < (theta or {}).get("theta1_sig", 0.0)
            grad = last["grad_norm"]["eps"] < (theta or {}).get("theta2_eps", 0.0) or \
                last["grad_norm"]["sig"] < (theta or {}).get("theta2_sig", 0.0)
            lv["stop"] = bool(theta is not None and small and grad)
            if lv["stop"]:
                break
        if i == n_refine:
            break
        ref = Refinement(desc, mesh, eps, sig, _per_level(beta_eps, i), _per_level(beta_sig, i))
        lv["marks"] = ref.marks.astype(bool)
        lv["n_bisected"] = ref.n_bisected
        mesh = ref.mesh
        eps = torch.tensor(ref.interpolate(eps), device=dev)
        sig = torch.tensor(ref.interpolate(sig), device=dev)
        ref.close()
    return {"eps": eps, "sigma": sig, "mesh": mesh, "levels": levels}
