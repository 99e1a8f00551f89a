"""Conjugate gradient reconstruction of eps and sigma (box "CGA") on the device.

Each iteration is the solver's step 1 (dd_set_coefficients, dd_forward with saving,
dd_adjoint_misfit, dd_gradient) and the library's steps 2-6 (dd_cga_update: gradient
functions of eq. gradeps with the Tikhonov terms of eq. tikhonov_functional, the
conjugate direction, the coefficient update kept in the box of
eq. epsilon_sigma_constraint, the step-size and regularisation rules and the stop test).
Everything stays on the device; the host reads the run's scalars once per iteration.
"""

import ctypes
from dataclasses import dataclass, fields

import numpy as np
import torch

from . import _lib
from .solver import _ptr, _stream


def taper_weights(n_steps, dt, delta):
    """The library's smoothing function z of eq. tikhonov_functional at the trace rows
    (dd_misfit_taper: 1 until delta before the end time, then a cosine ramp to 0)."""
    z = np.empty(int(n_steps), dtype=np.float64)
    _lib.check(_lib.load().dd_misfit_taper(int(n_steps), float(dt), float(delta), z.ctypes.data_as(ctypes.c_void_p)))
    return z


@dataclass
class CGAParams:
    gamma_eps: float
    gamma_sig: float
    p: float
    alpha_eps: float
    alpha_sig: float
    eps_max: float
    sig_max: float
    eta1_eps: float = 0.0
    eta1_sig: float = 0.0
    eta2_eps: float = 0.0
    eta2_sig: float = 0.0

    @staticmethod
    def from_gradient(g_eps, g_sig, h, eps_max, sig_max, step_eps=0.5, step_sig=0.1, p=0.5):
        """Step sizes and regularisation from the gradient of J at the initial guess (a host
        read of max|g|): the first update moves eps by at most step_eps and sigma by at most
        step_sig, and gamma^0 = max|g| / step, so that alpha^1 = 1 / gamma^0 keeps that scale."""
        h3 = float(h) ** 3
        gm = [max(float(torch.max(torch.abs(g)).item()) / h3, 1e-30) for g in (g_eps, g_sig)]
        return CGAParams(gamma_eps=gm[0] / step_eps, gamma_sig=gm[1] / step_sig, p=p, alpha_eps=step_eps / gm[0],
                         alpha_sig=step_sig / gm[1], eps_max=eps_max, sig_max=sig_max)

    def to_c(self):
        c = _lib.CgaParams()
        for f in fields(self):
            setattr(c, f.name, float(getattr(self, f.name)))
        return c


class CGA:
    """A CGA run on one problem: sources, observations [n_src][n_steps][n_det][3] and the
    initial guess (also the Tikhonov centre).  ``eps`` and ``sigma`` hold the iterate."""

    def __init__(self, problem, sources, obs, eps0, sig0, params, z=None, track_loss=False):
        """z: time weights of the misfit (numpy, one per step; None = 1); track_loss: also form
        J of every solve on the device (read by info())."""
        dev = torch.device("cuda", torch.cuda.current_device())
        self.problem = problem
        self.sources = list(sources)
        shape = (len(self.sources), problem.n_steps, problem.n_det, 3)
        if tuple(obs.shape) != shape or obs.dtype != torch.float32 or not obs.is_cuda:
            raise ValueError("observations must be a float32 CUDA (HIP) tensor of shape %s" % (shape,))
        self.obs = obs.contiguous()
        self.eps = torch.as_tensor(eps0, dtype=torch.float32, device=dev).clone().contiguous()
        self.sigma = torch.as_tensor(sig0, dtype=torch.float32, device=dev).clone().contiguous()
        self._shape = shape
        self.traces = self.g_eps = self.g_sig = self.cot = None     # allocated by the first solve()
        self.z = None if z is None else np.ascontiguousarray(z, dtype=np.float64)
        self.track_loss = bool(track_loss)
        self.J = None
        self.params = params
        self._cp = params.to_c()
        h = ctypes.c_void_p()
        _lib.check(_lib.load().dd_cga_create(problem._h, ctypes.byref(self._cp), _ptr(self.eps), _ptr(self.sigma),
                                             _stream(), ctypes.byref(h)), problem._h)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dd_cga_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self):
        """Step 1 at the current iterate: traces, misfit adjoint, gradient of J."""
        p = self.problem
        if self.traces is None:
            dev = self.eps.device
            self.traces = torch.empty(self._shape, dtype=torch.float32, device=dev)
            self.g_eps = torch.empty(p.n_fem, dtype=torch.float64, device=dev)
            self.g_sig = torch.empty(p.n_fem, dtype=torch.float64, device=dev)
        p.set_coefficients(self.eps, self.sigma)
        p.forward(self.sources, save=True, out=self.traces)
        if self.z is None:
            if self.track_loss:
                self.J, _ = p.misfit(self.traces, self.obs, cotangent=False)
            p.adjoint_misfit(self.traces, self.obs)
        else:
            if self.cot is None:
                self.cot = torch.empty_like(self.traces)
            self.J, _ = p.misfit(self.traces, self.obs, self.z, loss=self.track_loss, out=self.cot)
            p.adjoint(self.cot)
        p.gradient(out=(self.g_eps, self.g_sig))

    def steps_from_gradient(self, g_eps, g_sig, step_eps=0.5, step_sig=0.1):
        """gamma^0 and alpha^0 from the gradient of J at the initial guess, on the device (the
        first update moves eps by at most step_eps and sigma by at most step_sig); before the
        first update."""
        for t in (g_eps, g_sig):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.problem.n_fem):
                raise ValueError("gradients must be contiguous float64 CUDA tensors of n_fem entries")
        _lib.check(_lib.load().dd_cga_steps_from_gradient(self._h, _ptr(g_eps), _ptr(g_sig), float(step_eps),
                                                          float(step_sig), _stream()))

    def update(self, g_eps=None, g_sig=None):
        """Steps 2-6 from the gradient of the last solve, or from the given gradient arrays
        of J at the current iterate (float64, FEM nodes); asynchronous."""
        ge = self.g_eps if g_eps is None else g_eps
        gs = self.g_sig if g_sig is None else g_sig
        for t in (ge, gs):
            if t is None or not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.problem.n_fem):
                raise ValueError("gradients must be contiguous float64 CUDA tensors of n_fem entries")
        _lib.check(_lib.load().dd_cga_update(self._h, _ptr(ge), _ptr(gs), _ptr(self.eps), _ptr(self.sigma),
                                             _stream()))

    def iterate(self):
        self.solve()
        self.update()

    def info(self):
        """Scalars of the last update (synchronises the stream)."""
        c = _lib.CgaInfo()
        _lib.check(_lib.load().dd_cga_get_info(self._h, ctypes.byref(c), _stream()))
        out = {"iterations": c.iterations, "converged": bool(c.converged)}
        if self.track_loss and self.J is not None:
            out["J"] = float(self.J.item())     # J at the iterate the last update started from
        for name in ("grad_norm", "step_norm", "beta", "alpha_used", "alpha_next", "gamma_used", "gamma_next",
                     "change_norm"):
            arr = getattr(c, name)
            out[name] = {"eps": arr[0], "sig": arr[1]}
        return out

    def run(self, n_iter):
        """Up to n_iter iterations, stopping when the stop test holds; returns the infos."""
        hist = []
        for _ in range(n_iter):
            self.iterate()
            hist.append(self.info())
            if hist[-1]["converged"]:
                break
        return hist
