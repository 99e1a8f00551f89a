"""Python face of the batch C-ABI (dd_batch_*): several problems advanced by one launch per step."""

import ctypes

import torch

from . import _lib
from .solver import _ptr, _stream


class Batch:
    """Up to `max_slots` concurrent solves sharing every step launch."""

    def __init__(self, max_slots=16, fill_cells=None, hbm_budget=0):
        """fill_cells: a launch takes the oldest jobs until their cells per step reach this
        (None: the library's default; 0: every job in every launch).  hbm_budget: bytes the
        problems with an active job may hold together (0: no limit); a job over it is refused."""
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().dd_batch_create(int(max_slots), int(hbm_budget), ctypes.byref(self._h)))
        if fill_cells is not None:
            _lib.check(_lib.load().dd_batch_set_fill(self._h, int(fill_cells)))
        self.max_slots = int(max_slots)
        self.jobs = {}          # job id -> dict with the problem and the tensors it writes

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, problem, sources, obs=None, gradient=True):
        """Queue forward (+ adjoint and gradient when `obs` is given) of `problem` for `sources`."""
        dev = torch.device("cuda", torch.cuda.current_device())
        n = len(sources)
        traces = torch.empty((n, problem.n_steps, problem.n_det, 3), dtype=torch.float32, device=dev)
        ge = gs = None
        if obs is not None:
            obs = obs.to(torch.float32).contiguous()
            if tuple(obs.shape) != tuple(traces.shape):
                raise ValueError("observations must have the traces' shape")
            if gradient:
                ge = torch.empty(problem.n_fem, dtype=torch.float64, device=dev)
                gs = torch.empty(problem.n_fem, dtype=torch.float64, device=dev)
        job = ctypes.c_int32()
        problem.generation += 1
        _lib.check(_lib.load().dd_batch_submit(
            self._h, problem._h, _lib.make_sources(sources), n, _ptr(traces),
            _ptr(obs) if obs is not None else None, _ptr(ge) if ge is not None else None,
            _ptr(gs) if gs is not None else None, ctypes.byref(job)), problem._h)
        problem._n_src = n
        self.jobs[job.value] = dict(problem=problem, traces=traces, obs=obs, g_eps=ge, g_sigma=gs)
        return job.value

    def step(self, max_steps):
        _lib.check(_lib.load().dd_batch_step(self._h, int(max_steps), _stream()))

    def poll(self):
        """(finished job records, number of active jobs)."""
        buf = (ctypes.c_int32 * 64)()
        n, act = ctypes.c_int32(), ctypes.c_int32()
        done = []
        while True:
            _lib.check(_lib.load().dd_batch_poll(self._h, buf, 64, ctypes.byref(n), ctypes.byref(act)))
            for i in range(n.value):
                rec = self.jobs.pop(buf[i])
                rec["id"] = buf[i]
                done.append(rec)
            if n.value < 64:
                return done, act.value

    def run_to_completion(self, chunk=1024):
        out = []
        while True:
            self.step(chunk)
            d, act = self.poll()
            out += d
            if act == 0:
                return out
