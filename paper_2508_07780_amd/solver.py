"""Python face of the C-ABI: one Problem per dd_problem handle.

Only argument marshalling happens here: torch provides device memory and the
current stream; every step of the solve runs in the library's HIP kernels.
"""

import ctypes

import numpy as np

import torch

from . import _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _device_f32(x, n, name):
    t = torch.as_tensor(x)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    t = t.to(torch.float32).contiguous().reshape(-1)
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} entries, got {t.numel()}")
    return t


class TorchAllocator:
    """Routes a problem's device allocations through torch's caching allocator (on the stream
    current at each allocation) and counts the bytes it holds."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self.bytes = 0
        self.peak = 0
        self.alloc_fn = _lib.ALLOC_FN(self._alloc)
        self.free_fn = _lib.FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, torch.cuda.current_stream(self.device))
        except Exception:       # out of memory: the library reports DD_ERR_OOM
            return None
        self.live[ptr] = int(nbytes)
        self.bytes += int(nbytes)
        self.peak = max(self.peak, self.bytes)
        return ptr

    def _free(self, ptr, ctx):
        try:
            self.bytes -= self.live.pop(ptr, 0)
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass


class Problem:
    """A hybrid FE/FD problem resident on the current GPU.  Its device state is allocated
    through torch's caching allocator (allocator="torch", the default) or by the library
    with hipMalloc (allocator=None).

    mesh: None (the Kuhn split of the FEM box) or (extra_xyz, tets), a general tetrahedral mesh
    of the box: extra nodes (n_extra x 3, physical coordinates, strictly inside the box) after
    the lattice nodes, tetrahedra (n_tets x 4) in FEM-node indices (dd_create_mesh)."""

    def __init__(self, desc, allocator="torch", mesh=None):
        lib = _lib.load()
        self.desc = desc
        self._cdesc = _lib.make_desc(desc)
        h = ctypes.c_void_p()
        self.allocator = None
        if allocator == "torch":
            self.allocator = TorchAllocator(torch.cuda.current_device())
            fns = (self.allocator.alloc_fn, self.allocator.free_fn)
        elif allocator is None:
            fns = (_lib.ALLOC_FN(), _lib.FREE_FN())
        else:
            raise ValueError('allocator must be "torch" or None')
        if mesh is None:
            _lib.check(lib.dd_create(ctypes.byref(self._cdesc), *fns, None, ctypes.byref(h)))
        else:
            xyz = np.ascontiguousarray(np.asarray(mesh[0], dtype=np.float64).reshape(-1, 3))
            tets = np.ascontiguousarray(np.asarray(mesh[1], dtype=np.int32).reshape(-1, 4))
            _lib.check(lib.dd_create_mesh(ctypes.byref(self._cdesc), len(xyz),
                                          xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(tets),
                                          tets.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), *fns, None,
                                          ctypes.byref(h)))
        self._h = h
        nf, nd, ng = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(lib.dd_sizes(h, ctypes.byref(nf), ctypes.byref(nd), ctypes.byref(ng)), h)
        self.n_fem, self.n_det, self.n_grid = nf.value, nd.value, ng.value
        self.n_steps = int(desc.n_steps)
        self._n_src = 0
        # bumped by every call that replaces the saved forward state (coefficients, forward,
        # div-div form, initial data, a batched job): an autograd node checks it in backward
        self.generation = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def footprint_bytes(desc, n_src):
        c = _lib.make_desc(desc)
        return int(_lib.load().dd_footprint_bytes(ctypes.byref(c), int(n_src)))

    @staticmethod
    def detector_nodes(desc):
        import numpy as np
        c = _lib.make_desc(desc)
        n = ctypes.c_int64()
        lib = _lib.load()
        _lib.check(lib.dd_detector_nodes(ctypes.byref(c), None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int64)
        _lib.check(lib.dd_detector_nodes(ctypes.byref(c), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         n.value, ctypes.byref(n)))
        return out

    def set_coefficients(self, eps, sigma, wait=True):
        """eps, sigma on the FEM nodes.  wait=False: checked and applied on the device without a
        host round trip (refused coefficients leave the previous ones; coefficients_status tells)."""
        e = _device_f32(eps, self.n_fem, "eps")
        s = _device_f32(sigma, self.n_fem, "sigma")
        self.generation += 1
        fn = _lib.load().dd_set_coefficients if wait else _lib.load().dd_set_coefficients_async
        _lib.check(fn(self._h, _ptr(e), _ptr(s), _stream()), self._h)
        if not wait:
            self._coef_keep = (e, s)        # alive until the queued kernels have read them

    def coefficients_status(self):
        """Raise DDError (DD_ERR_CONSTRAINT) if the last set_coefficients(wait=False) was refused."""
        _lib.check(_lib.load().dd_coefficients_status(self._h, _stream()), self._h)

    def forward(self, sources, save=True, energy=False, out=None):
        srcs = _lib.make_sources(sources)
        n = len(sources)
        dev = torch.device("cuda", torch.cuda.current_device())
        shape = (n, self.n_steps, self.n_det, 3)
        traces = out if out is not None else torch.empty(shape, dtype=torch.float32, device=dev)
        if tuple(traces.shape) != shape or traces.dtype != torch.float32 or not traces.is_contiguous():
            raise ValueError("trace buffer must be a contiguous float32 tensor of shape %s" % (shape,))
        en = torch.empty((n, self.n_steps), dtype=torch.float64, device=dev) if energy else None
        self.generation += 1
        _lib.check(_lib.load().dd_forward(self._h, srcs, n, _ptr(traces), 1 if save else 0,
                                          _ptr(en) if en is not None else None, _stream()), self._h)
        self._n_src = n
        return (traces, en) if energy else traces

    def adjoint(self, cot):
        c = torch.as_tensor(cot)
        if not c.is_cuda:
            raise ValueError("cotangent must be a CUDA (HIP) tensor")
        c = c.to(torch.float32).contiguous()
        if self._n_src and c.numel() != self._n_src * self.n_steps * self.n_det * 3:
            raise ValueError("cotangent must match the traces of the last forward")
        _lib.check(_lib.load().dd_adjoint(self._h, _ptr(c), _stream()), self._h)

    def adjoint_misfit(self, traces, obs):
        """Adjoint for the misfit cotangent traces - obs, formed inside the adjoint kernels."""
        shape = (self._n_src, self.n_steps, self.n_det, 3)
        for name, t in (("traces", traces), ("observations", obs)):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()) or \
                    (self._n_src and tuple(t.shape) != shape):
                raise ValueError("%s must be a contiguous float32 CUDA (HIP) tensor of shape %s" % (name, shape))
        _lib.check(_lib.load().dd_adjoint_misfit(self._h, _ptr(traces), _ptr(obs), _stream()), self._h)

    def gradient(self, out=None, reg=None):
        """(dJ/deps, dJ/dsigma) on the FEM nodes (float64).  reg: None, or (gamma_eps, gamma_sig,
        eps0, sigma0) to add the derivative of the Tikhonov term of eq. tikhonov_functional."""
        if out is not None:
            ge, gs = out
            for t in (ge, gs):
                if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.n_fem):
                    raise ValueError("gradient buffers must be contiguous float64 CUDA tensors of n_fem entries")
        else:
            dev = torch.device("cuda", torch.cuda.current_device())
            ge = torch.empty(self.n_fem, dtype=torch.float64, device=dev)
            gs = torch.empty(self.n_fem, dtype=torch.float64, device=dev)
        treg = None
        if reg is not None:
            g_e, g_s, e0, s0 = reg
            e0 = _device_f32(e0, self.n_fem, "eps0")
            s0 = _device_f32(s0, self.n_fem, "sigma0")
            treg = _lib.Tikhonov(float(g_e), float(g_s), e0.data_ptr(), s0.data_ptr())
            self._reg_keep = (e0, s0)       # alive until the queued kernels have read them
        _lib.check(_lib.load().dd_gradient(self._h, _ptr(ge), _ptr(gs), ctypes.byref(treg) if treg else None,
                                           _stream()), self._h)
        return ge, gs

    def device_bytes(self):
        """Bytes the library holds through torch's allocator (None with hipMalloc)."""
        return None if self.allocator is None else self.allocator.bytes

    def misfit(self, traces, obs, z=None, cotangent=True, loss=True, out=None, no_alloc=False):
        """(J, cot) of the trace misfit with time weights z (numpy, n_steps, or None for z = 1):
        cot = z_n (traces - obs) (float32, into `out` when given, or None), J a float64 device
        scalar (or None).  no_alloc: through dd_misfit_noalloc (the library's scratch is a static
        device array; the output buffers are still torch allocations here unless given)."""
        import numpy as np
        n = traces.shape[0]
        shape = (n, self.n_steps, self.n_det, 3)
        for name, t in (("traces", traces), ("observations", obs)):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shape):
                raise ValueError("%s must be a contiguous float32 CUDA (HIP) tensor of shape %s" % (name, shape))
        zz = None
        if z is not None:
            zz = np.ascontiguousarray(z, dtype=np.float64)
            if zz.shape != (self.n_steps,):
                raise ValueError("z must have one weight per time step")
        cot = (out if out is not None else torch.empty_like(traces)) if cotangent else None
        if cot is not None and (cot.shape != traces.shape or cot.dtype != torch.float32 or not cot.is_contiguous()):
            raise ValueError("cotangent buffer must match the traces")
        J = torch.empty((), dtype=torch.float64, device=traces.device) if loss else None
        fn = _lib.load().dd_misfit_noalloc if no_alloc else _lib.load().dd_misfit
        _lib.check(fn(self._h, _ptr(traces), _ptr(obs), n,
                                         zz.ctypes.data_as(ctypes.c_void_p) if zz is not None else None,
                                         _ptr(cot) if cot is not None else None,
                                         _ptr(J) if J is not None else None, _stream()), self._h)
        return J, cot

    def set_divdiv_form(self, form):
        """"R1" (the scheme of eq. forward_prob) or "R2" (element mean of eps - 1 outside the
        divergence; the paper's gradient formula is then exact)."""
        code = {"R1": 1, "R2": 2}[form]
        self.generation += 1
        _lib.check(_lib.load().dd_set_divdiv_form(self._h, code), self._h)

    def set_graph(self, mode):
        """Forward and adjoint launches replayed as HIP graphs: "off", "on" or "auto" (the
        default: small grids, from the second call in a row with the same arguments)."""
        code = {"off": 0, "on": 1, "auto": 2}[mode]
        _lib.check(_lib.load().dd_set_graph(self._h, code), self._h)

    def graph_stats(self, which="forward"):
        """(graphs captured, calls replayed as a graph) so far, of "forward" or "adjoint"."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        code = {"forward": 0, "adjoint": 1}[which]
        _lib.check(_lib.load().dd_graph_stats(self._h, code, ctypes.byref(c), ctypes.byref(r)), self._h)
        return c.value, r.value

    def check_finite(self):
        """Raise DDError (DD_ERR_UNSTABLE) if the current fields hold non-finite values."""
        _lib.check(_lib.load().dd_check_finite(self._h, _stream()), self._h)

    def set_initial_data(self, f0=None, f1=None):
        """E(0) = f0, dE/dt(0) = f1 (eq. forward_initial_cond) for the following forwards:
        CUDA tensors of n_grid x 3 values (node-major, node index x + Nx (y + Ny z)).  Both None:
        start from rest again."""
        lib = _lib.load()
        self.generation += 1
        if f0 is None and f1 is None:
            _lib.check(lib.dd_set_initial_data(self._h, None, None, _stream()), self._h)
            return
        if f0 is None or f1 is None:
            raise ValueError("initial data needs both f0 and f1")
        a = _device_f32(f0, 3 * self.n_grid, "f0")
        b = _device_f32(f1, 3 * self.n_grid, "f1")
        _lib.check(lib.dd_set_initial_data(self._h, _ptr(a), _ptr(b), _stream()), self._h)

    def paper_gradient(self, on=True):
        """Accumulate the paper-formula gradient variant in the following adjoints."""
        _lib.check(_lib.load().dd_paper_gradient_enable(self._h, 1 if on else 0), self._h)

    def gradient_paper(self):
        """(g_eps of the paper formula, g_sigma) after an adjoint with the variant on."""
        dev = torch.device("cuda", torch.cuda.current_device())
        ge = torch.empty(self.n_fem, dtype=torch.float64, device=dev)
        gs = torch.empty(self.n_fem, dtype=torch.float64, device=dev)
        _lib.check(_lib.load().dd_gradient_paper(self._h, _ptr(ge), _ptr(gs), _stream()), self._h)
        return ge, gs

    # ---- kernel timing ---------------------------------------------------------------------
    def profile(self, stride=1):
        """Time every `stride`-th step launch with HIP events (0 switches timing off)."""
        _lib.check(_lib.load().dd_profile_enable(self._h, int(stride)), self._h)

    def profile_read(self, kind, reset=True):
        """(total kernel ms, launches) of one launch kind since the last reset."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _lib.check(_lib.load().dd_profile_read(self._h, int(kind), ctypes.byref(ms), ctypes.byref(n),
                                               1 if reset else 0), self._h)
        return ms.value, n.value

    def algorithmic_bytes(self, kind):
        b = ctypes.c_double()
        _lib.check(_lib.load().dd_algorithmic_bytes(self._h, int(kind), ctypes.byref(b)), self._h)
        return b.value
