"""ctypes view of the C-ABI in include/dd.h (argument marshalling only)."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DD_LIB_PATH") or os.path.join(HERE, "libddfem.so")

DD_OK = 0
ERRORS = {
    -1: "DD_ERR_INVALID_ARG", -2: "DD_ERR_CONSTRAINT", -3: "DD_ERR_UNSTABLE", -4: "DD_ERR_OOM",
    -5: "DD_ERR_HIP", -6: "DD_ERR_STATE", -7: "DD_ERR_UNSUPPORTED",
}

EXPORTS = [
    "dd_create", "dd_destroy", "dd_sizes", "dd_detector_nodes", "dd_footprint_bytes",
    "dd_set_coefficients", "dd_forward", "dd_adjoint", "dd_gradient", "dd_error_string", "dd_last_error",
    "dd_profile_enable", "dd_profile_read", "dd_algorithmic_bytes", "dd_debug_fem_apply",
    "dd_batch_create", "dd_batch_destroy", "dd_batch_submit", "dd_batch_step", "dd_batch_poll",
    "dd_adjoint_misfit", "dd_cga_create", "dd_cga_destroy", "dd_cga_update", "dd_cga_get_info",
    "dd_paper_gradient_enable", "dd_gradient_paper", "dd_misfit", "dd_set_divdiv_form", "dd_set_graph", "dd_graph_stats", "dd_set_initial_data", "dd_check_finite", "dd_batch_set_fill",
    "dd_misfit_noalloc", "dd_misfit_taper", "dd_set_coefficients_async", "dd_coefficients_status",
    "dd_cga_steps_from_gradient", "dd_create_mesh", "dd_debug_fem_apply_mesh", "dd_meshref_create",
    "dd_meshref_sizes", "dd_meshref_result", "dd_meshref_interpolate", "dd_meshref_destroy",
]

(PROF_FD_FWD, PROF_FEM_FWD, PROF_FD_ADJ, PROF_FEM_ADJ, PROF_FEM_RECOMPUTE, PROF_STEP_FWD, PROF_STEP_ADJ,
 PROF_PAIR_FWD, PROF_PAIR_ADJ, PROF_PAIR2_FWD, PROF_PAIR2_ADJ) = range(11)
PROF_NAMES = ["fd_step_fwd", "fem_step_fwd", "fd_step_adj", "fem_step_adj", "fem_step_recompute",
              "step_fwd", "step_adj", "pair_fwd", "pair_adj", "pair2_fwd", "pair2_adj"]


CKPT_FEM_IFACE, CKPT_STORE_ALL, CKPT_FULL = 0, 1, 2


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("n_outer", ctypes.c_int32 * 3),
        ("h", ctypes.c_double),
        ("origin", ctypes.c_double * 3),
        ("fem_lo", ctypes.c_int32 * 3),
        ("fem_cells", ctypes.c_int32 * 3),
        ("overlap", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("n_steps", ctypes.c_int32),
        ("ckpt_every", ctypes.c_int32),
        ("s_stab", ctypes.c_double),
        ("detector_faces", ctypes.c_uint32),
        ("absorbing_faces", ctypes.c_uint32),
        ("t_switch", ctypes.c_double),
        ("ckpt_mode", ctypes.c_int32),
    ]


class Tikhonov(ctypes.Structure):
    _fields_ = [
        ("gamma_eps", ctypes.c_double),
        ("gamma_sig", ctypes.c_double),
        ("eps0_dev", ctypes.c_void_p),
        ("sigma0_dev", ctypes.c_void_p),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Source(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("omega", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("width", ctypes.c_double),
        ("amp", ctypes.c_double),
        ("dir", ctypes.c_double * 3),
        ("pol", ctypes.c_double * 3),
        ("pos", ctypes.c_int32 * 3),
    ]


class CgaParams(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in (
        "gamma_eps", "gamma_sig", "p", "alpha_eps", "alpha_sig", "eps_max", "sig_max",
        "eta1_eps", "eta1_sig", "eta2_eps", "eta2_sig")]


class CgaInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32)] + [
        (name, ctypes.c_double * 2) for name in (
            "grad_norm", "step_norm", "beta", "alpha_used", "alpha_next", "gamma_used", "gamma_next",
            "change_norm")]


class DDError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libddfem.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2508_07780_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.dd_create.argtypes = [ctypes.POINTER(ProblemDesc), ALLOC_FN, FREE_FN, P, ctypes.POINTER(P)]
    lib.dd_create_mesh.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ALLOC_FN, FREE_FN, P,
                                   ctypes.POINTER(P)]
    lib.dd_destroy.argtypes = [P]
    lib.dd_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_int64)]
    lib.dd_detector_nodes.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.dd_footprint_bytes.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int32]
    lib.dd_footprint_bytes.restype = ctypes.c_size_t
    lib.dd_set_coefficients.argtypes = [P, P, P, P]
    lib.dd_set_coefficients_async.argtypes = [P, P, P, P]
    lib.dd_coefficients_status.argtypes = [P, P]
    lib.dd_cga_steps_from_gradient.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, P]
    lib.dd_forward.argtypes = [P, ctypes.POINTER(Source), ctypes.c_int32, P, ctypes.c_int32, P, P]
    lib.dd_adjoint.argtypes = [P, P, P]
    lib.dd_gradient.argtypes = [P, P, P, ctypes.POINTER(Tikhonov), P]
    lib.dd_error_string.argtypes = [ctypes.c_int]
    lib.dd_error_string.restype = ctypes.c_char_p
    lib.dd_last_error.argtypes = [P]
    lib.dd_last_error.restype = ctypes.c_char_p
    lib.dd_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.dd_profile_read.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_int32]
    lib.dd_algorithmic_bytes.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.dd_debug_fem_apply.argtypes = [ctypes.POINTER(ProblemDesc), P, P, ctypes.c_int32, P, P]
    lib.dd_debug_fem_apply_mesh.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int64, P, ctypes.c_int64, P, P, P,
                                            ctypes.c_int32, P, P]
    lib.dd_meshref_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int64, P, ctypes.c_int64, P, P, P,
                                      ctypes.c_double, ctypes.c_double, ctypes.POINTER(P)]
    lib.dd_meshref_sizes.argtypes = [P] + [ctypes.POINTER(ctypes.c_int64)] * 4
    lib.dd_meshref_result.argtypes = [P, P, P, P]
    lib.dd_meshref_interpolate.argtypes = [P, P, P]
    lib.dd_meshref_destroy.argtypes = [P]
    lib.dd_batch_create.argtypes = [ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.dd_batch_destroy.argtypes = [P]
    lib.dd_batch_submit.argtypes = [P, P, ctypes.POINTER(Source), ctypes.c_int32, P, P, P, P,
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.dd_batch_step.argtypes = [P, ctypes.c_int32, P]
    lib.dd_batch_poll.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]
    lib.dd_adjoint_misfit.argtypes = [P, P, P, P]
    lib.dd_paper_gradient_enable.argtypes = [P, ctypes.c_int32]
    lib.dd_misfit.argtypes = [P, P, P, ctypes.c_int32, P, P, P, P]
    lib.dd_misfit_noalloc.argtypes = [P, P, P, ctypes.c_int32, P, P, P, P]
    lib.dd_misfit_taper.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, P]
    lib.dd_set_divdiv_form.argtypes = [P, ctypes.c_int32]
    lib.dd_set_graph.argtypes = [P, ctypes.c_int32]
    lib.dd_graph_stats.argtypes = [P, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.dd_gradient_paper.argtypes = [P, P, P, P]
    lib.dd_set_initial_data.argtypes = [P, P, P, P]
    lib.dd_check_finite.argtypes = [P, P]
    lib.dd_batch_set_fill.argtypes = [P, ctypes.c_int64]
    lib.dd_cga_create.argtypes = [P, ctypes.POINTER(CgaParams), P, P, P, ctypes.POINTER(P)]
    lib.dd_cga_destroy.argtypes = [P]
    lib.dd_cga_update.argtypes = [P, P, P, P, P, P]
    lib.dd_cga_get_info.argtypes = [P, ctypes.POINTER(CgaInfo), P]
    for name in EXPORTS:
        if name not in ("dd_footprint_bytes", "dd_error_string", "dd_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc, handle=None):
    if rc != DD_OK:
        msg = ""
        if handle:
            msg = (load().dd_last_error(handle) or b"").decode()
        raise DDError(rc, msg)


def make_desc(d):
    """ProblemDesc from any object with the synth.ProblemDesc fields."""
    c = ProblemDesc()
    for a in range(3):
        c.n_outer[a] = int(d.n_outer[a])
        c.origin[a] = float(d.origin[a])
        c.fem_lo[a] = int(d.fem_lo[a])
        c.fem_cells[a] = int(d.fem_cells[a])
    c.h = float(d.h)
    c.dt = float(d.dt)
    c.n_steps = int(d.n_steps)
    c.ckpt_every = int(d.ckpt_every)
    c.detector_faces = int(d.detector_faces)
    c.absorbing_faces = int(d.absorbing_faces)
    c.t_switch = float(d.t_switch)
    c.overlap = int(getattr(d, "overlap", 2))
    c.s_stab = float(getattr(d, "s_stab", 1.0))
    c.ckpt_mode = int(getattr(d, "ckpt_mode", CKPT_FEM_IFACE))
    return c


def make_sources(srcs):
    arr = (Source * len(srcs))()
    for i, s in enumerate(srcs):
        arr[i].kind = int(s.kind)
        arr[i].omega = float(s.omega)
        arr[i].t0 = float(s.t0)
        arr[i].width = float(s.width)
        arr[i].amp = float(s.amp)
        d = getattr(s, "dir", (0.0, 0.0, 0.0))
        for a in range(3):
            arr[i].dir[a] = float(d[a])
            arr[i].pol[a] = float(s.pol[a])
            arr[i].pos[a] = int(s.pos[a])
    return arr
