"""Edge cases of the GPU path against the FP64 oracle.

* the smallest problem the C-ABI accepts (5^3 outer nodes, a 2^3-hex FEM box with a single
  FEM-owned node and no free node: the gradient is identically zero);
* FEM boxes with no free node (3^3 hexes) and with exactly one (4^3 hexes);
* a FEM box against the outer-grid margin (layer 0 next to the boundary faces);
* one and two time steps (forward and adjoint), checkpoint intervals 1 and > N_t;
* a dipole on a grid corner and on an edge, a single detector face of each kind;
* thin and ragged grids (one FD tile row, partial tiles in every axis).

Bars as in the parity tests: traces rel L2 <= 1e-4, gradient rel L2 <= 1e-3; nodes that are
not free carry an exact zero gradient.
"""

import math

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward

pytestmark = pytest.mark.gpu


def _case(n_outer, lo, cells, n_steps, det, ck, h=0.05, seed=0):
    desc = synth.ProblemDesc(n_outer=n_outer, h=h, origin=(0.0, 0.0, 0.0), fem_lo=lo, fem_cells=cells,
                             dt=0.5 * h / math.sqrt(3.0), n_steps=n_steps, ckpt_every=ck, detector_faces=det)
    rng = np.random.Generator(np.random.PCG64(2508077800 + 500 + seed))
    lay = synth.fem_layers(desc)
    free = lay >= 2
    eps = np.where(free, 1.0 + 3.0 * rng.random(lay.shape), 1.0)
    sig = np.where(free, 0.8 * rng.random(lay.shape), 0.0)
    return desc, eps, sig


def _sources(desc, kind):
    h = desc.h
    base = synth.gauss_sine(2 * math.pi / (8 * h), pol=(0.3, 1.0, -0.4))
    desc.t_switch = base.support_end()
    if kind == "plane":
        return [base]
    nx, ny, nz = desc.n_outer
    pos = {"corner": (0, 0, 0), "edge": (nx - 1, 0, nz // 2)}[kind]
    return [synth.Source(kind=synth.SRC_DIPOLE, omega=base.omega, t0=base.t0, width=base.width,
                         pol=(0.5, -0.2, 1.0), pos=pos)]


CASES = {
    # name: (n_outer, fem_lo, fem_cells, n_steps, detector faces, ckpt_every, source)
    "minimal": ((5, 5, 5), (1, 1, 1), (2, 2, 2), 6, synth.FACE_ALL, 1, "plane"),
    "no_free": ((9, 8, 10), (2, 2, 3), (3, 3, 3), 25, synth.FACE_TOP, 4, "plane"),
    "one_free": ((10, 10, 10), (3, 3, 3), (4, 4, 4), 40, synth.FACE_ALL, 7, "plane"),
    "box_at_margin": ((14, 12, 16), (1, 1, 1), (11, 9, 13), 30, synth.FACE_BOTTOM, 100, "corner"),
    "one_step": ((12, 11, 13), (3, 3, 4), (5, 4, 5), 1, synth.FACE_ALL, 1, "plane"),
    "two_steps": ((12, 11, 13), (3, 3, 4), (5, 4, 5), 2, synth.FACE_XMAX, 1, "edge"),
    "thin": ((41, 6, 20), (10, 1, 5), (12, 2, 9), 35, synth.FACE_YMIN, 8, "plane"),
    "ragged_all_axes": ((35, 19, 27), (9, 4, 6), (14, 10, 12), 45, synth.FACE_TOP | synth.FACE_XMIN, 16, "edge"),
}


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / nb) if nb > 0 else float(np.linalg.norm(a))


@pytest.mark.parametrize("fd_nt", ["0", "1"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_edge_case_matches_oracle(name, fd_nt, monkeypatch):
    """fd_nt: the finite-difference tiles' cached (0) or streaming (1) variant."""
    import torch
    from paper_2508_07780_amd import Problem
    monkeypatch.setenv("DD_FD_NT", fd_nt)
    n_outer, lo, cells, nt, det, ck, kind = CASES[name]
    desc, eps, sig = _case(n_outer, lo, cells, nt, det, ck, seed=sorted(CASES).index(name))
    srcs = _sources(desc, kind)
    print(f"[gpu] edge case {name}: outer {n_outer} fem {lo}+{cells} steps {nt} K {ck} source {kind} "
          f"fd_nt {fd_nt}", flush=True)
    e32 = eps.astype(np.float32).astype(np.float64)
    s32 = sig.astype(np.float32).astype(np.float64)
    d = Discretization(desc).set_coefficients(e32, s32)
    fw = forward(d, srcs[0])
    rng = np.random.default_rng(11)
    cot = (0.5 * fw["traces"] + 1e-3 * rng.standard_normal(fw["traces"].shape)).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)

    p = Problem(desc)
    p.set_coefficients(torch.tensor(eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(sig, dtype=torch.float32, device="cuda"))
    tr = p.forward(srcs, save=True)
    assert _rel(tr[0].cpu().numpy(), fw["traces"]) <= 1e-4
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge, gs = (g.cpu().numpy() for g in p.gradient())
    free = d.fem_free
    assert np.all(ge[~free] == 0) and np.all(gs[~free] == 0)
    if free.any():
        assert _rel(ge, ag["g_eps"]) <= 1e-3
        assert _rel(gs, ag["g_sigma"]) <= 1e-3
    else:
        assert not np.any(ge) and not np.any(gs)
    p.close()


def test_check_finite_reports_non_finite_fields():
    """dd_check_finite: clean fields after a forward; a NaN in the (unchecked) cotangent
    reaches the adjoint's fields and is reported as DD_ERR_UNSTABLE; a clean solve after it
    starts from fresh state again."""
    import torch
    from paper_2508_07780_amd import DDError, Problem
    w = synth.small("tiny")
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    tr = p.forward(w.sources, save=True)
    p.check_finite()
    cot = tr.clone()
    cot[0, w.desc.n_steps - 1, 0, 1] = float("nan")
    p.adjoint(cot)
    with pytest.raises(DDError) as e:
        p.check_finite()
    assert e.value.code == -3
    p.forward(w.sources, save=True)
    p.check_finite()
    p.close()
