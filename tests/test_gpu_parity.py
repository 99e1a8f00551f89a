"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Bars (FP32 state vs FP64 oracle): traces relative L2 <= 1e-4, gradient relative
L2 <= 1e-3.  The oracle gets the float32-rounded coefficients the GPU sees, and
both sides get the same float32 cotangent.  Cases span several FD tiles and FEM
partitions with ragged tails, non-cubic grids and FEM boxes, every detector
face, conductivity, the absorbing-face switch and sources of every kind.
"""

import math
import os

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward

pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-4
GRAD_TOL = 1e-3


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b))


def _report(**kw):
    """Append measured parity errors to $DD_PARITY_REPORT (one line per check)."""
    path = os.environ.get("DD_PARITY_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(" ".join(f"{k}={v}" for k, v in kw.items()) + "\n")


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _gpu_problem(torch, w):
    from paper_2508_07780_amd import Problem
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    return p


def _oracle(w):
    d = Discretization(w.desc).set_coefficients(_f32(w.eps), _f32(w.sigma))
    return d


CASES = ["tiny", "ragged", "skinlet", "c1"]


def _workload(name):
    return synth.c1() if name == "c1" else synth.small(name)


# DD_FD_NT: the finite-difference tiles' cached variant (2-plane z-chunks, ordinary accesses) and
# their streaming variant (8-plane z-chunks, non-temporal own-node accesses, the adjoint's top-face
# cotangent loaded ahead when the top face closes a full chunk), which grids whose two E levels
# exceed the last-level cache take by default
FD_VARIANTS = ["0", "1"]


@pytest.mark.parametrize("fd_nt", FD_VARIANTS)
@pytest.mark.parametrize("name", CASES)
def test_forward_traces_and_energy(torch_cuda, name, fd_nt, monkeypatch):
    torch = torch_cuda
    monkeypatch.setenv("DD_FD_NT", fd_nt)
    w = _workload(name)
    print(f"[gpu] forward parity {name} {w.desc.n_outer} fem {w.desc.fem_cells} steps {w.desc.n_steps} "
          f"fd_nt {fd_nt}", flush=True)
    p = _gpu_problem(torch, w)
    tr, en = p.forward(w.sources, save=False, energy=True)
    torch.cuda.synchronize()
    d = _oracle(w)
    ref = forward(d, w.sources[0])
    err = _rel(tr[0].cpu().numpy(), ref["traces"])
    eerr = _rel(en[0].cpu().numpy(), ref["energy"])
    _report(check="forward", case=name, fd_nt=fd_nt, trace_rel_l2=f"{err:.3e}", energy_rel_l2=f"{eerr:.3e}")
    assert err <= TRACE_TOL, err
    assert eerr <= 1e-4, eerr


@pytest.mark.parametrize("fd_nt", FD_VARIANTS)
@pytest.mark.parametrize("name", CASES)
def test_gradient(torch_cuda, name, fd_nt, monkeypatch):
    torch = torch_cuda
    monkeypatch.setenv("DD_FD_NT", fd_nt)
    w = _workload(name)
    print(f"[gpu] gradient parity {name} fd_nt {fd_nt}", flush=True)
    d = _oracle(w)
    fw = forward(d, w.sources[0])
    rng = np.random.default_rng(7)
    eobs = fw["traces"] * (1.0 + 0.03 * rng.standard_normal(fw["traces"].shape)) * 0.8
    cot = (fw["traces"] - eobs).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    p = _gpu_problem(torch, w)
    p.forward(w.sources, save=True)
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge, gs = p.gradient()
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    e1 = _rel(ge, ag["g_eps"])
    e2 = _rel(gs, ag["g_sigma"]) if np.any(ag["g_sigma"]) else 0.0
    _report(check="gradient", case=name, fd_nt=fd_nt, g_eps_rel_l2=f"{e1:.3e}", g_sigma_rel_l2=f"{e2:.3e}")
    assert e1 <= GRAD_TOL and e2 <= GRAD_TOL, (e1, e2)
    free = d.fem_free
    assert np.all(ge[~free] == 0) and np.all(gs[~free] == 0)


@pytest.mark.parametrize("name", CASES)
def test_streaming_variant_is_bitwise_identical(torch_cuda, name, monkeypatch):
    """The two finite-difference tile variants differ in z-chunk length and access kind only, not
    in any node's arithmetic: a saving forward and the misfit adjoint (cotangent traces - obs
    formed in the tiles, through the top-face prefetch where the top face closes a full chunk)
    give the same traces and gradients bit for bit; the energy sums (per-tile partials) agree to
    rounding."""
    torch = torch_cuda
    w = _workload(name)
    out = {}
    for fd_nt in FD_VARIANTS:
        monkeypatch.setenv("DD_FD_NT", fd_nt)
        print(f"[gpu] tile variant {fd_nt} on {name}", flush=True)
        p = _gpu_problem(torch, w)
        tr, en = p.forward(w.sources, save=True, energy=True)
        tr = tr.clone()
        obs = (0.7 * tr + 1e-3).contiguous()
        p.adjoint_misfit(tr, obs)
        ge, gs = p.gradient()
        torch.cuda.synchronize()
        out[fd_nt] = (tr.cpu(), en.cpu(), ge.cpu(), gs.cpu())
        p.close()
    a, b = out["0"], out["1"]
    assert torch.equal(a[0], b[0]), "traces differ between the tile variants"
    assert torch.equal(a[2], b[2]) and torch.equal(a[3], b[3]), "gradients differ between the tile variants"
    assert float((a[1] - b[1]).norm() / a[1].norm()) <= 1e-12


def test_checkpoint_interval_does_not_change_gradient_bits(torch_cuda):
    torch = torch_cuda
    base = synth.small("ragged")
    rng = np.random.default_rng(3)
    n_det = len(Discretization(base.desc).det)
    cot = torch.tensor(rng.standard_normal((1, base.desc.n_steps, n_det, 3)).astype(np.float32), device="cuda")
    outs = []
    for K in (1, 7, 16, base.desc.n_steps, 4 * base.desc.n_steps):
        w = synth.small("ragged")
        w.desc.ckpt_every = K
        print(f"[gpu] checkpoint K={K}", flush=True)
        p = _gpu_problem(torch, w)
        p.forward(w.sources, save=True)
        p.adjoint(cot)
        outs.append([g.cpu().numpy() for g in p.gradient()])
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_repeat_runs_are_bitwise_identical(torch_cuda):
    torch = torch_cuda
    w = synth.small("skinlet")
    p = _gpu_problem(torch, w)
    a = p.forward(w.sources, save=True).clone()
    b = p.forward(w.sources, save=True).clone()
    assert torch.equal(a, b)
    cot = (a * 0.1).contiguous()
    p.adjoint(cot)
    g1 = [g.clone() for g in p.gradient()]
    p.adjoint(cot)
    g2 = p.gradient()
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])


def test_sources_of_every_kind_and_multi_source_sum(torch_cuda):
    torch = torch_cuda
    w = synth.small("ragged")
    nx, ny, nz = w.desc.n_outer
    srcs = [
        synth.Source(kind=synth.SRC_SINE1, omega=2 * math.pi / (12 * w.desc.h), amp=0.7, pol=(0.0, 1.0, 0.0)),
        synth.gauss_sine(2 * math.pi / (10 * w.desc.h), pol=(1.0, 0.2, 0.0)),
        synth.Source(kind=synth.SRC_DIPOLE, omega=2 * math.pi / (12 * w.desc.h), t0=18 * w.desc.h,
                     width=6 * w.desc.h, pol=(0.2, -0.5, 1.0), pos=(nx // 2, ny // 2, nz - 4)),
    ]
    d = _oracle(w)
    p = _gpu_problem(torch, w)
    tr = p.forward(srcs, save=True).cpu().numpy()
    rng = np.random.default_rng(9)
    cots = rng.standard_normal(tr.shape).astype(np.float32)
    g_sum = np.zeros(d.n_fem)
    for i, s in enumerate(srcs):
        print(f"[gpu] source kind {s.kind}", flush=True)
        ref = forward(d, s)
        assert _rel(tr[i], ref["traces"]) <= TRACE_TOL
        g_sum += adjoint_gradient(d, cots[i].astype(np.float64), ref)["g_eps"]
    p.adjoint(torch.tensor(cots, device="cuda"))
    ge, _ = p.gradient()
    assert _rel(ge.cpu().numpy(), g_sum) <= GRAD_TOL


def test_top_face_switch_mid_run_gradient(torch_cuda):
    torch = torch_cuda
    w = synth.small("tiny")
    w.desc.t_switch = 13.5 * w.desc.dt      # source cut while still on: switch inside the run
    d = _oracle(w)
    fw = forward(d, w.sources[0])
    cot = (0.5 * fw["traces"]).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    p = _gpu_problem(torch, w)
    tr = p.forward(w.sources, save=True)
    assert _rel(tr[0].cpu().numpy(), fw["traces"]) <= TRACE_TOL
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge, gs = p.gradient()
    assert _rel(ge.cpu().numpy(), ag["g_eps"]) <= GRAD_TOL
    assert _rel(gs.cpu().numpy(), ag["g_sigma"]) <= GRAD_TOL


def test_error_paths(torch_cuda):
    torch = torch_cuda
    from paper_2508_07780_amd import DDError
    w = synth.small("tiny")
    p = _gpu_problem(torch, w)
    with pytest.raises(DDError) as e:
        p.adjoint(torch.zeros((1, w.desc.n_steps, p.n_det, 3), device="cuda"))
    assert e.value.code == -6
    with pytest.raises(DDError) as e:
        p.gradient()
    assert e.value.code == -6
    bad = torch.tensor(w.eps, dtype=torch.float32, device="cuda")
    lay = synth.fem_layers(w.desc)
    bad[torch.tensor(lay == 1, device="cuda")] = 2.0
    with pytest.raises(DDError) as e:
        p.set_coefficients(bad, torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    assert e.value.code == -2
    # the previous coefficients stay in force
    tr = p.forward(w.sources, save=False)
    ref = forward(_oracle(w), w.sources[0])["traces"]
    assert _rel(tr[0].cpu().numpy(), ref) <= TRACE_TOL
    nan = torch.tensor(w.sigma, dtype=torch.float32, device="cuda")
    nan[0] = float("nan")
    with pytest.raises(DDError):
        p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"), nan)


def test_autograd_function_matches_c_abi(torch_cuda):
    torch = torch_cuda
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.autograd import solve
    w = synth.small("skinlet")
    d = _oracle(w)
    fw = forward(d, w.sources[0])
    # observations from the oracle's traces (the loss's cotangent is then the oracle's own)
    eobs_np = (0.9 * fw["traces"]).astype(np.float32)
    ag = adjoint_gradient(d, fw["traces"] - eobs_np.astype(np.float64), fw)
    p = Problem(w.desc)
    eps = torch.tensor(w.eps, dtype=torch.float32, device="cuda", requires_grad=True)
    sig = torch.tensor(w.sigma, dtype=torch.float32, device="cuda", requires_grad=True)
    tr = solve(p, eps, sig, w.sources)
    eobs = torch.tensor(eobs_np[None], device="cuda")
    loss = 0.5 * ((tr - eobs) ** 2).sum()
    loss.backward()
    assert _rel(eps.grad.cpu().numpy(), ag["g_eps"]) <= GRAD_TOL
    assert _rel(sig.grad.cpu().numpy(), ag["g_sigma"]) <= GRAD_TOL


def test_autograd_refuses_a_stale_saved_forward(torch_cuda):
    """Two solves on one Problem before backward: the first node's saved forward was replaced,
    so its backward raises instead of returning the other solve's gradient.  One Problem per
    solve works, and eps given on the FEM lattice's 3-D shape gets a gradient of that shape."""
    torch = torch_cuda
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.autograd import solve
    w = synth.small("tiny")
    shape = tuple(int(c) + 1 for c in w.desc.fem_cells)[::-1]
    eps = torch.tensor(w.eps.reshape(shape), dtype=torch.float32, device="cuda", requires_grad=True)
    sig = torch.tensor(w.sigma, dtype=torch.float32, device="cuda", requires_grad=True)
    p = Problem(w.desc)
    a = solve(p, eps, sig, w.sources)
    b = solve(p, eps.detach() * 1.0, sig.detach(), w.sources)
    with pytest.raises(RuntimeError):
        (a.sum() + b.sum()).backward()
    q = Problem(w.desc)
    a = solve(q, eps, sig, w.sources)
    b = solve(p, eps, sig, w.sources)
    (0.5 * (a ** 2).sum() + 0.5 * (b ** 2).sum()).backward()
    assert eps.grad.shape == eps.shape and sig.grad.shape == sig.shape
    # both solves are the same, so the summed gradient is twice one of them
    ref = Problem(w.desc)
    eps1 = eps.detach().clone().requires_grad_(True)
    sig1 = sig.detach().clone().requires_grad_(True)
    (0.5 * (solve(ref, eps1, sig1, w.sources) ** 2).sum()).backward()
    assert torch.allclose(eps.grad, 2 * eps1.grad, rtol=1e-6, atol=0)
    assert torch.allclose(sig.grad, 2 * sig1.grad, rtol=1e-6, atol=0)


@pytest.mark.parametrize("gather", ["1", "0"])
@pytest.mark.parametrize("name", ["ragged", "skinlet"])
def test_element_colored_fem_path(torch_cuda, name, gather, monkeypatch):
    """The element-colored FEM kernel (general tetrahedral meshes) against the oracle, in its
    node-gather form (default) and its colour-by-colour scatter form."""
    torch = torch_cuda
    monkeypatch.setenv("DD_FEM_PATH", "element")
    monkeypatch.setenv("DD_FEM_GATHER", gather)
    w = synth.small(name)
    print(f"[gpu] element path {name} gather {gather}", flush=True)
    d = _oracle(w)
    fw = forward(d, w.sources[0])
    cot = (0.3 * fw["traces"]).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    p = _gpu_problem(torch, w)
    tr = p.forward(w.sources, save=True)
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge, gs = p.gradient()
    e0 = _rel(tr[0].cpu().numpy(), fw["traces"])
    e1 = _rel(ge.cpu().numpy(), ag["g_eps"])
    e2 = _rel(gs.cpu().numpy(), ag["g_sigma"])
    _report(check="element_path", case=name, trace_rel_l2=f"{e0:.3e}", g_eps_rel_l2=f"{e1:.3e}", g_sigma_rel_l2=f"{e2:.3e}")
    assert e0 <= TRACE_TOL and e1 <= GRAD_TOL and e2 <= GRAD_TOL
