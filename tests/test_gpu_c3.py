"""Differentiation at full size: 192^3 outer nodes, 96^3 FEM hexes (5.3M tetrahedra),
1500 steps, forward checkpoints every 64 steps, through the torch.autograd.Function.

* The gradient from the hand adjoint (checkpointed recompute) is checked against central
  finite differences of the loss computed by the GPU forward itself, along directions over
  all free nodes (eps and sigma separately): the gradient direction and a smooth seeded
  field.  Random-sign directions are not used: their directional derivative cancels by
  orders of magnitude and drowns in the FP32 rounding of the loss (J ~ 3e4 here).  The observed data here are
  the noise-free traces of the true medium and the evaluation point is far from it, so the
  residual is the full backscattered misfit and FP32 rounding in the loss stays far below
  the finite-difference signal; steps delta and
  2*delta must agree to 1% (the truncation error is then O(delta^2)), and their Richardson
  extrapolation is compared with the adjoint directional derivative.
* The checkpointed gradient (K = 64, 24 recomputed segments) equals, bit for bit, the one
  computed with every forward level stored (K >= N_t, no recompute).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3_setup():
    import torch
    from paper_2508_07780_amd import Problem
    w = synth.c3()
    print(f"[gpu] c3 setup {w.desc.n_outer} fem {w.desc.fem_cells} steps {w.desc.n_steps}", flush=True)
    dev = torch.device("cuda", 0)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device=dev),
                       torch.tensor(w.sigma_true, dtype=torch.float32, device=dev))
    eobs = p.forward(w.sources, save=False).clone()
    free = synth.fem_layers(w.desc) >= 2
    # evaluation point far from the truth: the residual is the full backscattered misfit,
    # so FP32 rounding of the traces (~5e-7 of the direct wave) is small relative to it
    eps0 = np.where(free, 1.05 + 0.2 * (w.eps_true - 1.0), 1.0)
    sig0 = np.where(free, 0.5 * w.sigma_true + 0.05, 0.0)
    return w, p, eobs, eps0, sig0, free


def _loss(p, w, eobs, eps, sig):
    import torch
    from paper_2508_07780_amd.autograd import solve
    tr = solve(p, eps, sig, w.sources)
    r = (tr - eobs).double()
    return 0.5 * torch.sum(r * r)


def _directions(w, free, g):
    """Directions without random-sign cancellation: the gradient itself (steepest descent)
    and a smooth low-frequency field over the free nodes, both scaled to max |d| = 1."""
    x = synth.fem_node_coords(w.desc)
    rng = np.random.Generator(np.random.PCG64(w.seed + 5))
    k = rng.normal(size=3) * 2.0 * np.pi
    smooth = np.where(free, 1.0 + 0.5 * np.sin(x @ k + rng.uniform(0, 2 * np.pi)), 0.0)
    out = []
    for d in (np.where(free, g, 0.0), smooth):
        out.append(d / np.abs(d).max())
    return out


def test_c3_gradient_directional_finite_differences(c3_setup):
    import torch
    w, p, eobs, eps0, sig0, free = c3_setup
    dev = eobs.device
    eps = torch.tensor(eps0, dtype=torch.float32, device=dev, requires_grad=True)
    sig = torch.tensor(sig0, dtype=torch.float32, device=dev, requires_grad=True)
    J = _loss(p, w, eobs, eps, sig)
    J.backward()
    g_eps = eps.grad.double().cpu().numpy()
    g_sig = sig.grad.double().cpu().numpy()
    assert np.isfinite(g_eps).all() and np.isfinite(g_sig).all()
    assert np.all(g_eps[~free] == 0) and np.all(g_sig[~free] == 0)
    for which, g, base in (("eps", g_eps, eps0), ("sigma", g_sig, sig0)):
        for name, d in zip(("gradient", "smooth"), _directions(w, free, g)):
            pred = float(g @ d)
            fds = []
            for delta in (1e-2, 2e-2):
                vals = []
                for sgn in (1.0, -1.0):
                    x = base + sgn * delta * d
                    e = torch.tensor(x if which == "eps" else eps0, dtype=torch.float32, device=dev)
                    s = torch.tensor(sig0 if which == "eps" else x, dtype=torch.float32, device=dev)
                    with torch.no_grad():
                        vals.append(float(_loss(p, w, eobs, e, s)))
                fds.append((vals[0] - vals[1]) / (2 * delta))
            rich = (4.0 * fds[0] - fds[1]) / 3.0
            print(f"[gpu] c3 {which}/{name}: J {float(J.detach()):.6e} adjoint {pred:.8e} fd(1e-2) {fds[0]:.8e} "
                  f"fd(2e-2) {fds[1]:.8e} richardson {rich:.8e} rel {abs(pred - rich) / abs(rich):.2e}", flush=True)
            assert abs(fds[0] - fds[1]) <= 1e-2 * abs(fds[0]), "finite differences not converged"
            assert abs(pred - rich) <= 1e-3 * abs(rich)


def test_c3_checkpointed_gradient_equals_store_all(c3_setup):
    import torch
    from paper_2508_07780_amd import Problem
    w, p, eobs, eps0, sig0, free = c3_setup
    dev = eobs.device
    e = torch.tensor(eps0, dtype=torch.float32, device=dev)
    s = torch.tensor(sig0, dtype=torch.float32, device=dev)
    p.set_coefficients(e, s)
    tr = p.forward(w.sources, save=True)
    cot = (tr - eobs).contiguous()
    p.adjoint(cot)
    g_ck = [g.clone() for g in p.gradient()]
    w_all = synth.c3()
    w_all.desc.ckpt_every = w_all.desc.n_steps
    q = Problem(w_all.desc)
    q.set_coefficients(e, s)
    tr2 = q.forward(w.sources, save=True)
    assert torch.equal(tr, tr2)
    q.adjoint(cot)
    g_all = q.gradient()
    q.close()
    assert torch.equal(g_ck[0], g_all[0]) and torch.equal(g_ck[1], g_all[1])
