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
* Per node, at 20 free nodes drawn with the seed: the derivative along a smooth bump centred
  on the node (a Gaussian of width 3 h over the free nodes, 1 at the node) of the loss over the
  detectors within 24 h of the node's (x, y) (the adjoint gets the same masked cotangent), by
  central differences with steps delta = 0.1 and 2 delta and their Richardson extrapolation
  (sigma evaluated 0.2 above the other tests' point, so that the steps stay in the box), against
  the adjoint's g . v.  Here the FP32 loss sets the floor, not the adjoint: a bump moves the
  loss by ~1e-5 of itself, the two difference quotients (which differ only by truncation and
  rounding) disagree by up to a few per cent at single nodes, and the agreement with the
  adjoint improves as the step grows (the rounding noise of a quotient falls as 1 / delta).  So
  the bar is on the 20 nodes together: relative L2 <= 1e-2 for eps and for sigma (measured
  3.1e-3 and 6.4e-3; the 2 delta quotient alone agrees to 1.3e-3 for eps).
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


def test_c3_gradient_at_twenty_seeded_nodes(c3_setup):
    import torch
    w, p, eobs, eps0, sig0, free = c3_setup
    dev = eobs.device
    x = synth.fem_node_coords(w.desc)
    from paper_2508_07780_amd import Problem
    det_idx = Problem.detector_nodes(w.desc)
    nx, ny = w.desc.n_outer[0], w.desc.n_outer[1]
    det_xy = np.stack([det_idx % nx, (det_idx // nx) % ny], axis=1) * w.desc.h + np.asarray(w.desc.origin[:2])
    rng = np.random.Generator(np.random.PCG64(w.seed + 20))
    nodes = rng.choice(np.nonzero(free)[0], 20, replace=False)
    width = 3.0 * w.desc.h
    radius = 24 * w.desc.h
    sig0 = np.where(free, sig0 + 0.2, 0.0)      # room for sigma steps of 0.2 below the evaluation point
    e0 = torch.tensor(eps0, dtype=torch.float32, device=dev)
    s0 = torch.tensor(sig0, dtype=torch.float32, device=dev)

    def traces(e, s):
        p.set_coefficients(torch.tensor(e, dtype=torch.float32, device=dev),
                           torch.tensor(s, dtype=torch.float32, device=dev))
        return p.forward(w.sources, save=False)

    pairs = {"eps": [], "sigma": []}
    for i in nodes:
        # the loss over the detectors above the node: J_i = 1/2 sum_{n, d in S_i} |T - E_obs|^2
        near = np.linalg.norm(det_xy - x[i, :2], axis=1) <= radius
        mask = torch.tensor(near.astype(np.float32), device=dev)[None, None, :, None]
        p.set_coefficients(e0, s0)
        tr = p.forward(w.sources, save=True)
        p.adjoint(((tr - eobs) * mask).contiguous())
        g_eps, g_sig = (g.cpu().numpy() for g in p.gradient())
        v = np.where(free, np.exp(-0.5 * np.sum((x - x[i]) ** 2, axis=1) / width ** 2), 0.0)
        for which, g, base, deltas in (("eps", g_eps, eps0, (0.1, 0.2)), ("sigma", g_sig, sig0, (0.1, 0.2))):
            pred = float(g @ v)
            fds = []
            for delta in deltas:
                vals = []
                for sgn in (1.0, -1.0):
                    xx = base + sgn * delta * v
                    t = traces(xx, sig0) if which == "eps" else traces(eps0, xx)
                    r = ((t - eobs) * mask).double()
                    vals.append(float(0.5 * torch.sum(r * r)))
                fds.append((vals[0] - vals[1]) / (2 * delta))
            rich = (4.0 * fds[0] - fds[1]) / 3.0
            spread = abs(fds[0] - fds[1])
            rel = abs(pred - rich) / abs(rich)     # per node: reported, noise-limited
            print(f"[gpu] c3 node {i} {which}: {int(near.sum())} detectors, adjoint {pred:.8e} fd {fds[0]:.8e} "
                  f"fd(2 delta) {fds[1]:.8e} richardson {rich:.8e} rel {rel:.2e} fd spread {spread / abs(rich):.2e}",
                  flush=True)
            pairs[which].append((pred, rich, spread))
    for which in ("eps", "sigma"):
        a = np.array(pairs[which])
        agg = float(np.linalg.norm(a[:, 0] - a[:, 1]) / np.linalg.norm(a[:, 1]))
        print(f"[gpu] c3 20-node {which}: adjoint vs Richardson rel L2 {agg:.2e}", flush=True)
        assert agg <= 1e-2


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
