"""The symmetric div-div form R2 on the GPU against the FP64 oracle's R2 discretisation.

R2 replaces the nodal product (eps - 1) E inside the element divergence by the element mean of
eps - 1 outside it; the paper's gradient formula (eq. gradeps with grad(eps~).E dropped) is
then the exact gradient.  Against the oracle with divdiv_form="R2" on the same float32 inputs:
traces rel L2 <= 1e-4, energy <= 1e-4, gradient (= paper formula) <= 1e-3, with checkpoint
recompute (K < N_t) and with every level kept; dd_gradient_paper equals dd_gradient; switching
back to R1 reproduces the R1 solve bit for bit; batched jobs of an R2 problem are refused.
"""

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b))


def _solve(p, w, cot, torch):
    tr, en = p.forward(w.sources, save=True, energy=True)
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge, gs = (g.cpu().numpy() for g in p.gradient())
    return tr[0].cpu().numpy(), en[0].cpu().numpy(), ge, gs


@pytest.mark.parametrize("name,store_all", [("tiny", False), ("ragged", False), ("skinlet", True)])
def test_r2_matches_oracle(name, store_all):
    import torch
    from paper_2508_07780_amd import Problem
    w = synth.small(name)
    if store_all:
        w.desc.ckpt_every = w.desc.n_steps
    e32 = w.eps.astype(np.float32).astype(np.float64)
    s32 = w.sigma.astype(np.float32).astype(np.float64)
    d = Discretization(w.desc, divdiv_form="R2").set_coefficients(e32, s32)
    src = w.sources[0]
    fw = forward(d, src)
    rng = np.random.default_rng(41)
    cot = (0.5 * fw["traces"] + 1e-3 * rng.standard_normal(fw["traces"].shape)).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    print(f"[gpu] R2 {name}: K {w.desc.ckpt_every}, steps {w.desc.n_steps}", flush=True)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    r1 = _solve(p, w, cot, torch)
    p.set_divdiv_form("R2")
    tr, en, ge, gs = _solve(p, w, cot, torch)
    errs = (_rel(tr, fw["traces"]), _rel(en, fw["energy"]), _rel(ge, ag["g_eps"]), _rel(gs, ag["g_sigma"]))
    print("[gpu]   traces %.2e energy %.2e g_eps %.2e g_sigma %.2e" % errs, flush=True)
    assert errs[0] <= 1e-4 and errs[1] <= 1e-4 and errs[2] <= 1e-3 and errs[3] <= 1e-3
    gp = p.gradient_paper()[0].cpu().numpy()
    np.testing.assert_array_equal(gp, ge)
    assert np.all(ge[~d.fem_free] == 0)
    p.set_divdiv_form("R1")
    back = _solve(p, w, cot, torch)
    for a, b in zip(back, r1):
        np.testing.assert_array_equal(a, b)
    p.close()


def test_r2_differs_from_r1_and_batch_refuses():
    import torch
    from paper_2508_07780_amd import DDError, Problem
    from paper_2508_07780_amd.batch import Batch
    w = synth.small("skinlet")
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    t1 = p.forward(w.sources, save=False).cpu().numpy()
    p.set_divdiv_form("R2")
    t2 = p.forward(w.sources, save=False).cpu().numpy()
    assert _rel(t2, t1) > 1e-6          # a different scheme where eps varies
    b = Batch(2)
    with pytest.raises(DDError) as e:
        b.submit(p, w.sources)
    assert e.value.code == -7
    b.close()
    p.close()


def test_r2_gradient_at_full_size_against_directional_differences():
    """The form R2 at the main workload's size (160^3 outer nodes, 64^3 FEM hexes, 2000 steps),
    where the oracle is too slow: the gradient (the paper formula, exact for R2) against
    central differences of the GPU loss along the gradient and a smooth field, for eps and
    sigma; steps 1e-2 and 2e-2 agree to 1 %, and their Richardson extrapolation matches the
    adjoint directional derivative to 1e-3.  Observations: the noise-free R2 traces of the
    true medium; evaluation point far from it (as in the 192^3 autograd test)."""
    import torch
    from paper_2508_07780_amd import Problem
    w = synth.c2()
    dev = torch.device("cuda", 0)
    print("[gpu] R2 at full size: 160^3, 2000 steps", flush=True)
    p = Problem(w.desc)
    p.set_divdiv_form("R2")
    f32 = lambda a: torch.tensor(a, dtype=torch.float32, device=dev)  # noqa: E731
    p.set_coefficients(f32(w.eps_true), f32(w.sigma_true))
    eobs = p.forward(w.sources, save=False).clone()
    free = synth.fem_layers(w.desc) >= 2
    eps0 = np.where(free, 1.05 + 0.2 * (w.eps_true - 1.0), 1.0)
    sig0 = np.where(free, 0.5 * w.sigma_true + 0.05, 0.0)

    def loss(e, s):
        p.set_coefficients(f32(e), f32(s))
        r = (p.forward(w.sources, save=False) - eobs).double()
        return float(0.5 * torch.sum(r * r))

    p.set_coefficients(f32(eps0), f32(sig0))
    tr = p.forward(w.sources, save=True)
    p.adjoint_misfit(tr, eobs)
    g_eps, g_sig = (g.cpu().numpy() for g in p.gradient())
    np.testing.assert_array_equal(p.gradient_paper()[0].cpu().numpy(), g_eps)
    x = synth.fem_node_coords(w.desc)
    rng = np.random.Generator(np.random.PCG64(w.seed + 7))
    k = rng.normal(size=3) * 2.0 * np.pi
    smooth = np.where(free, 1.0 + 0.5 * np.sin(x @ k + rng.uniform(0, 2 * np.pi)), 0.0)
    for which, g, base in (("eps", g_eps, eps0), ("sigma", g_sig, sig0)):
        for name, d in (("gradient", np.where(free, g, 0.0)), ("smooth", smooth)):
            d = d / np.abs(d).max()
            pred = float(g @ d)
            fds = []
            for delta in (1e-2, 2e-2):
                vals = [loss(base + sg * delta * d if which == "eps" else eps0,
                             base + sg * delta * d if which == "sigma" else sig0) for sg in (1.0, -1.0)]
                fds.append((vals[0] - vals[1]) / (2 * delta))
            rich = (4.0 * fds[0] - fds[1]) / 3.0
            rel = abs(pred - rich) / abs(rich)
            print(f"[gpu]   R2 {which}/{name}: adjoint {pred:.8e} fd {fds[0]:.8e} / {fds[1]:.8e} "
                  f"richardson {rich:.8e} rel {rel:.2e}", flush=True)
            assert abs(fds[0] - fds[1]) <= 1e-2 * abs(fds[0]), "finite differences not converged"
            assert rel <= 1e-3
    p.close()
