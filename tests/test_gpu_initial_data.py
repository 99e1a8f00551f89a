"""General initial data (eq. forward_initial_cond: E(0) = f_0, dE/dt(0) = f_1) on the GPU
against the FP64 oracle started from the same levels E^0 = f_0, E^{-1} = f_0 - dt f_1.

On the same float32 inputs: traces and energy rel L2 <= 1e-4, gradient <= 1e-3, with
checkpoint recompute (K < N_t, the level-0 state from the first checkpoint) and with every
level kept (one segment, the level-0 state from the kept tail); under both div-div forms and
for the paper-formula variant (the level-0 rows of the gradient are added after the last
adjoint step).  Clearing the data reproduces the start from rest bit for bit; batched jobs,
a single null argument and non-finite data are refused (the data set before stay).
"""

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / np.linalg.norm(b))


def _setup(name, form="R1", store_all=False, seed=71):
    import torch
    from paper_2508_07780_amd import Problem
    w = synth.small(name)
    if store_all:
        w.desc.ckpt_every = w.desc.n_steps
    f0, f1 = (f.astype(np.float32) for f in synth.initial_pulses(w.desc, synth.configs.SEED_BASE + seed))
    e32 = w.eps.astype(np.float32).astype(np.float64)
    s32 = w.sigma.astype(np.float32).astype(np.float64)
    d = Discretization(w.desc, divdiv_form=form).set_coefficients(e32, s32)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    if form != "R1":
        p.set_divdiv_form(form)
    return w, d, p, f0, f1


def _solve(p, w, cot, torch):
    tr, en = p.forward(w.sources, save=True, energy=True)
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge, gs = (g.cpu().numpy() for g in p.gradient())
    return tr[0].cpu().numpy(), en[0].cpu().numpy(), ge, gs


@pytest.mark.parametrize("name,form,store_all", [("tiny", "R1", False), ("ragged", "R1", False),
                                                 ("skinlet", "R1", True), ("ragged", "R2", False),
                                                 ("tiny", "R2", True)])
def test_initial_data_matches_oracle(name, form, store_all):
    import torch
    w, d, p, f0, f1 = _setup(name, form, store_all)
    src = w.sources[0]
    fw = forward(d, src, initial=(f0.astype(np.float64), f1.astype(np.float64)))
    cot = (0.5 * fw["traces"] + 1e-3 * synth.noise(fw["traces"].shape, 72)).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    print(f"[gpu] initial data {name} {form}: K {w.desc.ckpt_every}, steps {w.desc.n_steps}", flush=True)
    rest = _solve(p, w, cot, torch)
    p.set_initial_data(torch.tensor(f0, device="cuda"), torch.tensor(f1, device="cuda"))
    tr, en, ge, gs = _solve(p, w, cot, torch)
    errs = (_rel(tr, fw["traces"]), _rel(en, fw["energy"]), _rel(ge, ag["g_eps"]), _rel(gs, ag["g_sigma"]))
    print("[gpu]   traces %.2e energy %.2e g_eps %.2e g_sigma %.2e" % errs, flush=True)
    assert errs[0] <= 1e-4 and errs[1] <= 1e-4 and errs[2] <= 1e-3 and errs[3] <= 1e-3
    assert np.all(ge[~d.fem_free] == 0) and np.all(gs[~d.fem_free] == 0)
    # the data changes the solve (not a start from rest in disguise)
    assert _rel(tr, rest[0]) > 1e-2 and _rel(ge, rest[2]) > 1e-3
    p.set_initial_data(None, None)
    back = _solve(p, w, cot, torch)
    for a, b in zip(back, rest):
        np.testing.assert_array_equal(a, b)
    p.close()


def test_initial_data_paper_gradient_variant():
    import torch
    w, d, p, f0, f1 = _setup("ragged")
    src = w.sources[0]
    fw = forward(d, src, initial=(f0.astype(np.float64), f1.astype(np.float64)))
    cot = (0.5 * fw["traces"] + 1e-3 * synth.noise(fw["traces"].shape, 73)).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    p.set_initial_data(torch.tensor(f0, device="cuda"), torch.tensor(f1, device="cuda"))
    p.paper_gradient(True)
    p.forward(w.sources, save=True)
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    ge = p.gradient()[0].cpu().numpy()
    gp = p.gradient_paper()[0].cpu().numpy()
    e1, e2 = _rel(ge, ag["g_eps"]), _rel(gp, ag["g_eps_paper"])
    print(f"[gpu] initial data, paper variant: exact {e1:.2e} paper {e2:.2e}", flush=True)
    assert e1 <= 1e-3 and e2 <= 1e-3
    p.close()


def test_initial_data_refusals():
    import torch
    from paper_2508_07780_amd import DDError
    from paper_2508_07780_amd.batch import Batch
    w, d, p, f0, f1 = _setup("tiny")
    F0 = torch.tensor(f0, device="cuda")
    from paper_2508_07780_amd import _lib
    lib = _lib.load()
    rc = lib.dd_set_initial_data(p._h, ctypes_ptr(F0), None, None)
    assert rc == -1
    F1 = torch.tensor(f1, device="cuda")
    p.set_initial_data(F0, F1)
    t_ok = p.forward(w.sources, save=False).cpu().numpy()
    # a non-finite value is rejected and the data set before stay
    bad = F1.clone()
    bad[5, 1] = float("nan")
    with pytest.raises(DDError) as e:
        p.set_initial_data(F0, bad)
    assert e.value.code == -2
    np.testing.assert_array_equal(p.forward(w.sources, save=False).cpu().numpy(), t_ok)
    b = Batch(2)
    with pytest.raises(DDError) as e:
        b.submit(p, w.sources)
    assert e.value.code == -7
    b.close()
    p.close()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("n_steps,ckpt_every,n_src", [(1, 64, 1), (9, 1, 1), (7, 3, 1), (12, 5, 2)])
def test_initial_data_edge_cases(n_steps, ckpt_every, n_src):
    """One step (the level-0 state from the kept tail), a checkpoint every step, a ragged last
    segment, and two sources sharing the data (gradients summed over the sources)."""
    import torch
    from paper_2508_07780_amd import Problem
    w = synth.with_steps(synth.small("tiny"), n_steps)
    w.desc.ckpt_every = ckpt_every
    f0, f1 = (f.astype(np.float32) for f in synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 74))
    e32 = w.eps.astype(np.float32).astype(np.float64)
    s32 = w.sigma.astype(np.float32).astype(np.float64)
    d = Discretization(w.desc).set_coefficients(e32, s32)
    srcs = [w.sources[0]] * n_src
    if n_src == 2:
        srcs = [w.sources[0], synth.gauss_sine(w.sources[0].omega * 1.3, pol=(1.0, -0.4, 0.2))]
    fws = [forward(d, s, initial=(f0.astype(np.float64), f1.astype(np.float64))) for s in srcs]
    cots = [(0.5 * f["traces"] + 1e-3 * synth.noise(f["traces"].shape, 75 + i)).astype(np.float32)
            for i, f in enumerate(fws)]
    ge_o = np.zeros(d.n_fem)
    gs_o = np.zeros(d.n_fem)
    for f, c in zip(fws, cots):
        ag = adjoint_gradient(d, c.astype(np.float64), f)
        ge_o += ag["g_eps"]
        gs_o += ag["g_sigma"]
    print(f"[gpu] initial data edge: steps {n_steps}, K {ckpt_every}, sources {n_src}", flush=True)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    p.set_initial_data(torch.tensor(f0, device="cuda"), torch.tensor(f1, device="cuda"))
    tr = p.forward(srcs, save=True).cpu().numpy()
    p.adjoint(torch.tensor(np.stack(cots), device="cuda"))
    ge, gs = (g.cpu().numpy() for g in p.gradient())
    errs = [_rel(tr[i], fws[i]["traces"]) for i in range(n_src)]
    for g, go in ((ge, ge_o), (gs, gs_o)):
        # with very few steps the adjoint has not reached the free nodes: zero on both sides
        errs.append(_rel(g, go) if np.linalg.norm(go) > 0 else float(np.abs(g).max()))
    print("[gpu]   " + " ".join("%.2e" % e for e in errs), flush=True)
    assert max(errs[:n_src]) <= 1e-4 and errs[-2] <= 1e-3 and errs[-1] <= 1e-3
    p.close()


def test_cga_with_initial_data_matches_oracle():
    """Two CGA iterations (box "CGA") of a problem with initial data, against the oracle's CGA
    from the same levels; step sizes from the oracle's gradient at the initial guess (the first
    update moves eps by at most 0.5 and sigma by at most 0.1)."""
    import torch
    from oracle.cga import cga, solve_gradient
    from paper_2508_07780_amd import CGA, CGAParams, Problem
    w = synth.small("ragged")
    src = w.sources[0]
    f0, f1 = (f.astype(np.float32) for f in synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 76))
    init = (f0.astype(np.float64), f1.astype(np.float64))
    eobs = forward(Discretization(w.desc).set_coefficients(w.eps, w.sigma), src, initial=init)["traces"][None]
    n = len(w.eps)
    eps0, sig0 = np.ones(n), np.zeros(n)
    ge, gs, _ = solve_gradient(Discretization(w.desc), [src], eobs, None, init)(eps0, sig0)
    m = w.desc.h ** 3
    ae, asg = 0.5 / (np.abs(ge).max() / m), 0.1 / (np.abs(gs).max() / m)
    prm = dict(gamma_eps=1.0 / ae, gamma_sig=1.0 / asg, p=0.5, alpha_eps=ae, alpha_sig=asg, eps_max=8.0,
               sig_max=2.0)
    ref = cga(Discretization(w.desc), [src], eobs, eps0, sig0, prm, 2, initial=init)
    p = Problem(w.desc)
    p.set_initial_data(torch.tensor(f0, device="cuda"), torch.tensor(f1, device="cuda"))
    c = CGA(p, [src], torch.tensor(eobs, dtype=torch.float32, device="cuda"), torch.tensor(eps0, device="cuda"),
            torch.tensor(sig0, device="cuda"), CGAParams(**prm))
    for it in range(2):
        c.iterate()
        for f, t, base in (("eps", c.eps, eps0), ("sig", c.sigma, sig0)):
            err = _rel(t.cpu().numpy().astype(np.float64) - base, ref[it][f]["coef"] - base)
            print(f"[gpu] cga with initial data m={it} {f}: change rel L2 {err:.2e}", flush=True)
            assert err <= 2e-3
    c.close()
    p.close()


def test_initial_data_superposition_at_full_size():
    """The main workload's grid (160^3 outer nodes, 64^3 FEM hexes, 2000 steps) with initial
    data, where the oracle is too slow: the scheme is linear in (f_0, f_1, source), so the
    traces with both equal the traces with the source alone (from rest) plus those with the
    initial data alone (source of amplitude 0), to the FP32 rounding of 2000 steps (each
    solve stays within about 1e-6 of the FP64 recursion at this size): rel L2 <= 1e-5.
    Clearing the data reproduces the start from rest bit for bit at this size too."""
    import dataclasses
    import torch
    from paper_2508_07780_amd import Problem
    w = synth.c2()
    src = w.sources[0]
    silent = dataclasses.replace(src, amp=0.0)
    f0, f1 = (torch.tensor(f.astype(np.float32), device="cuda")
              for f in synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 77))
    print("[gpu] initial data at full size: 160^3, 2000 steps", flush=True)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma_true, dtype=torch.float32, device="cuda"))
    t_rest = p.forward([src], save=False).double()
    p.set_initial_data(f0, f1)
    t_both = p.forward([src], save=False).double()
    t_init = p.forward([silent], save=False).double()
    err = float(torch.linalg.norm(t_both - (t_rest + t_init)) / torch.linalg.norm(t_both))
    share = float(torch.linalg.norm(t_init) / torch.linalg.norm(t_both))
    print(f"[gpu]   superposition rel L2 {err:.2e}; the initial data's share of the traces {share:.2e}", flush=True)
    assert err <= 1e-5 and share > 1e-2
    p.set_initial_data(None, None)
    assert torch.equal(p.forward([src], save=False).double(), t_rest)
    p.close()
