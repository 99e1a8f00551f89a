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
