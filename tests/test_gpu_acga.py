"""Box "ACGA" on the GPU against the FP64 oracle: the CGA on a refined mesh (per-node lumped
masses in its inner products, the inserted nodes free), and the adaptive loop itself (the CGA
on the uniform mesh, marking by eq. meshref, longest-edge bisection and interpolation in the
library's host code, the CGA on each refined mesh, step 4's stop test).

Bars as for the CGA (tests/test_gpu_cga.py): the coefficient change rel L2 <= 2e-3 per
iteration and the gradient norms rel <= 1e-3 on one mesh.  On each refined level the CGA
starts from each side's own result of the level before and is centred on it, so a level
carries the earlier levels' error (<= 2e-3 of their change) on top of its own: its gradient
norms and its distance from its start are held to 4e-3, and so is the final coefficients'
change from the initial guess.  The marks are an integer decision taken from the results of
the two sides: the test checks that no node of a tested field lies within 1e-3 (relative) of
its threshold, well above the float32 solves' error in the coefficients, so that both sides
must take the same decisions, and then that they do, and that the refined meshes are equal.
dt stays below 0.8 of the finest mesh's own step limit (power iteration on the oracle's
operator).
"""

import math

import numpy as np
import pytest

import synth
from oracle import acga as oacga
from oracle.cga import cga
from oracle.discretization import Discretization
from oracle.solver import forward

pytestmark = pytest.mark.gpu


def _rel(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _params(desc, src, eobs, eps0, sig0, mesh=None):
    """CGA parameters as in the CGA tests: alpha^0 from the oracle's gradient at the initial
    guess (first step of at most 0.1 in eps, 0.02 in sigma, in the mass-weighted mean)."""
    prm = dict(gamma_eps=0.5, gamma_sig=0.5, p=0.5, alpha_eps=0.0, alpha_sig=0.0, eps_max=8.0, sig_max=2.0)
    d = Discretization(desc, mesh=mesh)
    g0 = cga(d, [src], eobs, eps0, sig0, prm, 1)[0]
    wt = float(np.sum(d.m_fem_lumped[d.fem_free]))
    prm.update(alpha_eps=0.1 / max(g0["eps"]["grad_norm"] / math.sqrt(wt), 1e-30),
               alpha_sig=0.02 / max(g0["sig"]["grad_norm"] / math.sqrt(wt), 1e-30))
    return prm


def _step_limit(d, iters=300, seed=0):
    """2 / sqrt(lambda_max(M_eps^-1 A)) by power iteration on the oracle's operator."""
    v = np.random.default_rng(seed).standard_normal((d.N, 3))
    lam = 0.0
    for _ in range(iters):
        u = d.apply_A(v) / d.M_eps[:, None]
        lam = float(np.linalg.norm(u) / np.linalg.norm(v))
        v = u / np.linalg.norm(u)
    return 2.0 / math.sqrt(lam)


def test_cga_on_a_refined_mesh_matches_oracle():
    import torch
    from paper_2508_07780_amd import CGA, CGAParams, Problem
    w = synth.small("ragged")
    marks = synth.meshref_marks(w.desc, w.eps, 0.6)
    mesh = synth.refined_mesh(w.desc, marks)
    eps_t = synth.refined_values(w.desc, marks, w.eps)
    sig_t = synth.refined_values(w.desc, marks, w.sigma)
    d = Discretization(w.desc, mesh=mesh).set_coefficients(eps_t, sig_t)
    assert w.desc.dt < 0.8 * _step_limit(d)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    n = d.n_fem
    eps0, sig0 = np.ones(n), np.zeros(n)
    prm = _params(w.desc, src, eobs, eps0, sig0, mesh)
    ref = cga(Discretization(w.desc, mesh=mesh), [src], eobs, eps0, sig0, prm, 3)
    print(f"[gpu] cga on a refined mesh: {int(marks.sum())} cells refined, {n} FEM nodes", flush=True)
    p = Problem(w.desc, mesh=mesh)
    c = CGA(p, [src], torch.tensor(eobs, dtype=torch.float32, device="cuda"), torch.tensor(eps0, device="cuda"),
            torch.tensor(sig0, device="cuda"), CGAParams(**prm))
    for m in range(3):
        c.iterate()
        info = c.info()
        for f, t, base in (("eps", c.eps, eps0), ("sig", c.sigma, sig0)):
            err = _rel(t.cpu().numpy().astype(np.float64) - base, ref[m][f]["coef"] - base)
            print(f"[gpu]   m={m} {f}: change rel L2 {err:.2e}, |g| {info['grad_norm'][f]:.4e} vs "
                  f"{ref[m][f]['grad_norm']:.4e}", flush=True)
            assert err <= 2e-3, (m, f, err)
            assert info["grad_norm"][f] == pytest.approx(ref[m][f]["grad_norm"], rel=1e-3)
            assert info["change_norm"][f] == pytest.approx(ref[m][f]["change_norm"], rel=2e-3)
    c.close()
    p.close()


@pytest.mark.parametrize("name,beta_eps,beta_sig", [("tiny", 0.0, 0.7), ("ragged", 0.5, 0.0)])
def test_acga_matches_oracle(name, beta_eps, beta_sig):
    """Two refinements (three CGA levels of two iterations): tiny with sigma-driven marks,
    ragged with eps-driven marks (every owned cell refined first, then 2 584 bisections).
    dt is 0.7 of the uniform mesh's default, below 0.8 of the finest mesh's own limit, with
    the step count raised to keep the simulated time."""
    import torch
    from paper_2508_07780_amd import CGAParams
    from paper_2508_07780_amd.acga import acga
    w = synth.small(name)
    w.desc.dt *= 0.7
    w.desc.n_steps = int(math.ceil(w.desc.n_steps / 0.7))
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    n = d.n_fem
    eps0, sig0 = np.ones(n), np.zeros(n)
    prm = _params(w.desc, src, eobs, eps0, sig0)
    ref = oacga.acga(w.desc, [src], eobs, eps0, sig0, prm, 2, beta_eps, beta_sig, n_refine=2)
    assert len(ref["levels"]) == 3
    for i, lv in enumerate(ref["levels"][:-1]):
        ext, tets = oacga._mesh(w.desc, lv["mesh"])
        hk = oacga.diameters(oacga.node_coords(w.desc, ext), tets)[:, None]
        for vals, beta in ((lv["eps"], beta_eps), (lv["sigma"], beta_sig)):
            if beta > 0:
                prod = hk * np.abs(vals)[tets]
                thr = beta * prod.max()
                margin = float(np.min(np.abs(prod - thr)) / thr)
                print(f"[gpu] acga {name} level {i}: beta {beta}, threshold margin {margin:.1e}, "
                      f"{int(lv['marks'].sum())} marked, {len(lv['refinement']['edges'])} bisected", flush=True)
                assert margin > 1e-3
    fin = ref["levels"][-1]["mesh"]
    assert w.desc.dt < 0.8 * _step_limit(Discretization(w.desc, mesh=fin).set_coefficients(ref["eps"], ref["sigma"]))
    out = acga(w.desc, [src], torch.tensor(eobs, dtype=torch.float32, device="cuda"), eps0, sig0, CGAParams(**prm),
               2, beta_eps, beta_sig, n_refine=2)
    assert len(out["levels"]) == 3
    for i in range(2):
        o, g = ref["levels"][i], out["levels"][i]
        assert np.array_equal(g["marks"], o["marks"])
        assert g["n_bisected"] == len(o["refinement"]["edges"])
    assert np.array_equal(out["mesh"][1], fin[1].astype(np.int32))
    assert np.abs(out["mesh"][0] - fin[0]).max() <= 1e-14 * max(1.0, float(np.abs(fin[0]).max()))
    for i, (o, g) in enumerate(zip(ref["levels"], out["levels"])):
        bar = 1e-3 if i == 0 else 4e-3
        assert len(g["history"]) == len(o["history"])
        for m in range(len(o["history"])):
            for f in ("eps", "sig"):
                g_ref = o["history"][m][f]["grad_norm"]
                print(f"[gpu]   level {i} m={m} {f}: |g| {g['history'][m]['grad_norm'][f]:.4e} vs {g_ref:.4e}",
                      flush=True)
                assert g["history"][m]["grad_norm"][f] == pytest.approx(g_ref, rel=bar)
        if i > 0:
            for f in ("eps", "sig"):
                print(f"[gpu]   level {i} {f}: change from its start {g['change'][f]:.4e} vs {o['change'][f]:.4e}",
                      flush=True)
                assert g["change"][f] == pytest.approx(o["change"][f], rel=bar)
            assert not g["stop"]
    base_e = np.ones(len(ref["eps"]))
    base_s = np.zeros(len(ref["sigma"]))
    e_err = _rel(out["eps"].cpu().numpy().astype(np.float64) - base_e, ref["eps"] - base_e)
    s_err = _rel(out["sigma"].cpu().numpy().astype(np.float64) - base_s, ref["sigma"] - base_s)
    print(f"[gpu]   final change from the initial guess, rel L2: eps {e_err:.2e} sigma {s_err:.2e}", flush=True)
    assert e_err <= 4e-3 and s_err <= 4e-3


def test_acga_stops_on_loose_tolerances():
    """Step 4 with tolerances every level meets: the loop ends after its first refinement, as
    the oracle's does."""
    import torch
    from paper_2508_07780_amd import CGAParams
    from paper_2508_07780_amd.acga import acga
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    n = d.n_fem
    prm = _params(w.desc, src, eobs, np.ones(n), np.zeros(n))
    th = dict(theta1_eps=1e9, theta1_sig=1e9, theta2_eps=1e9, theta2_sig=1e9)
    ref = oacga.acga(w.desc, [src], eobs, np.ones(n), np.zeros(n), prm, 1, 0.5, 0.0, n_refine=3, theta=th)
    out = acga(w.desc, [src], torch.tensor(eobs, dtype=torch.float32, device="cuda"), np.ones(n), np.zeros(n),
               CGAParams(**prm), 1, 0.5, 0.0, n_refine=3, theta=th)
    assert len(ref["levels"]) == len(out["levels"]) == 2
    assert out["levels"][1]["stop"] and ref["levels"][1]["stop"]
