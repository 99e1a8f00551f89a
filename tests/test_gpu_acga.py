"""Box "ACGA" on the GPU against the FP64 oracle: the CGA on a refined mesh (per-node lumped
masses in its inner products, the inserted centres free), and the adaptive loop itself (the
CGA on the uniform mesh, refinement by eq. meshref, interpolation, the CGA on the refined mesh).

Bars as for the CGA (tests/test_gpu_cga.py): the coefficient change rel L2 <= 2e-3 per
iteration and the gradient norms rel <= 1e-3 on one mesh.  On the refined level of the
adaptive loop the CGA starts from each side's own coarse result and is centred on it, so that
level carries the coarse level's error (<= 2e-3 of its change) on top of its own: the final
coefficients' change from the initial guess is held to 4e-3 and that level's gradient norms
to 4e-3.  The marks are an integer decision taken from the coarse results of the two sides:
the test checks that no node of a tested field lies within 1e-3 (relative) of its threshold,
well above the float32 solves' error in the coefficients, so that both sides must take the
same decisions, and then that they do.  dt stays below the refined meshes' own step limit
(power iteration on the oracle's operator).
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
    c.close()
    p.close()


@pytest.mark.parametrize("name,beta_eps,beta_sig", [("tiny", 0.5, 0.0), ("ragged", 0.0, 0.7)])
def test_acga_matches_oracle(name, beta_eps, beta_sig):
    import torch
    from paper_2508_07780_amd import CGAParams
    from paper_2508_07780_amd.acga import acga
    w = synth.small(name)
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"][None]
    n = d.n_fem
    eps0, sig0 = np.ones(n), np.zeros(n)
    prm = _params(w.desc, src, eobs, eps0, sig0)
    ref = oacga.acga(w.desc, [src], eobs, eps0, sig0, prm, 2, beta_eps, beta_sig)
    for vals, beta in ((ref["eps_coarse"], beta_eps), (ref["sig_coarse"], beta_sig)):
        if beta > 0:
            a = np.abs(vals)
            thr = beta * a.max()
            margin = float(np.min(np.abs(a - thr)) / thr)
            print(f"[gpu] acga {name}: beta {beta}, threshold margin {margin:.1e}", flush=True)
            assert margin > 1e-3
    ext, tets = ref["mesh"]
    assert w.desc.dt < 0.8 * _step_limit(Discretization(w.desc, mesh=ref["mesh"]).set_coefficients(
        ref["eps"], ref["sigma"]))
    print(f"[gpu] acga {name}: {int(ref['marks'].sum())} of {ref['marks'].size} cells refined, "
          f"{len(tets)} tets", flush=True)
    out = acga(w.desc, [src], torch.tensor(eobs, dtype=torch.float32, device="cuda"), eps0, sig0, CGAParams(**prm),
               2, beta_eps, beta_sig)
    assert np.array_equal(out["marks"].astype(bool), ref["marks"])
    for lvl, (hist, bar) in enumerate(((ref["coarse"], 1e-3), (ref["fine"], 4e-3))):
        got = out["history"][lvl]
        assert len(got) == len(hist)
        for m in range(len(hist)):
            for f in ("eps", "sig"):
                g_ref = hist[m][f]["grad_norm"]
                print(f"[gpu]   level {lvl} m={m} {f}: |g| {got[m]['grad_norm'][f]:.4e} vs {g_ref:.4e}", flush=True)
                assert got[m]["grad_norm"][f] == pytest.approx(g_ref, rel=bar)
    base_e = oacga.interpolate(w.desc, ref["marks"], eps0)
    base_s = oacga.interpolate(w.desc, ref["marks"], sig0)
    e_err = _rel(out["eps"].cpu().numpy().astype(np.float64) - base_e, ref["eps"] - base_e)
    s_err = _rel(out["sigma"].cpu().numpy().astype(np.float64) - base_s, ref["sigma"] - base_s)
    print(f"[gpu]   final change from the initial guess, rel L2: eps {e_err:.2e} sigma {s_err:.2e}", flush=True)
    assert e_err <= 4e-3 and s_err <= 4e-3
