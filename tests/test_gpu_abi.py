"""The C-ABI's allocator, footprint, Tikhonov term and batch budget on the GPU.

* Every device buffer of a problem goes through the allocator given to dd_create: with torch's
  caching allocator the results equal those of the library's own hipMalloc bit for bit, and
  dd_destroy hands every byte back.
* dd_footprint_bytes bounds what a problem really allocates through that allocator, with every
  optional buffer in use (initial data, the paper-formula gradient, the misfit, a CGA run), for
  the main workload with every level kept, the differentiation workload with K = 64 and a
  batched job; and it is not far above it (admission would waste little).
* dd_gradient's Tikhonov term against the oracle's definition (eq. tikhonov_functional with
  the lumped-mass quadrature): the nodal derivative gamma m_i (c_i - c0_i) on the free nodes.
* A batch's HBM budget refuses a job that does not fit and admits it once another completes.
"""

import math

import numpy as np
import pytest

import synth
from oracle.cga import gradient_function
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward

pytestmark = pytest.mark.gpu


def _problem(torch, w, allocator="torch", eps=None, sig=None):
    from paper_2508_07780_amd import Problem
    p = Problem(w.desc, allocator=allocator)
    p.set_coefficients(torch.tensor(w.eps if eps is None else eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma if sig is None else sig, dtype=torch.float32, device="cuda"))
    return p


def test_torch_allocator_equals_hipmalloc_bit_for_bit():
    import torch
    w = synth.small("ragged")
    out = []
    for alloc in ("torch", None):
        print(f"[gpu] allocator {alloc}", flush=True)
        p = _problem(torch, w, allocator=alloc)
        tr = p.forward(w.sources, save=True).clone()
        p.adjoint_misfit(tr, (0.5 * tr).contiguous())
        ge, gs = p.gradient()
        torch.cuda.synchronize()
        out.append((tr, ge.clone(), gs.clone(), p.device_bytes()))
        held = p.allocator.live if p.allocator else None
        p.close()
        if held is not None:
            assert not held and p.allocator.bytes == 0      # every buffer handed back
    (a, b) = out
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    assert a[3] > 0 and b[3] is None


def _all_modes_bytes(torch, w, n_src):
    """Bytes a problem holds through torch's allocator after a saving forward with n_src sources
    and with every optional buffer allocated."""
    from paper_2508_07780_amd.cga import CGA, CGAParams
    p = _problem(torch, w, eps=w.eps_true, sig=w.sigma_true)
    srcs = (w.sources * n_src)[:n_src]
    f = torch.zeros((p.n_grid, 3), dtype=torch.float32, device="cuda")
    p.set_initial_data(f, f)
    p.set_initial_data(None, None)
    p.paper_gradient(True)
    tr = p.forward(srcs, save=True)
    p.misfit(tr, tr, z=np.ones(p.n_steps))
    prm = CGAParams(gamma_eps=1.0, gamma_sig=1.0, p=0.5, alpha_eps=0.1, alpha_sig=0.1, eps_max=20.0, sig_max=3.0)
    cga = CGA(p, srcs, tr, torch.tensor(w.eps_true, device="cuda"), torch.tensor(w.sigma_true, device="cuda"), prm)
    torch.cuda.synchronize()
    held = p.device_bytes()
    cga.close()
    p.close()
    return held


@pytest.mark.parametrize("case", ["c2_store_all", "c3_k64", "small_two_sources"])
def test_footprint_bounds_the_allocations(case):
    import torch
    from paper_2508_07780_amd import Problem
    if case == "c2_store_all":
        w = synth.c2()
        w.desc.ckpt_every = w.desc.n_steps
        n_src = 1
    elif case == "c3_k64":
        w = synth.c3()
        n_src = 1
    else:
        w = synth.small("skinlet")
        n_src = 2
    print(f"[gpu] footprint {case}: outer {w.desc.n_outer} fem {w.desc.fem_cells} K {w.desc.ckpt_every}", flush=True)
    held = _all_modes_bytes(torch, w, n_src)
    fp = Problem.footprint_bytes(w.desc, n_src)
    print(f"[gpu]   held {held} footprint {fp} ratio {fp / held:.4f}", flush=True)
    assert held <= fp
    assert fp <= 1.05 * held + (8 << 20)


def test_footprint_bounds_a_batched_job():
    import torch
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.batch import Batch
    w = synth.small("skinlet")
    p = _problem(torch, w)
    srcs = w.sources * 2
    obs = torch.zeros((2, p.n_steps, p.n_det, 3), dtype=torch.float32, device="cuda")
    b = Batch(2)
    b.submit(p, srcs, obs=obs)
    held = p.device_bytes()
    b.run_to_completion(chunk=64)
    torch.cuda.synchronize()
    assert p.device_bytes() == held              # stepping allocates nothing
    assert held <= Problem.footprint_bytes(w.desc, 2)
    b.close()
    p.close()


def test_tikhonov_term_matches_the_oracle():
    import torch
    w = synth.small("skinlet")
    rng = np.random.default_rng(21)
    free = synth.fem_layers(w.desc) >= 2
    eps0 = np.where(free, 1.0 + 2.0 * rng.random(free.shape), 1.0)
    sig0 = np.where(free, 0.5 * rng.random(free.shape), 0.0)
    ge_, gs_ = 0.37, 1.9
    e32, s32 = (np.asarray(x, dtype=np.float32).astype(np.float64) for x in (w.eps, w.sigma))
    e032, s032 = (np.asarray(x, dtype=np.float32).astype(np.float64) for x in (eps0, sig0))
    d = Discretization(w.desc).set_coefficients(e32, s32)
    fw = forward(d, w.sources[0])
    cot = (0.4 * fw["traces"]).astype(np.float32)
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    wts = d.m[d.fem_grid]
    # nodal derivative of J + Tikhonov = lumped mass x the oracle's gradient function
    ref_e = wts * gradient_function(ag["g_eps"], wts, e32, e032, ge_, d.fem_free)
    ref_s = wts * gradient_function(ag["g_sigma"], wts, s32, s032, gs_, d.fem_free)
    p = _problem(torch, w)
    p.forward(w.sources, save=True)
    p.adjoint(torch.tensor(cot[None], device="cuda"))
    g0e, g0s = (g.cpu().numpy() for g in p.gradient())
    e0t = torch.tensor(eps0, dtype=torch.float32, device="cuda")
    s0t = torch.tensor(sig0, dtype=torch.float32, device="cuda")
    gre, grs = (g.cpu().numpy() for g in p.gradient(reg=(ge_, gs_, e0t, s0t)))
    torch.cuda.synchronize()
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))  # noqa: E731
    print(f"[gpu] Tikhonov gradient rel L2 eps {rel(gre, ref_e):.2e} sigma {rel(grs, ref_s):.2e}", flush=True)
    assert rel(gre, ref_e) <= 1e-3 and rel(grs, ref_s) <= 1e-3
    # the term itself, exactly: gamma m (c - c0) on the free nodes, 0 elsewhere
    te = np.where(d.fem_free, ge_ * wts * (e32 - e032), 0.0)
    ts = np.where(d.fem_free, gs_ * wts * (s32 - s032), 0.0)
    assert np.abs((gre - g0e) - te).max() <= 1e-12 * np.abs(te).max()
    assert np.abs((grs - g0s) - ts).max() <= 1e-12 * np.abs(ts).max()
    from paper_2508_07780_amd import DDError
    with pytest.raises(DDError) as e:
        p.gradient(reg=(-1.0, 0.0, e0t, s0t))
    assert e.value.code == -1
    p.close()


def test_batch_budget_refuses_and_later_admits():
    import torch
    from paper_2508_07780_amd import DDError, Problem
    from paper_2508_07780_amd.batch import Batch
    w = synth.small("tiny")
    fp = Problem.footprint_bytes(w.desc, 1)
    probs = [_problem(torch, w) for _ in range(2)]
    obs = torch.zeros((1, w.desc.n_steps, probs[0].n_det, 3), dtype=torch.float32, device="cuda")
    b = Batch(4, hbm_budget=fp + fp // 2)        # room for one job
    b.submit(probs[0], w.sources, obs=obs)
    with pytest.raises(DDError) as e:
        b.submit(probs[1], w.sources, obs=obs)
    assert e.value.code == -6
    done = b.run_to_completion(chunk=64)
    assert len(done) == 1
    b.submit(probs[1], w.sources, obs=obs)       # the first job's bytes came back
    assert len(b.run_to_completion(chunk=64)) == 1
    b.close()
    for p in probs:
        p.close()


def test_store_all_mode_equals_k_equal_n_steps():
    """DD_CKPT_STORE_ALL is the checkpoint interval K = n_steps: the same gradient bit for bit."""
    import torch
    from paper_2508_07780_amd import _lib
    w = synth.small("tiny")
    cot = None
    out = []
    for mode, K in ((_lib.CKPT_STORE_ALL, 3), (_lib.CKPT_FEM_IFACE, w.desc.n_steps)):
        w.desc.ckpt_mode = mode
        w.desc.ckpt_every = K
        p = _problem(torch, w)
        tr = p.forward(w.sources, save=True).clone()
        if cot is None:
            cot = (0.3 * tr).contiguous()
        p.adjoint(cot)
        out.append([g.clone() for g in p.gradient()])
        p.close()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert math.isfinite(float(out[0][0].abs().max()))
