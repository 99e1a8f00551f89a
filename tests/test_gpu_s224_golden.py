"""Streaming-regime parity: the 224^3 outer grid with a 96^3-hex FEM box (layered skin, one
point dipole above the box, 420 steps, K = 64), whose two levels of E (270 MB) exceed the
256 MB last-level cache, so the finite-difference tiles run their streaming variant by default
(8-plane z-chunks, non-temporal own-node accesses; nz = 224 is a multiple of 8, so the top face
closes a full chunk and the adjoint's cotangent is loaded ahead there), against the FP64 oracle.

The oracle run takes about an hour on one host core, so its result is stored:
tests/golden/make_s224_golden.py (which calls only the oracle and the seeded input generators)
wrote a seeded sample of 8192 trace entries and 8192 free-node gradient entries, the per-step
trace norms, the gradient norms and the energy history, for the misfit of seeded synthetic
observations that this test regenerates from the same generator (the GPU forms traces - obs
inside its adjoint tiles).

Bars: traces rel L2 <= 1e-4 (sampled entries and per-step norms), gradient rel L2 <= 1e-3
(sampled entries and norms), energy rel L2 <= 1e-4.
"""

import importlib.util
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "s224_oracle_sample_420.npz")
LLC_BYTES = 256 * 1024 * 1024


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def s224_run():
    import torch
    from paper_2508_07780_amd import Problem
    spec = importlib.util.spec_from_file_location("make_s224_golden", os.path.join(HERE, "golden", "make_s224_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    ref = np.load(GOLDEN)
    w = synth.stream224(n_steps=int(ref["n_steps"]))
    assert 24 * w.desc.n_grid() > LLC_BYTES          # the streaming variant is the default here
    print(f"[gpu] s224 golden: {w.desc.n_outer} fem {w.desc.fem_cells} steps {w.desc.n_steps} "
          f"K {w.desc.ckpt_every}", flush=True)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma_true, dtype=torch.float32, device="cuda"))
    tr = p.forward(w.sources, save=True).clone()
    obs = mk.observations(tuple(tr.shape[1:]), w.seed, float(ref["obs_scale"]))
    p.adjoint_misfit(tr, torch.tensor(obs[None], device="cuda"))
    ge, gs = (g.cpu().numpy() for g in p.gradient())
    _, en = p.forward(w.sources, save=False, energy=True)
    torch.cuda.synchronize()
    out = dict(traces=tr[0].cpu().numpy(), g_eps=ge, g_sigma=gs, energy=en[0].cpu().numpy())
    p.close()
    return ref, out


def test_s224_traces_match_oracle(s224_run):
    ref, out = s224_run
    tr = out["traces"]
    e_sample = _rel(tr[ref["t_idx"], ref["d_idx"], :], ref["traces"])
    e_norm = _rel(np.sqrt(np.sum(tr.astype(np.float64) ** 2, axis=(1, 2))), ref["trace_row_norm"])
    print(f"[gpu] s224 traces: sampled rel L2 {e_sample:.3e}, per-step norms rel L2 {e_norm:.3e}", flush=True)
    assert e_sample <= 1e-4 and e_norm <= 1e-4


def test_s224_gradient_matches_oracle(s224_run):
    ref, out = s224_run
    gi = ref["g_idx"]
    e_eps = _rel(out["g_eps"][gi], ref["g_eps"])
    e_sig = _rel(out["g_sigma"][gi], ref["g_sigma"])
    n_eps = abs(np.linalg.norm(out["g_eps"]) / float(ref["g_eps_norm"]) - 1.0)
    n_sig = abs(np.linalg.norm(out["g_sigma"]) / float(ref["g_sigma_norm"]) - 1.0)
    print(f"[gpu] s224 gradient: sampled rel L2 eps {e_eps:.3e} sigma {e_sig:.3e}; "
          f"norm ratio - 1: eps {n_eps:.2e} sigma {n_sig:.2e}", flush=True)
    assert e_eps <= 1e-3 and e_sig <= 1e-3
    assert n_eps <= 1e-3 and n_sig <= 1e-3


def test_s224_energy_matches_oracle(s224_run):
    ref, out = s224_run
    e = _rel(out["energy"], ref["energy"])
    print(f"[gpu] s224 energy rel L2 {e:.3e}", flush=True)
    assert e <= 1e-4
