"""dd_misfit_noalloc (the misfit with its scratch in a static device array) against dd_misfit.

Both run the same kernels, so the cotangent and J are compared bit for bit, on two calls in a
row (the second with a smaller input: fewer sources and no weights, then a problem with fewer
steps and other weights), through the C-ABI.  Sizes beyond the array's maximum are rejected
before any device work.
"""

import ctypes
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _problem(torch, w):
    from paper_2508_07780_amd import Problem
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    return p


def _both(torch, p, traces, obs, z):
    """(cot, J) from dd_misfit and from dd_misfit_noalloc on the same inputs."""
    out = []
    for no_alloc in (False, True):
        cot = torch.full_like(traces, float("nan"))
        J, _ = p.misfit(traces, obs, z=z, out=cot, no_alloc=no_alloc)
        torch.cuda.synchronize()
        out.append((cot.clone(), J.clone()))
    return out


def test_noalloc_misfit_equals_misfit_on_consecutive_calls():
    import torch
    w = synth.small("ragged")
    srcs = [w.sources[0], synth.gauss_sine(2 * math.pi / (10 * w.desc.h), pol=(1.0, 0.0, 0.3))]
    p = _problem(torch, w)
    print(f"[gpu] no-alloc misfit: ragged, {len(srcs)} sources, {w.desc.n_steps} steps", flush=True)
    tr = p.forward(srcs, save=False).clone()
    obs = (0.8 * tr + 1e-3).contiguous()
    z = synth.noise(w.desc.n_steps, 3) ** 2           # any non-negative weights
    (c0, j0), (c1, j1) = _both(torch, p, tr, obs, z)
    assert torch.equal(c0, c1) and torch.equal(j0, j1)
    assert float(j0) > 0
    # second call: a smaller input (one source, z = 1) on the same problem
    print("[gpu] no-alloc misfit: second call, one source, no weights", flush=True)
    tr1 = tr[:1].contiguous()
    ob1 = obs[:1].contiguous()
    (c0, j0), (c1, j1) = _both(torch, p, tr1, ob1, None)
    assert torch.equal(c0, c1) and torch.equal(j0, j1)
    ref = 0.5 * float(((tr1.double() - ob1.double()) ** 2).sum())
    assert abs(float(j1) - ref) <= 1e-12 * ref
    # a problem with fewer steps and fewer detectors, weights again
    w2 = synth.small("tiny")
    p2 = _problem(torch, w2)
    print(f"[gpu] no-alloc misfit: tiny, {w2.desc.n_steps} steps", flush=True)
    tr2 = p2.forward(w2.sources, save=False).clone()
    ob2 = torch.zeros_like(tr2)
    z2 = np.linspace(1.0, 0.0, w2.desc.n_steps)
    (c0, j0), (c1, j1) = _both(torch, p2, tr2, ob2, z2)
    assert torch.equal(c0, c1) and torch.equal(j0, j1)
    p.close()
    p2.close()


def test_noalloc_misfit_rejects_more_steps_than_its_scratch_holds():
    import torch
    from paper_2508_07780_amd import _lib
    from paper_2508_07780_amd.solver import _ptr, _stream
    lib = _lib.load()
    w = synth.small("tiny")
    w.desc.n_steps = 65537                 # one more than DD_MISFIT_NOALLOC_MAX_STEPS
    w.desc.ckpt_every = 64
    p = _problem(torch, w)
    buf = torch.zeros(16, dtype=torch.float32, device="cuda")
    j = torch.zeros((), dtype=torch.float64, device="cuda")
    rc = lib.dd_misfit_noalloc(p._h, _ptr(buf), _ptr(buf), 1, None, None, _ptr(j), _stream())
    assert rc == -1
    assert b"maximum" in lib.dd_last_error(p._h)
    p.close()
