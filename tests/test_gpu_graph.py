"""Forward and adjoint launches replayed as HIP graphs (dd_set_graph) against launch by launch.

A graph holds the same kernels with the same arguments as the launch-by-launch call, so the
bar is bit-for-bit: traces, energy, and gradients (an adjoint graph reads the saved forward a
forward graph wrote).  Each graph is replayed several times, with other work queued and the
device synchronised between replays; a change of the call's sources, buffers or save flag, of
the div-div form or of the initial data captures anew.  The adjoint runs with one, two and
several checkpoint segments; only an adjoint of one segment is captured (with several, its
recompute stream's branch made the graph's launch hold the host), the others run launch by
launch and must give the same gradients.  One case is also held to the FP64 oracle at the bar
of every parity test (traces 1e-4).  The automatic mode replays only on a repeated call on a
small grid, and never while kernel timing is on.
"""

import dataclasses

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle.solver import forward

pytestmark = pytest.mark.gpu


def _problem(torch, w, mode, desc=None):
    from paper_2508_07780_amd import Problem
    p = Problem(desc or w.desc)
    p.set_graph(mode)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    return p


def _dipole(w, pos):
    s = w.sources[0]
    return synth.Source(kind=synth.SRC_DIPOLE, omega=s.omega, t0=s.t0, width=s.width, pol=(0.2, 1.0, -0.4),
                        pos=pos)


def _grad(torch, p, traces, obs):
    p.adjoint_misfit(traces, obs)
    return [g.clone() for g in p.gradient()]


@pytest.mark.parametrize("name,segments", [("tiny", "many"), ("ragged", "many"), ("tiny", "one"), ("tiny", "two")])
def test_graph_replays_equal_launch_by_launch(name, segments):
    import torch
    w = synth.small(name)
    nt = w.desc.n_steps
    if segments != "many":
        ck = nt if segments == "one" else (nt + 1) // 2
        w = dataclasses.replace(w, desc=dataclasses.replace(w.desc, ckpt_every=ck))
    pe, pg = _problem(torch, w, "off"), _problem(torch, w, "on")
    dip = _dipole(w, (1, 1, 1))
    ref = pe.forward(w.sources, save=True).clone()
    obs = torch.tensor(1e-3 * synth.noise(tuple(ref.shape), 5), dtype=torch.float32, device="cuda")
    g_ref = _grad(torch, pe, ref, obs)
    buf = torch.full_like(ref, float("nan"))
    for r in range(4):
        pe.forward([dip], save=False)            # other work between the replays
        torch.cuda.synchronize()
        buf.fill_(float("nan"))
        pg.forward(w.sources, save=True, out=buf)
        torch.cuda.synchronize()
        assert torch.equal(buf, ref), f"replay {r}"
    assert pg.graph_stats() == (1, 4)
    for r in range(3):
        g = _grad(torch, pg, buf, obs)
        for a, b in zip(g, g_ref):
            assert torch.equal(a, b), f"adjoint replay {r}"
        pe.forward([dip], save=False)
        torch.cuda.synchronize()
    one = segments == "one"
    assert pg.graph_stats("adjoint") == ((1, 3) if one else (0, 0))

    # a new source, the save flag, energy: captured anew, still bitwise
    te = pe.forward([dip], save=True).clone()
    pg.forward([dip], save=True, out=buf)
    assert torch.equal(buf, te)
    te = pe.forward(w.sources, save=False).clone()
    pg.forward(w.sources, save=False, out=buf)
    assert torch.equal(buf, te)
    te, ee = pe.forward(w.sources, save=True, energy=True)
    tg, eg = pg.forward(w.sources, save=True, energy=True)
    assert torch.equal(tg, te) and torch.equal(eg, ee)
    assert pg.graph_stats() == (4, 7)

    # the R2 div-div form, then initial data: the options change the launches
    for p in (pe, pg):
        p.set_divdiv_form("R2")
    te = pe.forward(w.sources, save=True).clone()
    for _ in range(2):
        pg.forward(w.sources, save=True, out=buf)
        assert torch.equal(buf, te)
    g_ref, g = _grad(torch, pe, te, obs), _grad(torch, pg, buf, obs)
    for a, b in zip(g, g_ref):
        assert torch.equal(a, b)
    f0, f1 = synth.initial_pulses(w.desc, 17)
    for p in (pe, pg):
        p.set_divdiv_form("R1")
        p.set_initial_data(torch.tensor(f0, dtype=torch.float32, device="cuda"),
                           torch.tensor(f1, dtype=torch.float32, device="cuda"))
    te = pe.forward(w.sources, save=True).clone()
    pg.forward(w.sources, save=True, out=buf)
    assert torch.equal(buf, te)
    g_ref, g = _grad(torch, pe, te, obs), _grad(torch, pg, buf, obs)
    for a, b in zip(g, g_ref):
        assert torch.equal(a, b)
    assert pg.graph_stats() == (6, 10)
    assert pg.graph_stats("adjoint") == ((3, 5) if one else (0, 0))
    pe.close()
    pg.close()


def test_graph_forward_matches_oracle():
    import torch
    w = synth.small("tiny")
    p = _problem(torch, w, "on")
    buf = p.forward(w.sources, save=False)
    p.forward(w.sources, save=False, out=buf)
    got = buf[0].cpu().numpy()
    assert p.graph_stats() == (1, 2)
    p.close()
    e32 = np.asarray(w.eps, dtype=np.float32).astype(np.float64)
    s32 = np.asarray(w.sigma, dtype=np.float32).astype(np.float64)
    want = forward(Discretization(w.desc).set_coefficients(e32, s32), w.sources[0])["traces"]
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= 1e-4, err


def test_auto_mode_replays_repeated_calls_on_small_grids():
    import torch
    w = synth.small("tiny")
    w = dataclasses.replace(w, desc=dataclasses.replace(w.desc, ckpt_every=w.desc.n_steps))   # one segment
    pe, pa = _problem(torch, w, "off"), _problem(torch, w, "auto")
    dip = _dipole(w, (1, 1, 1))
    ref = pe.forward(w.sources, save=True).clone()
    ref_d = pe.forward([dip], save=True).clone()
    buf = torch.empty_like(ref)
    expect = [(0, 0), (1, 1), (1, 2)]
    for want in expect:
        pa.forward(w.sources, save=True, out=buf)
        assert torch.equal(buf, ref)
        assert pa.graph_stats() == want
    pa.forward([dip], save=True, out=buf)          # a new call: launch by launch
    assert torch.equal(buf, ref_d) and pa.graph_stats() == (1, 2)
    pa.forward([dip], save=True, out=buf)          # its repeat: captured
    assert torch.equal(buf, ref_d) and pa.graph_stats() == (2, 3)
    pa.forward(w.sources, save=True, out=buf)      # back to the first call: launch by launch
    assert torch.equal(buf, ref) and pa.graph_stats() == (2, 3)
    obs = torch.tensor(1e-3 * synth.noise(tuple(ref.shape), 5), dtype=torch.float32, device="cuda")
    pe.forward(w.sources, save=True)
    g_ref = _grad(torch, pe, ref, obs)
    for want in [(0, 0), (1, 1), (1, 2)]:
        for a, b in zip(_grad(torch, pa, buf, obs), g_ref):
            assert torch.equal(a, b)
        assert pa.graph_stats("adjoint") == want
    # kernel timing on: launch by launch
    pa.profile(1)
    for _ in range(2):
        pa.forward(w.sources, save=True, out=buf)
        assert torch.equal(buf, ref)
    assert pa.graph_stats() == (2, 3)
    pe.close()
    pa.close()

    # a grid of more than 2^19 nodes: launch by launch in the automatic mode
    d = dataclasses.replace(w.desc, n_outer=(84, 82, 80), fem_lo=(40, 38, 37), n_steps=12)
    big = dataclasses.replace(w, desc=d)
    pe, pa = _problem(torch, big, "off", d), _problem(torch, big, "auto", d)
    ref = pe.forward(big.sources, save=False).clone()
    buf = torch.empty_like(ref)
    for _ in range(3):
        pa.forward(big.sources, save=False, out=buf)
        assert torch.equal(buf, ref)
    assert pa.graph_stats() == (0, 0)
    pe.close()
    pa.close()
