#!/usr/bin/env python3
"""Benchmark: one step = one full forward + adjoint + gradient solve on the GPU.

Workload (default): layered-skin model, 160^3 outer grid nodes, 64^3 FEM hexes
(1.57M Kuhn tetrahedra), 2000 time steps, one Gaussian-sine plane wave on the
top face, detectors on the top face, every forward FEM level kept for the adjoint
(no recompute; --ckpt-every K checkpoints every K steps instead).  Observed data
come from the seeded true model plus 3% Gaussian noise; the gradient is taken at
the initial guess eps = 1, sigma = 0.  Inputs are resident in HBM before timing.

Prints one JSON line with the throughput in Gcell-steps/s, where a cell is an
outer-grid node or a FEM-owned node and forward and adjoint steps both count,
the roofline of the dominant kernel (the fused FD + FEM forward step, HIP-event timed
over the timed region on the solver's stream), per-solve latency p50/p99, the same
kernels on a 288^3 probe whose fields exceed the last-level cache, the 192^3
autograd workload with checkpointed recompute, the batched and serving comparisons, and
the FP64 oracle timed on the host on a bounded sample of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_c2_traffic.md")
PROBE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_probe288.md")
LLC_BYTES = 256 * 1024 * 1024   # MI355X last-level (Infinity) cache


def measured_traffic(key, path=TRAFFIC_FILE):
    """HBM bytes per launch recorded from PMC counters, if they were taken on these kernel sources."""
    from paper_2508_07780_amd.profiling import kernel_source_hash
    try:
        txt = open(path).read()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in txt.splitlines() if ":" in line and not line.startswith(("#", " ", "|")))
    vals = {k.strip(): v.strip() for k, v in vals.items()}
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = vals.get(key)
    return float(v) if v else None


# Algorithmic bytes per unit and step of the fused step launches, the roofline's units: an FD
# node 36 B (three-level form: E^n, E^{n-1} read, E^{n+1} written), a FEM-owned node 120 B
# forward (state 48, coordinates 12, coefficients 12, six tetrahedra of 8 B connectivity) and
# 176 B adjoint (+24 B forward window, +32 B FP64 gradient accumulators), a detector 12 B.
# The stencil path reads no coordinates or connectivity; its own minimum is reported beside.
UNIT_BYTES = {"fd": 36.0, "fem_fwd": 120.0, "fem_adj": 176.0, "det": 12.0}


def unit_bytes(desc, n_det, adjoint):
    n_own = desc.n_fem_owned()
    n_fd = desc.n_grid() - n_own
    return (UNIT_BYTES["fd"] * n_fd + UNIT_BYTES["fem_adj" if adjoint else "fem_fwd"] * n_own +
            UNIT_BYTES["det"] * n_det)


def progress(msg):
    """One line on stderr as each part of the run completes (the JSON result goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    f, c = math.floor(k), math.ceil(k)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def cpu_baseline(workload, n_steps):
    """The FP64 oracle, as it stands, on the first n_steps forward + n_steps adjoint steps."""
    import numpy as np
    from oracle.discretization import Discretization
    from oracle.solver import adjoint_gradient, forward
    import synth
    w = synth.with_steps(workload, n_steps)
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    cot = np.random.default_rng(0).standard_normal((n_steps, len(d.det), 3)) * 1e-3
    t0, c0 = time.perf_counter(), time.process_time()
    fw = forward(d, w.sources[0])
    adjoint_gradient(d, cot, fw)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    cells = w.desc.n_grid() + w.desc.n_fem_owned()
    return {
        "value": cells * 2 * n_steps / wall / 1e9,
        "unit": "Gcell-steps/s",
        "cores": max(1, int(math.ceil(cpu / wall - 0.05))),
        "kind": "oracle",
        "sample": f"FP64 numpy/scipy oracle, full {w.desc.n_outer[0]}^3 grid with {w.desc.fem_cells[0]}^3 FEM "
                  f"hexes, first {n_steps} forward + {n_steps} adjoint steps with gradient accumulation "
                  f"({wall:.1f} s wall, {cpu:.1f} s CPU; host has {len(os.sched_getaffinity(0))} cores available)",
    }


def batch_comparison():
    """16 uneven problems (outer 96-224^3, FEM 32-96^3 hexes, 1000-2500 steps, plane-wave or
    dipole source each), forward + adjoint + gradient: one batch (one launch per step for all
    of them) vs one problem after the other through the single-problem calls."""
    import torch
    import synth
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.batch import Batch
    from paper_2508_07780_amd.serving import cell_steps
    mix = synth.batch_mix(16)
    dev = torch.device("cuda", 0)
    probs, obs = [], []
    for w in mix:
        p = Problem(w.desc)
        p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device=dev),
                           torch.tensor(w.sigma, dtype=torch.float32, device=dev))
        g = torch.Generator(device=dev)
        g.manual_seed(w.seed)
        obs.append(1e-3 * torch.randn((1, w.desc.n_steps, p.n_det, 3), generator=g, device=dev))
        probs.append(p)
    work = sum(cell_steps(w.desc, 1) for w in mix)
    torch.cuda.synchronize()
    grads = [(torch.empty(p.n_fem, dtype=torch.float64, device=dev), torch.empty(p.n_fem, dtype=torch.float64, device=dev))
             for p in probs]
    t0 = time.perf_counter()
    for p, w, o, g in zip(probs, mix, obs, grads):
        tr = p.forward(w.sources, save=True)
        p.adjoint_misfit(tr, o)
        p.gradient(out=g)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    b = Batch(16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = [b.submit(p, w.sources, obs=o) for p, w, o in zip(probs, mix, obs)]
    recs = {r["id"]: r for r in b.run_to_completion()}
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    # the batched gradients against the single-problem calls' (the same device code: bit for bit)
    same = all(torch.equal(recs[i]["g_eps"], g[0]) and torch.equal(recs[i]["g_sigma"], g[1]) for i, g in zip(ids, grads))
    b.close()
    for p in probs:
        p.close()
    return {"workload": "16 problems: outer " + ",".join(str(w.desc.n_outer[0]) for w in mix) + "; FEM "
                        + ",".join(str(w.desc.fem_cells[0]) for w in mix) + "; steps "
                        + ",".join(str(w.desc.n_steps) for w in mix) + "; K = 64",
            "batched_gcell_steps_s": round(work / t_batch / 1e9, 3), "batched_s": round(t_batch, 3),
            "one_at_a_time_gcell_steps_s": round(work / t_serial / 1e9, 3), "one_at_a_time_s": round(t_serial, 3),
            "ratio": round(t_serial / t_batch, 3), "gradients_equal_one_at_a_time": bool(same),
            "sources": "even problems: Gaussian-sine plane waves of seeded incidence (0-30 degrees), odd: point dipoles"}


def refined_mesh_measure(w, stride=16):
    """The main workload's solve (forward with saving, adjoint, gradient) on a locally refined
    FEM mesh of box "ACGA": the elements where the true eps is largest (beta_eps 0.6) refined
    once by longest-edge bisection (the library's refinement), eps and sigma interpolated.  The
    FEM rows then run on the element-coloured kernel, fused with the FD tiles in one launch per
    step (forward and adjoint).  dt is 0.7 of the uniform mesh's (the refined elements lower the
    step limit);
    the per-step cost does not depend on it.  For comparison the uniform mesh through the same
    element-coloured path."""
    import numpy as np
    import torch
    from paper_2508_07780_amd import Problem, _lib
    from paper_2508_07780_amd.acga import Refinement
    from dataclasses import replace
    dev = torch.device("cuda", 0)
    desc = replace(w.desc, dt=0.7 * w.desc.dt)
    ref = Refinement(desc, None, w.eps_true, w.sigma_true, 0.6, 0.0)
    eps = torch.tensor(ref.interpolate(w.eps_true), device=dev)
    sig = torch.tensor(ref.interpolate(w.sigma_true), device=dev)
    out = {"workload": f"layered skin, outer {desc.n_outer[0]}^3, FEM {desc.fem_cells[0]}^3 hexes, "
                       f"{desc.n_steps} steps; {ref.n_marked} elements marked, {ref.n_bisected} bisected, "
                       f"{len(ref.mesh[1])} tetrahedra (uniform: {6 * int(np.prod(desc.fem_cells))})"}
    prev = os.environ.get("DD_FEM_PATH")
    os.environ["DD_FEM_PATH"] = "element"
    try:
        for name, mesh, e, sg in (("refined", ref.mesh, eps, sig),
                                  ("uniform_element_path", None,
                                   torch.tensor(w.eps_true, dtype=torch.float32, device=dev),
                                   torch.tensor(w.sigma_true, dtype=torch.float32, device=dev))):
            p = Problem(desc, mesh=mesh)
            p.set_coefficients(e, sg)
            tr = p.forward(w.sources, save=True)
            cot = (1e-3 * tr).contiguous()
            p.adjoint(cot)
            p.gradient()
            torch.cuda.synchronize()
            p.profile(stride)
            for k in range(len(_lib.PROF_NAMES)):
                p.profile_read(k, reset=True)
            t0 = time.perf_counter()
            tr = p.forward(w.sources, save=True)
            p.adjoint(cot)
            ge, gs = p.gradient()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            cells = (desc.n_grid() + desc.n_fem_owned()) * 2 * desc.n_steps * len(w.sources)
            r = {"solve_ms": round(wall * 1e3, 2), "gcell_steps_s": round(cells / wall / 1e9, 3),
                 "gradient_finite": bool(torch.isfinite(ge).all() and torch.isfinite(gs).all())}
            for kind in ("step_fwd", "step_adj", "fd_step_fwd", "fem_step_fwd", "fd_step_adj", "fem_step_adj"):
                ms, n = p.profile_read(_lib.PROF_NAMES.index(kind), reset=True)
                if n:
                    r[kind + "_us"] = round(ms / n * 1e3, 2)
            out[name] = r
            p.close()
    finally:
        if prev is None:
            os.environ.pop("DD_FEM_PATH", None)
        else:
            os.environ["DD_FEM_PATH"] = prev
    ref.close()
    return out


def small_graphs_measure(reps=20):
    """The plain forward config (25^3 outer nodes, 8^3 FEM hexes, 300 steps), whose steps are
    bound by launch latency: per-step times of the forward (with saving) and of the misfit
    adjoint, and the whole solve (forward, adjoint, gradient), launch by launch and replayed
    as HIP graphs, with the configured checkpoint interval (K = 64) and with one segment."""
    import torch
    import synth
    from dataclasses import replace
    from paper_2508_07780_amd import Problem
    w = synth.c1()
    nt = w.desc.n_steps
    out = {"workload": "plain forward config: outer 25^3, FEM 8^3 hexes, 300 steps, one source"}

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    for label, desc in (("k64", w.desc), ("one_segment", replace(w.desc, ckpt_every=nt))):
        res, grads = {}, {}
        for mode in ("off", "on"):
            p = Problem(desc)
            p.set_graph(mode)
            p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                               torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
            tr = p.forward(w.sources, save=True)
            obs = torch.full_like(tr, 1e-3)
            ge = torch.empty(p.n_fem, dtype=torch.float64, device="cuda")
            gs = torch.empty_like(ge)

            def fwd():
                p.forward(w.sources, save=True, out=tr)

            def adj():
                p.adjoint_misfit(tr, obs)

            def solve():
                fwd()
                adj()
                p.gradient(out=(ge, gs))

            tf, ta, ts = timed(fwd), timed(adj), timed(solve)
            r = {"forward_us_per_step": round(tf / nt * 1e6, 2), "adjoint_us_per_step": round(ta / nt * 1e6, 2),
                 "solve_ms": round(ts * 1e3, 3)}
            if mode == "on":
                r["graphs_captured_replayed"] = {"forward": p.graph_stats("forward"),
                                                 "adjoint": p.graph_stats("adjoint")}
            res["launch_by_launch" if mode == "off" else "graphs"] = r
            grads[mode] = ge.clone()
            p.close()
        res["gradient_bitwise_equal"] = bool(torch.equal(grads["off"], grads["on"]))
        out[label] = res
    return out


def acga_measure(w, n_iter=2, n_refine=2, beta_eps=0.9):
    """Box "ACGA" on the main workload from eps = 1, sigma = 0: n_iter CGA iterations per mesh,
    n_refine refinements (longest-edge bisection where h_K |eps| >= beta_eps of its largest
    value, in the library's host code) with the interpolated reconstruction as the next start;
    dt 0.7 of the uniform mesh's (the refined meshes' step limit is lower).  The step sizes come
    from the gradient at the initial guess (setup, not timed)."""
    import numpy as np
    import torch
    from dataclasses import replace
    from paper_2508_07780_amd import CGAParams, Problem
    from paper_2508_07780_amd.acga import acga
    dev = torch.device("cuda", 0)
    desc = replace(w.desc, dt=0.7 * w.desc.dt)
    p = Problem(desc)
    p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device=dev),
                       torch.tensor(w.sigma_true, dtype=torch.float32, device=dev))
    obs = p.forward(w.sources, save=False).clone()
    n = p.n_fem
    eps0 = torch.ones(n, dtype=torch.float32, device=dev)
    sig0 = torch.zeros(n, dtype=torch.float32, device=dev)
    p.set_coefficients(eps0, sig0)
    p.adjoint_misfit(p.forward(w.sources, save=True), obs)
    ge, gs = p.gradient()
    prm = CGAParams.from_gradient(ge, gs, desc.h, eps_max=20.0, sig_max=3.0)
    p.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = acga(desc, w.sources, obs, eps0, sig0, prm, n_iter, beta_eps, 0.0, n_refine=n_refine)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lv = out["levels"]
    return {"workload": f"layered skin, outer {desc.n_outer[0]}^3, FEM {desc.fem_cells[0]}^3 hexes, "
                        f"{desc.n_steps} steps; {n_iter} CGA iterations per mesh, {n_refine} refinements "
                        f"(beta_eps {beta_eps})",
            "wall_s": round(wall, 2), "meshes": len(lv),
            "bisections": [l.get("n_bisected") for l in lv[:-1]],
            "final_extra_nodes": len(out["mesh"][0]) if out["mesh"] is not None else 0,
            "final_tets": len(out["mesh"][1]) if out["mesh"] is not None else 6 * int(np.prod(desc.fem_cells)),
            "grad_norm_eps": [[round(h["grad_norm"]["eps"], 1) for h in l["history"]] for l in lv],
            "finite": bool(torch.isfinite(out["eps"]).all() and torch.isfinite(out["sigma"]).all())}


def large_probe(n_steps=300, stride=16):
    """The fused step kernels on a 288^3 outer grid (96^3 FEM hexes, layered skin), whose
    per-step field set (860 MB) exceeds the 256 MB last-level cache, so that the achieved
    bandwidth is HBM's and not the cache's: one forward (every level kept) + adjoint +
    gradient, kernels timed with HIP events on the solver's stream."""
    import torch
    import synth
    from paper_2508_07780_amd import Problem, _lib
    w = synth.probe288(n_steps)
    dev = torch.device("cuda", 0)
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device=dev),
                       torch.tensor(w.sigma_true, dtype=torch.float32, device=dev))
    tr = p.forward(w.sources, save=True)             # warm-up
    cot = (1e-3 * tr).contiguous()
    p.adjoint(cot)
    p.gradient()
    torch.cuda.synchronize()
    p.profile(stride)
    for k in range(len(_lib.PROF_NAMES)):
        p.profile_read(k, reset=True)
    t0 = time.perf_counter()
    p.forward(w.sources, save=True)
    p.adjoint(cot)
    p.gradient()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"workload": f"layered skin, outer {w.desc.n_outer[0]}^3, FEM {w.desc.fem_cells[0]}^3 hexes, "
                       f"{n_steps} steps forward + adjoint",
           "field_set_MB": round(w.desc.n_grid() * 36 / 1e6, 1),
           "gcell_steps_s": round((w.desc.n_grid() + w.desc.n_fem_owned()) * 2 * n_steps / wall / 1e9, 3)}
    for kind in ("step_fwd", "step_adj"):
        k = _lib.PROF_NAMES.index(kind)
        ms, n = p.profile_read(k, reset=True)
        b = unit_bytes(w.desc, p.n_det, kind == "step_adj")
        bmin = p.algorithmic_bytes(k)
        if n:
            sec = ms / n * 1e-3
            gbs = b / sec / 1e9
            out[kind] = {"avg_us": round(ms / n * 1e3, 2), "algorithmic_bytes": b,
                         "algorithmic_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "min_bytes": bmin, "min_bytes_GBs": round(bmin / sec / 1e9, 1),
                         "traffic": measured_traffic("traffic_bytes_per_launch_" + kind, PROBE_TRAFFIC_FILE)}
    p.profile(0)
    p.close()
    return out


def c3_autograd(reps=2):
    """Differentiation workload: 192^3 outer nodes, 96^3 FEM hexes, 1500 steps, forward
    checkpoints every 64 steps; one torch.autograd forward (traces) + backward (hand adjoint
    with segment recompute) of the loss 1/2 sum |E - E_obs|^2.  Recompute steps are not
    counted as cell-steps."""
    import numpy as np
    import torch
    import synth
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.autograd import solve
    w = synth.c3()
    dev = torch.device("cuda", 0)
    t_setup = time.perf_counter()
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device=dev),
                       torch.tensor(w.sigma_true, dtype=torch.float32, device=dev))
    eobs = p.forward(w.sources, save=False).clone()
    t_setup = time.perf_counter() - t_setup
    eps = torch.ones(p.n_fem, dtype=torch.float32, device=dev, requires_grad=True)
    sig = torch.zeros(p.n_fem, dtype=torch.float32, device=dev, requires_grad=True)

    def step():
        eps.grad = sig.grad = None
        r = (solve(p, eps, sig, w.sources) - eobs).double()
        loss = 0.5 * torch.sum(r * r)
        loss.backward()
        return loss

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    cells = w.desc.n_grid() + w.desc.n_fem_owned()
    finite = bool(torch.isfinite(eps.grad).all() and torch.isfinite(sig.grad).all())
    p.close()
    return {"workload": f"outer {w.desc.n_outer[0]}^3, FEM {w.desc.fem_cells[0]}^3 hexes, {w.desc.n_steps} steps, "
                        f"K = {w.desc.ckpt_every}, torch.autograd forward + backward",
            "ms": round(dt * 1e3, 2), "gcell_steps_s": round(cells * 2 * w.desc.n_steps / dt / 1e9, 3),
            "gradient_finite": finite, "setup_s": round(t_setup, 2)}


def paper_gradient_measure(prob, solve, eobs, t_exact):
    """The paper-formula gradient variant (eq. gradeps with grad(eps~).E dropped) on the main
    workload's solve: its cost on top of the exact gradient and how far it is from it."""
    import torch
    prob.profile(0)
    prob.paper_gradient(True)
    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ge, gs = solve()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    gp, _ = prob.gradient_paper()
    prob.paper_gradient(False)
    ge, gp = ge.double(), gp.double()
    rel = float(torch.linalg.norm(gp - ge) / torch.linalg.norm(ge))
    cos = float(torch.dot(gp, ge) / (torch.linalg.norm(gp) * torch.linalg.norm(ge)))
    return {"solve_ms": round(t * 1e3, 2), "extra_ms": round((t - t_exact) * 1e3, 2),
            "rel_l2_vs_exact": round(rel, 4), "cosine_vs_exact": round(cos, 4)}


def r2_measure(prob, solve, t_r1):
    """The main workload's solve with the symmetric div-div form R2 (element mean of eps - 1
    outside the divergence; the paper's gradient formula is then exact), against the R1 solve."""
    import torch
    prob.set_divdiv_form("R2")
    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solve()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    prob.set_divdiv_form("R1")
    return {"solve_ms": round(t * 1e3, 2), "r1_solve_ms": round(t_r1 * 1e3, 2)}


def cga_measure(prob, w, eobs, n_iter):
    """Reconstruction iterations (box "CGA") on the main workload from the paper's initial
    guess eps = 1, sigma = 0: each iteration is a solve (forward with saving, the misfit J on
    the device, misfit adjoint, gradient) and the device update.  The step sizes and regularisation are set from the
    gradient at the initial guess (setup, not timed): the first update moves eps by at most
    0.5 and sigma by at most 0.1, and gamma^0 = max|g^0| / that bound, so that alpha^1 =
    1 / gamma^0 keeps the same scale."""
    import numpy as np
    import torch
    from paper_2508_07780_amd import CGA, CGAParams
    dev = eobs.device
    n = prob.n_fem
    eps0 = torch.ones(n, dtype=torch.float32, device=dev)
    sig0 = torch.zeros(n, dtype=torch.float32, device=dev)
    prob.set_coefficients(eps0, sig0)
    tr = prob.forward(w.sources, save=True)
    prob.adjoint_misfit(tr, eobs)
    ge, gs = prob.gradient()
    prm = CGAParams.from_gradient(ge, gs, w.desc.h, eps_max=20.0, sig_max=3.0)
    del tr, ge, gs
    c = CGA(prob, w.sources, eobs, eps0, sig0, prm, track_loss=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * n_iter)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for m in range(n_iter):
        c.solve()
        ev[2 * m].record()
        c.update()
        ev[2 * m + 1].record()
        hist.append(c.info())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    upd_us = sum(ev[2 * m].elapsed_time(ev[2 * m + 1]) for m in range(n_iter)) / n_iter * 1e3
    n_free = int(np.prod([max(int(x) - 3, 0) for x in w.desc.fem_cells]))
    upd_bytes = 104.0 * n_free     # gradient, iterate, centre read twice; direction read and written; iterate written
    cells = (w.desc.n_grid() + w.desc.n_fem_owned()) * 2 * w.desc.n_steps * len(w.sources)
    c.close()
    rnd = lambda x: float("%.4g" % x)  # noqa: E731
    return {
        "iterations": n_iter, "ms_per_iteration": round(elapsed / n_iter * 1e3, 2),
        "gcell_steps_s": round(cells * n_iter / elapsed / 1e9, 2),
        "update_us": round(upd_us, 2), "update_algorithmic_bytes": upd_bytes,
        "update_GBs": round(upd_bytes / (upd_us * 1e-6) / 1e9, 1),
        "params": {k: rnd(v) for k, v in vars(prm).items() if not k.startswith("eta")},
        "history": [{"J": rnd(i["J"]), "grad_norm": [rnd(i["grad_norm"]["eps"]), rnd(i["grad_norm"]["sig"])],
                     "step_norm": [rnd(i["step_norm"]["eps"]), rnd(i["step_norm"]["sig"])],
                     "beta": [rnd(i["beta"]["eps"]), rnd(i["beta"]["sig"])]} for i in hist],
    }


def serving_comparison(n_jobs=48, ranges="small"):
    """Continuous batching vs one solve at a time on the same uneven request stream.

    Requests (seeded), ranges "small": outer grids {64, 96, 128}^3, FEM boxes {32, 48}^3 hexes,
    1-4 plane-wave or dipole sources, 300-800 steps, 2-4 reconstruction iterations each;
    "full": outer {64, 96, 128, 160, 224}^3, FEM {32, 48, 64, 96}^3, 1-8 sources, 500-2000
    steps, 3-10 iterations.  A burst (all jobs at t = 0) measures throughput; Poisson
    arrivals at 0.8x the measured one-at-a-time capacity measure latency.
    """
    import synth
    from paper_2508_07780_amd import serving
    if ranges == "full":
        kw = {}
        label = "outer {64,96,128,160,224}^3, FEM {32,48,64,96}^3 hexes, 1-8 sources, 500-2000 steps, 3-10 iterations"
    else:
        kw = dict(outer=(64, 96, 128), fem=(32, 48), sources=(1, 4), steps=(300, 800), iterations=(2, 4))
        label = "outer {64,96,128}^3, FEM {32,48}^3 hexes, 1-4 sources, 300-800 steps, 2-4 iterations"
    burst = synth.serving_requests(n_jobs, 1e9, **kw)
    for r in burst:
        r.arrival = 0.0
    serving.serve_serial(burst[:2])                       # warm-up
    s_serial, _ = serving.serve_serial(burst)
    progress("serving: burst, one at a time")
    s_batch, _ = serving.serve_batched(burst, max_slots=16)
    progress("serving: burst, batched")
    rate = 0.8 * s_serial["jobs"] / s_serial["makespan_s"]
    stream = synth.serving_requests(n_jobs, rate, **kw)
    l_serial, _ = serving.serve_serial(stream)
    progress("serving: Poisson stream, one at a time")
    l_batch, _ = serving.serve_batched(stream, max_slots=16)
    progress("serving: Poisson stream, batched")
    keep = ("jobs", "solves", "makespan_s", "throughput_gcell_steps_s", "latency_p50_s", "latency_p99_s")
    pick = lambda d: {k: (round(d[k], 4) if isinstance(d[k], float) else d[k]) for k in keep}  # noqa: E731
    return {
        "workload": "%d jobs: %s; seeded" % (n_jobs, label),
        "burst": {"batched": pick(s_batch), "one_at_a_time": pick(s_serial),
                  "throughput_ratio": round(s_batch["throughput_gcell_steps_s"] / s_serial["throughput_gcell_steps_s"], 3)},
        "poisson_0.8x": {"rate_jobs_per_s": round(rate, 3), "batched": pick(l_batch), "one_at_a_time": pick(l_serial)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-steps", type=int, default=2000, help="time steps per solve")
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="forward checkpoint interval K for the adjoint; 0 = store every FEM level "
                         "(no recompute; 12.6 GB for the default workload)")
    ap.add_argument("--cpu-sample-steps", type=int, default=20, help="0 skips the oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="skip the HIP-event kernel timing")
    ap.add_argument("--serving", type=int, default=1, help="0 skips the batched / serving comparison")
    ap.add_argument("--serving-jobs", type=int, default=48, help="requests of the serving comparison")
    ap.add_argument("--serving-ranges", choices=("small", "full"), default="small",
                    help="request size ranges of the serving comparison")
    ap.add_argument("--serving-full-jobs", type=int, default=6,
                    help="requests of a second serving comparison at the full serving ranges (0 skips)")
    ap.add_argument("--probe", type=int, default=1, help="0 skips the 288^3 bandwidth probe")
    ap.add_argument("--probe-only", action="store_true",
                    help="run only the 288^3 probe (for profilers) and print its JSON")
    ap.add_argument("--probe-steps", type=int, default=300, help="time steps of the probe")
    ap.add_argument("--c3", type=int, default=1, help="0 skips the 192^3 autograd measurement")
    ap.add_argument("--cga", type=int, default=3, help="CGA iterations to time on the main workload (0 skips)")
    ap.add_argument("--paper-gradient", type=int, default=1,
                    help="0 skips the paper-formula gradient variant's measurement")
    ap.add_argument("--refined", type=int, default=1, help="0 skips the solve on a locally refined mesh")
    ap.add_argument("--acga", type=int, default=1, help="0 skips the adaptive reconstruction (box ACGA)")
    ap.add_argument("--small", type=int, default=1,
                    help="0 skips the plain forward config's launch-by-launch / graph comparison")
    ap.add_argument("--profile-stride", type=int, default=64,
                    help="time every k-th step launch with HIP events (k >= 16 barely perturbs the run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs one problem per GPU and this build has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2508_07780_amd import Problem, _lib

    torch.cuda.set_device(0)
    if args.probe_only:
        print(json.dumps(large_probe(args.probe_steps)), flush=True)
        return
    w = synth.c2(n_steps=args.n_steps)
    w.desc.ckpt_every = args.ckpt_every if args.ckpt_every > 0 else w.desc.n_steps
    dev = torch.device("cuda", 0)
    prob = Problem(w.desc)
    # observed data: seeded true model + 3% Gaussian noise (setup, not timed)
    prob.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device=dev),
                          torch.tensor(w.sigma_true, dtype=torch.float32, device=dev))
    tr_true = prob.forward(w.sources, save=False)
    xi = synth.noise(tuple(tr_true.shape), w.seed).astype(np.float32)
    eobs = tr_true * (1.0 + w.noise_level * torch.from_numpy(xi).to(dev))
    del xi, tr_true
    eps0 = torch.ones(prob.n_fem, dtype=torch.float32, device=dev)     # initial guess (paper: eps = 1, sigma = 0)
    sig0 = torch.zeros(prob.n_fem, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    traces = torch.empty_like(eobs)
    g_out = (torch.empty(prob.n_fem, dtype=torch.float64, device=dev),
             torch.empty(prob.n_fem, dtype=torch.float64, device=dev))

    def solve():
        prob.set_coefficients(eps0, sig0)
        prob.forward(w.sources, save=True, out=traces)
        prob.adjoint_misfit(traces, eobs)     # cotangent traces - E_obs of J = 1/2 sum |E - E_obs|^2
        return prob.gradient(out=g_out)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    if not args.no_profile:
        prob.profile(args.profile_stride)
        for k in range(len(_lib.PROF_NAMES)):
            prob.profile_read(k, reset=True)
    lat = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        g_eps, g_sig = solve()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    kern = {}
    if not args.no_profile:
        for k, name in enumerate(_lib.PROF_NAMES):
            ms, n = prob.profile_read(k, reset=True)
            b = prob.algorithmic_bytes(k)
            if n:
                kern[name] = {"launches": n, "avg_us": ms / n * 1e3, "min_bytes": b,
                              "min_bytes_GBs": b / (ms / n * 1e-3) / 1e9}
                if name in ("step_fwd", "step_adj"):
                    u = unit_bytes(w.desc, prob.n_det, name == "step_adj")
                    kern[name]["algorithmic_bytes"] = u
                    kern[name]["algorithmic_GBs"] = u / (ms / n * 1e-3) / 1e9
        prob.profile(0)

    n_src = len(w.sources)
    cells = w.desc.n_grid() + w.desc.n_fem_owned()
    cell_steps = cells * 2 * w.desc.n_steps * n_src
    value = cell_steps * args.steps / elapsed / 1e9
    finite = bool(torch.isfinite(g_eps).all() and torch.isfinite(g_sig).all())

    roofline = None
    dom = "step_fwd" if "step_fwd" in kern else None
    if dom:
        k = kern[dom]
        achieved = k["algorithmic_GBs"]
        traffic = measured_traffic("traffic_bytes_per_launch_step_fwd") if dom == "step_fwd" else None
        llc = 24 * w.desc.n_grid() <= LLC_BYTES
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": "step_kernel (fused FD + FEM, forward)",
                    "avg_us": round(k["avg_us"], 2), "algorithmic_bytes_per_launch": k["algorithmic_bytes"],
                    "bytes_per_unit": UNIT_BYTES,
                    "min_bytes_per_launch": k["min_bytes"], "min_bytes_frac": round(k["min_bytes_GBs"] / HBM_PEAK_GBS, 4),
                    "llc_resident": llc,
                    "note": ("the grid's two E levels fit the 256 MB last-level cache: an algorithmic rate against "
                             "the HBM peak, not an HBM fraction; roofline_hbm is the HBM-valid figure")
                    if llc else "fields exceed the last-level cache"}

    out = {
        "metric": "Gcell-steps/s fwd+adj (HBM % of peak), FP32 vs oracle err; p50/p99 solve latency",
        "value": round(value, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "layered-skin forward+adjoint+gradient solve", "outer_nodes": list(w.desc.n_outer),
                   "fem_hexes": list(w.desc.fem_cells), "tets": 6 * int(np.prod(w.desc.fem_cells)),
                   "time_steps": w.desc.n_steps, "sources": n_src, "ckpt_every": w.desc.ckpt_every,
                   "cells": cells},
        "latency_ms": {"p50": round(_percentile(lat, 50), 2), "p99": round(_percentile(lat, 99), 2)},
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 2) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "gradient_finite": finite,
    }
    if args.paper_gradient:
        out["paper_formula_gradient"] = paper_gradient_measure(prob, solve, eobs, elapsed / args.steps)
    if args.paper_gradient:
        out["r2_form"] = r2_measure(prob, solve, elapsed / args.steps)
    if args.cga:
        out["cga"] = cga_measure(prob, w, eobs, args.cga)
    del prob
    if args.refined:
        out["refined_mesh"] = refined_mesh_measure(w)
        progress("refined mesh")
    if args.acga:
        out["acga"] = acga_measure(w)
        progress("adaptive reconstruction")
    if args.small:
        out["small_graphs"] = small_graphs_measure()
        progress("plain forward config, graphs")
    progress("main workload")
    if args.probe:
        out["hbm_probe"] = large_probe(args.probe_steps)
        pf = out["hbm_probe"].get("step_fwd")
        if pf:
            out["roofline_hbm"] = {"bound": "hbm", "achieved": pf["algorithmic_GBs"], "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": pf["frac"], "traffic": pf["traffic"],
                                   "kernel": "step_kernel (fused FD + FEM, forward, streaming tile variant)",
                                   "avg_us": pf["avg_us"], "algorithmic_bytes_per_launch": pf["algorithmic_bytes"],
                                   "bytes_per_unit": UNIT_BYTES, "min_bytes_per_launch": pf["min_bytes"],
                                   "min_bytes_frac": round(pf["min_bytes_GBs"] / HBM_PEAK_GBS, 4),
                                   "workload": out["hbm_probe"]["workload"], "llc_resident": False}
        progress("288^3 probe")
    if args.c3:
        out["c3_autograd"] = c3_autograd()
        progress("192^3 autograd")
    if args.serving:
        out["batched_mix"] = batch_comparison()
        progress("batched mix")
        out["serving"] = serving_comparison(args.serving_jobs, args.serving_ranges)
        if args.serving_full_jobs > 0:
            out["serving_full_ranges"] = serving_comparison(args.serving_full_jobs, "full")
    if args.cpu_sample_steps > 0:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
        progress("oracle baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
