"""Batched solves and the serving loop on the GPU.

* Alone vs in the mix: problems of different grid sizes, FEM boxes, step counts,
  source counts and checkpoint intervals give the same traces and gradients when
  solved one by one through dd_forward / dd_adjoint / dd_gradient and when solved
  together in a batch (one launch per step for all of them), also when a job joins
  the batch while others are running.  The kernels are the same device code, so the
  results are expected bit for bit; the bar is 1e-6 relative.
* One batched problem is also checked against the FP64 oracle (absolute correctness).
* Serving: every job of a request stream completes under continuous batching and
  one-at-a-time, the HBM admission budget is never exceeded, and results of a job do not
  depend on what else was in the batch.
"""

import math

import numpy as np
import pytest

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward

pytestmark = pytest.mark.gpu


def _mix():
    out = []
    specs = [((40, 40, 40), 1.0 / 20, (10, 10, 10), (20, 20, 20), 90, 32),
             ((56, 48, 52), 1.0 / 24, (14, 12, 13), (24, 22, 24), 140, 140),
             ((33, 37, 35), 0.03, (11, 12, 10), (11, 13, 14), 75, 16)]
    for i, (no, h, lo, cells, nt, ck) in enumerate(specs):
        desc = synth.ProblemDesc(n_outer=no, h=h, origin=(0.0, 0.0, 0.0), fem_lo=lo, fem_cells=cells,
                                 dt=0.5 * h / math.sqrt(3.0), n_steps=nt, ckpt_every=ck,
                                 detector_faces=synth.FACE_TOP | (synth.FACE_XMAX if i == 1 else 0))
        src = synth.gauss_sine(2 * math.pi / (12 * h), pol=(0.2 * i, 1.0, 0.1))
        desc.t_switch = src.support_end()
        rng = np.random.Generator(np.random.PCG64(77 + i))
        eps, sig, _ = synth.configs.skin_media(desc, rng) if i != 2 else (*synth.configs.random_media(desc, rng), None)
        srcs = [src]
        if i == 1:
            srcs.append(synth.Source(kind=synth.SRC_DIPOLE, omega=src.omega, t0=src.t0, width=src.width,
                                     pol=(0.0, 0.3, 1.0), pos=(no[0] // 2, no[1] // 2, no[2] - 3)))
        out.append(synth.Workload(f"b{i}", desc, eps, sig, srcs, 100 + i))
    return out


def _obs(torch, p, n_src, seed):
    """Seeded synthetic observations (host generator), on the device."""
    return torch.tensor(1e-2 * synth.noise((n_src, p.n_steps, p.n_det, 3), seed), dtype=torch.float32,
                        device="cuda")


def _alone(torch, w, obs):
    from paper_2508_07780_amd import Problem
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    tr = p.forward(w.sources, save=True).clone()
    p.adjoint((tr - obs).contiguous())
    ge, gs = p.gradient()
    return tr, ge.clone(), gs.clone()


def _rel(a, b):
    return float((a - b).double().norm() / b.double().norm())


@pytest.mark.parametrize("fd_nt", ["0", "1"])
@pytest.mark.parametrize("fill", [None, 0, 1])
def test_batch_equals_alone_including_late_join(fill, fd_nt, monkeypatch):
    """fill: the library's default fill target (these small jobs all share each launch), 0
    (every job in every launch), 1 (one job per launch, oldest first: the late job waits).
    fd_nt: the finite-difference tiles' cached (0) or streaming (1) variant, for the batch's
    launches (the batched kernel's streaming instantiation) and the problems alone."""
    import torch
    monkeypatch.setenv("DD_FD_NT", fd_nt)
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.batch import Batch
    mix = _mix()
    probs, obs = [], []
    for i, w in enumerate(mix):
        p = Problem(w.desc)
        p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                           torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
        probs.append(p)
        obs.append(_obs(torch, p, len(w.sources), 5 + i))
    batch = Batch(8, fill_cells=fill)
    ids = [batch.submit(probs[i], mix[i].sources, obs=obs[i]) for i in (0, 1)]
    batch.step(25)                     # the third job joins while the others run
    ids.append(batch.submit(probs[2], mix[2].sources, obs=obs[2]))
    recs = {r["id"]: r for r in batch.run_to_completion(chunk=16)}
    torch.cuda.synchronize()
    for i, w in enumerate(mix):
        print(f"[gpu] batch (fill {fill}, fd_nt {fd_nt}) vs alone {w.name}", flush=True)
        r = recs[ids[i]]
        tr, ge, gs = _alone(torch, w, obs[i])
        same = torch.equal(r["traces"], tr) and torch.equal(r["g_eps"], ge) and torch.equal(r["g_sigma"], gs)
        print(f"[gpu]   bitwise equal: {same}", flush=True)
        assert _rel(r["traces"], tr) <= 1e-6
        assert _rel(r["g_eps"], ge) <= 1e-6 and _rel(r["g_sigma"], gs) <= 1e-6
    batch.close()


def test_batched_solve_matches_oracle():
    import torch
    from paper_2508_07780_amd import Problem
    from paper_2508_07780_amd.batch import Batch
    w = _mix()[2]
    p = Problem(w.desc)
    p.set_coefficients(torch.tensor(w.eps, dtype=torch.float32, device="cuda"),
                       torch.tensor(w.sigma, dtype=torch.float32, device="cuda"))
    d = Discretization(w.desc).set_coefficients(w.eps.astype(np.float32).astype(np.float64),
                                                w.sigma.astype(np.float32).astype(np.float64))
    fw = forward(d, w.sources[0])
    # observations from the oracle's traces: a coherent misfit, as in a reconstruction
    ob = torch.tensor((0.9 * fw["traces"])[None].astype(np.float32), device="cuda")
    b = Batch(4)
    b.submit(p, w.sources, obs=ob)
    rec = b.run_to_completion(chunk=8)[0]
    tr = rec["traces"][0].cpu().numpy()
    assert np.linalg.norm(tr - fw["traces"]) <= 1e-4 * np.linalg.norm(fw["traces"])
    cot = fw["traces"] - ob[0].cpu().numpy().astype(np.float64)
    ag = adjoint_gradient(d, cot, fw)
    ge = rec["g_eps"].cpu().numpy()
    assert np.linalg.norm(ge - ag["g_eps"]) <= 1e-3 * np.linalg.norm(ag["g_eps"])
    b.close()


def test_serving_completes_and_respects_budget():
    import torch
    from paper_2508_07780_amd import serving
    reqs = synth.serving_requests(6, 20.0, outer=(40, 48), fem=(16, 24), sources=(1, 3), steps=(40, 90),
                                  iterations=(2, 3))
    for r in reqs:
        r.arrival = 0.0                 # a burst: admission is bound by the budget alone
    fps = sorted(serving.job_footprint(r) for r in reqs)
    budget = fps[-1] + fps[-2]          # the two largest jobs fit at once, never all six
    s_b, rec_b = serving.serve_batched(reqs, max_slots=4, hbm_budget=budget, chunk=16, keep=True)
    s_s, rec_s = serving.serve_serial(reqs, keep=True)
    print(f"[gpu] serving batched {s_b}", flush=True)
    print(f"[gpu] serving serial  {s_s}", flush=True)
    assert s_b["jobs"] == len(reqs) == s_s["jobs"]
    assert s_b["solves"] == s_s["solves"] == sum(r.iterations for r in reqs)
    assert all(r["done"] >= r["arrival"] for r in rec_b + rec_s)
    assert s_b["peak_admitted_bytes"] <= budget
    assert 2 <= s_b["peak_concurrent_jobs"] < len(reqs)
    # both servers run the same CGA iterations per job: the same reconstruction (the
    # gradients' FP64 sums differ only in order)
    by_rid = {r["rid"]: r for r in rec_s}
    for r in rec_b:
        for f, base in (("eps", 1.0), ("sigma", 0.0)):
            a, b = (x[f].double() - base for x in (r, by_rid[r["rid"]]))
            assert float(torch.linalg.norm(b)) > 0
            assert float(torch.linalg.norm(a - b)) <= 1e-4 * float(torch.linalg.norm(b)), (r["rid"], f)


@pytest.mark.parametrize("overlap,slots", [(True, 2), (True, 1), (False, 1)])
def test_serving_runs_large_jobs_alone(overlap, slots):
    """Jobs at or above the solo threshold run through the single-problem calls (the
    one-at-a-time server's calls: the same reconstruction bit for bit), on streams and host
    threads of their own beside the batch (two or one at a time), or after the batch has
    drained; the others are batched; every job completes."""
    import torch
    from paper_2508_07780_amd import serving
    reqs = synth.serving_requests(6, 20.0, outer=(40, 48), fem=(16, 24), sources=(1, 3), steps=(40, 90),
                                  iterations=(2, 3))
    cells = sorted(serving.step_cells(r.workload.desc) for r in reqs)
    thr = cells[len(cells) // 2]
    solo = {r.rid for r in reqs if serving.step_cells(r.workload.desc) >= thr}
    assert 0 < len(solo) < len(reqs)
    s_b, rec_b = serving.serve_batched(reqs, max_slots=4, chunk=16, keep=True, solo_cells=thr,
                                       solo_overlap=overlap, solo_slots=slots)
    assert s_b["in_use_end_bytes"] == 0
    s_s, rec_s = serving.serve_serial(reqs, keep=True)
    print(f"[gpu] serving with {len(solo)} solo jobs: {s_b}", flush=True)
    assert s_b["jobs"] == len(reqs) and s_b["solves"] == s_s["solves"]
    by_rid = {r["rid"]: r for r in rec_s}
    for r in rec_b:
        for f, base in (("eps", 1.0), ("sigma", 0.0)):
            a, b = (x[f].double() - base for x in (r, by_rid[r["rid"]]))
            if r["rid"] in solo:
                assert torch.equal(a, b), (r["rid"], f)
            else:
                assert float(torch.linalg.norm(a - b)) <= 1e-4 * float(torch.linalg.norm(b)), (r["rid"], f)


def test_batch_and_serving_refusals():
    """A negative fill target is rejected; a request larger than the whole HBM budget raises
    instead of waiting for room that never comes."""
    from paper_2508_07780_amd import DDError, serving
    from paper_2508_07780_amd.batch import Batch
    with pytest.raises(DDError) as e:
        Batch(2, fill_cells=-1)
    assert e.value.code == -1
    reqs = synth.serving_requests(2, 20.0, outer=(40, 48), fem=(16, 24), sources=(1, 2), steps=(40, 60),
                                  iterations=(2, 2))
    small = min(serving.job_footprint(r) for r in reqs) // 2
    with pytest.raises(ValueError):
        serving.serve_batched(reqs, max_slots=2, hbm_budget=small, chunk=16)


def _small_requests(n, seed_shift=0):
    return synth.serving_requests(n, 20.0, seed=synth.configs.SEED_BASE + 5 + seed_shift, outer=(40, 48),
                                  fem=(16, 24), sources=(1, 2), steps=(40, 70), iterations=(2, 3))


def test_serving_failures_release_budget_and_requeue_or_reject(monkeypatch):
    """Failures injected on the host (no device fault): a submit that fails once is queued again
    and completes; a job whose submit always fails is rejected after its retry; a batch step that
    fails sends every job of the batch back to the queue.  Every byte of the budget comes back and
    the other jobs finish."""
    from paper_2508_07780_amd import DDError, serving
    from paper_2508_07780_amd.batch import Batch
    reqs = _small_requests(6)
    doomed, flaky = reqs[1].workload.desc, reqs[3].workload.desc
    calls = {"flaky": 0, "step": 0}
    real_submit, real_step = Batch.submit, Batch.step

    def submit(self, problem, sources, obs=None, gradient=True):
        if problem.desc is doomed:
            raise DDError(-4, "injected")
        if problem.desc is flaky and calls["flaky"] == 0:
            calls["flaky"] += 1
            raise DDError(-4, "injected once")
        return real_submit(self, problem, sources, obs=obs, gradient=gradient)

    def step(self, max_steps):
        calls["step"] += 1
        if calls["step"] == 3:
            raise DDError(-5, "injected step failure")
        return real_step(self, max_steps)

    monkeypatch.setattr(Batch, "submit", submit)
    monkeypatch.setattr(Batch, "step", step)
    s, rec = serving.serve_batched(reqs, max_slots=4, chunk=16, solo_cells=None)
    print(f"[gpu] serving with injected failures: {s}", flush=True)
    assert s["rejected"] == 1 and s["jobs"] == len(reqs) - 1
    assert s["in_use_end_bytes"] == 0
    done = {r["rid"] for r in rec if not r.get("rejected")}
    assert reqs[1].rid not in done and reqs[3].rid in done
    assert s["solves"] == sum(r.iterations for r in reqs if r.rid != reqs[1].rid)


def test_serving_solo_failure_is_requeued(monkeypatch):
    """A job beside the batch whose solve fails once (injected on the host, in its thread) is
    released, queued again and completes; the budget comes back."""
    from paper_2508_07780_amd import DDError, serving
    reqs = synth.serving_requests(4, 20.0, outer=(40, 48), fem=(16, 24), sources=(1, 2), steps=(40, 60),
                                  iterations=(2, 2))
    cells = sorted(serving.step_cells(r.workload.desc) for r in reqs)
    thr = cells[-1]
    big = [r for r in reqs if serving.step_cells(r.workload.desc) >= thr][0]
    real = serving._run_alone
    calls = {"n": 0}

    def run_alone(job):
        if job.req.rid == big.rid and calls["n"] == 0:
            calls["n"] += 1
            raise DDError(-4, "injected")
        return real(job)

    monkeypatch.setattr(serving, "_run_alone", run_alone)
    s, rec = serving.serve_batched(reqs, max_slots=4, chunk=16, solo_cells=thr)
    print(f"[gpu] serving with an injected solo failure: {s}", flush=True)
    assert calls["n"] == 1 and s["rejected"] == 0 and s["jobs"] == len(reqs)
    assert s["in_use_end_bytes"] == 0 and s["retried"] == 1


def test_served_job_matches_the_oracle_cga():
    """One request through the batched server: its reconstruction after its iterations equals the
    oracle's CGA from the same start, data and step-size rule (step sizes from the first gradient:
    the first update moves eps by at most 0.5 and sigma by at most 0.1)."""
    import torch
    from oracle.cga import cga, solve_gradient
    from paper_2508_07780_amd import serving
    w = synth.small("tiny")
    w.desc.n_steps = 60
    h3 = w.desc.h ** 3
    d = Discretization(w.desc).set_coefficients(w.eps.astype(np.float32).astype(np.float64),
                                                w.sigma.astype(np.float32).astype(np.float64))
    eobs = forward(d, w.sources[0])["traces"][None].astype(np.float32)      # data of the true medium
    n = w.desc.n_fem_nodes()
    start = synth.Workload("served", w.desc, np.ones(n), np.zeros(n), w.sources, 7, extra={"obs": eobs})
    req = synth.Request(0, 0.0, start, 2)
    s, rec = serving.serve_batched([req], max_slots=2, chunk=16, keep=True, solo_cells=None)
    torch.cuda.synchronize()
    assert s["jobs"] == 1
    do = Discretization(w.desc)
    grad_fn = solve_gradient(do, w.sources, eobs.astype(np.float64))
    ge, gs, _ = grad_fn(np.ones(n), np.zeros(n))
    G = [max(np.abs(g).max() / h3, 1e-30) for g in (ge, gs)]
    prm = dict(gamma_eps=G[0] / 0.5, gamma_sig=G[1] / 0.1, p=0.5, alpha_eps=0.5 / G[0], alpha_sig=0.1 / G[1],
               eps_max=20.0, sig_max=3.0)
    hist = cga(do, w.sources, eobs.astype(np.float64), np.ones(n), np.zeros(n), prm, 2)
    for f, key, base in (("eps", "eps", 1.0), ("sig", "sigma", 0.0)):
        ref = hist[-1][f]["coef"] - base
        got = rec[0][key].double().cpu().numpy() - base
        e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"[gpu] served job vs oracle CGA, {f}: change rel L2 {e:.2e}", flush=True)
        assert e <= 2e-3
