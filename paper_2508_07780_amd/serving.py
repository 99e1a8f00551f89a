"""Request loop: continuous batching of reconstruction solves with HBM admission.

Jobs arrive over time.  Each job is a sequence of reconstruction iterations of one
problem (box "CGA": forward, misfit adjoint, eps/sigma gradient, then the conjugate
gradient update of eps and sigma on the device); the problem's fields stay resident
between its solves.  A job is admitted
when a batch slot is free and its device footprint (dd_footprint_bytes plus its trace,
observation and gradient buffers) fits in the HBM budget; admitted solves join the
running batch at the next launch, so work of jobs of different sizes overlaps on the
device.  A job whose single step already fills the GPU (at least `solo_cells` cells per
step) gains nothing from sharing launches and is slower through the batch kernel: it waits
until the batch is empty and then runs alone through the single-problem calls, in arrival
order like every other job.  The one-at-a-time server runs the same jobs in arrival order through the
single-problem calls, for comparison.

Requests are plain objects with `arrival` (s), `iterations` and `workload` (desc, sources,
initial eps / sigma, seed).  Observations are seeded synthetic data of the traces' shape:
the cost of a solve does not depend on their values.
"""

import time

import numpy as np
import torch

from .batch import Batch
from .cga import CGA, CGAParams
from .solver import Problem


# coefficient box of the reconstruction (eq. epsilon_sigma_constraint)
EPS_MAX, SIG_MAX = 20.0, 3.0


def cell_steps(desc, n_src):
    """Cells (outer nodes + FEM-owned nodes) x (forward + adjoint steps) x sources of one solve."""
    n_own = int(np.prod([max(int(c) - 1, 0) for c in desc.fem_cells]))
    n_grid = int(np.prod([int(v) for v in desc.n_outer]))
    return (n_grid + n_own) * 2 * int(desc.n_steps) * n_src


class _Job:
    def __init__(self, req, dev):
        w = req.workload
        self.req = req
        self.problem = Problem(w.desc)
        self.eps = torch.tensor(w.eps, dtype=torch.float32, device=dev)
        self.sigma = torch.tensor(w.sigma, dtype=torch.float32, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(int(w.seed))
        shape = (len(w.sources), w.desc.n_steps, self.problem.n_det, 3)
        self.obs = 1e-3 * torch.randn(shape, generator=g, device=dev, dtype=torch.float32)
        self.done_iters = 0
        self.cga = None
        self.problem.set_coefficients(self.eps, self.sigma)

    def update(self, g_eps, g_sigma):
        """CGA steps 2-6 on the device; the run (and its step sizes) starts at the first gradient."""
        if self.cga is None:
            w = self.req.workload
            prm = CGAParams.from_gradient(g_eps, g_sigma, w.desc.h, eps_max=EPS_MAX, sig_max=SIG_MAX)
            self.cga = CGA(self.problem, w.sources, self.obs, self.eps, self.sigma, prm)
        self.cga.update(g_eps, g_sigma)
        self.problem.set_coefficients(self.cga.eps, self.cga.sigma)

    def close(self):
        if self.cga is not None:
            self.cga.close()
        self.problem.close()


def job_footprint(req):
    w = req.workload
    n_src = len(w.sources)
    traces = n_src * int(w.desc.n_steps) * _n_det(w.desc) * 3 * 4
    # problem, traces and observations, gradients (FP64), iterate (float32) and the CGA state
    # (Tikhonov centres float32, directions FP64)
    return Problem.footprint_bytes(w.desc, n_src) + 2 * traces + (16 + 8 + 24) * w.desc.n_fem_nodes()


def _n_det(desc):
    return len(Problem.detector_nodes(desc))


def _summary(lat, solves, makespan, work):
    lat = sorted(lat)
    pct = lambda q: float(np.percentile(lat, q)) if lat else None  # noqa: E731
    return {"jobs": len(lat), "solves": solves, "makespan_s": makespan,
            "throughput_gcell_steps_s": work / makespan / 1e9 if makespan > 0 else None,
            "latency_p50_s": pct(50), "latency_p99_s": pct(99), "latency_mean_s": float(np.mean(lat)) if lat else None}


def _final(job):
    return {"eps": job.cga.eps.clone(), "sigma": job.cga.sigma.clone()}


def step_cells(desc):
    """Cells (outer nodes + FEM-owned nodes) one time step of the problem advances."""
    return cell_steps(desc, 1) // (2 * int(desc.n_steps))


def _run_alone(job):
    """All iterations of one job through the single-problem calls."""
    req = job.req
    for _ in range(req.iterations):
        tr = job.problem.forward(req.workload.sources, save=True)
        job.problem.adjoint_misfit(tr, job.obs)
        ge, gs = job.problem.gradient()
        job.update(ge, gs)
        job.done_iters += 1


def serve_batched(requests, max_slots=16, hbm_budget=None, chunk=256, time_fn=time.perf_counter, keep=False,
                  solo_cells=3_000_000, fill_cells=None):
    """Continuous batching: returns a summary dict and per-job records (with each job's final
    eps and sigma when keep is set).  Jobs of at least solo_cells cells per step run alone
    through the single-problem calls (None: every job is batched).  fill_cells: the batch's
    fill target per launch (None: the library's default)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if hbm_budget is None:
        free, _ = torch.cuda.mem_get_info()
        hbm_budget = int(0.9 * free)
    pending = sorted(requests, key=lambda r: r.arrival)
    batch = Batch(max_slots, fill_cells=fill_cells)
    active = {}           # job id in the batch -> _Job
    in_use = 0
    lat, records = [], []
    solves = 0
    work = 0
    peak_bytes = peak_jobs = 0
    t0 = time_fn()
    while pending or active:
        now = time_fn() - t0
        # admission: arrived, a slot free, the footprint fits
        while pending and pending[0].arrival <= now and len(active) < max_slots:
            fp = job_footprint(pending[0])
            if fp > hbm_budget:
                raise ValueError(f"request {pending[0].rid} needs {fp} bytes, over the HBM budget of {hbm_budget}")
            if solo_cells is not None and step_cells(pending[0].workload.desc) >= solo_cells:
                if active:
                    break                # the batch drains first (arrival order is kept)
                req = pending.pop(0)
                peak_bytes = max(peak_bytes, fp)
                peak_jobs = max(peak_jobs, 1)
                job = _Job(req, dev)
                _run_alone(job)
                solves += req.iterations
                work += cell_steps(req.workload.desc, len(req.workload.sources)) * req.iterations
                t_done = time_fn() - t0
                lat.append(t_done - req.arrival)
                records.append({"rid": req.rid, "arrival": req.arrival, "done": t_done, "iterations": req.iterations,
                                **(_final(job) if keep else {})})
                job.close()
                now = time_fn() - t0
                continue
            if in_use + fp > hbm_budget:
                break
            req = pending.pop(0)
            job = _Job(req, dev)
            job.footprint = fp
            in_use += fp
            jid = batch.submit(job.problem, req.workload.sources, obs=job.obs)
            active[jid] = job
            peak_bytes = max(peak_bytes, in_use)
            peak_jobs = max(peak_jobs, len(active))
        if not active:
            if not pending:
                break            # the last jobs ran alone
            # idle until the next arrival
            time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
            continue
        batch.step(chunk)
        finished, _ = batch.poll()
        for rec in finished:
            job = active.pop(rec["id"])
            job.update(rec["g_eps"], rec["g_sigma"])      # synchronises the stream
            solves += 1
            work += cell_steps(job.req.workload.desc, len(job.req.workload.sources))
            job.done_iters += 1
            if job.done_iters < job.req.iterations:
                jid = batch.submit(job.problem, job.req.workload.sources, obs=job.obs)
                active[jid] = job
            else:
                t_done = time_fn() - t0
                lat.append(t_done - job.req.arrival)
                records.append({"rid": job.req.rid, "arrival": job.req.arrival, "done": t_done,
                                "iterations": job.done_iters, **(_final(job) if keep else {})})
                job.close()
                in_use -= job.footprint
    torch.cuda.synchronize()
    makespan = time_fn() - t0
    batch.close()
    out = _summary(lat, solves, makespan, work)
    out.update(hbm_budget_bytes=hbm_budget, peak_admitted_bytes=peak_bytes, peak_concurrent_jobs=peak_jobs)
    return out, records


def serve_serial(requests, time_fn=time.perf_counter, keep=False):
    """One solve at a time, jobs in arrival order, through the single-problem calls."""
    dev = torch.device("cuda", torch.cuda.current_device())
    lat, records = [], []
    solves = 0
    work = 0
    t0 = time_fn()
    for req in sorted(requests, key=lambda r: r.arrival):
        now = time_fn() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        job = _Job(req, dev)
        for _ in range(req.iterations):
            tr = job.problem.forward(req.workload.sources, save=True)
            job.problem.adjoint_misfit(tr, job.obs)
            ge, gs = job.problem.gradient()
            job.update(ge, gs)
            solves += 1
            work += cell_steps(req.workload.desc, len(req.workload.sources))
        t_done = time_fn() - t0
        lat.append(t_done - req.arrival)
        records.append({"rid": req.rid, "arrival": req.arrival, "done": t_done, "iterations": req.iterations,
                        **(_final(job) if keep else {})})
        job.close()
    torch.cuda.synchronize()
    makespan = time_fn() - t0
    return _summary(lat, solves, makespan, work), records
