"""Request loop: continuous batching of reconstruction solves with HBM admission.

Jobs arrive over time.  Each job is a sequence of reconstruction iterations of one
problem (box "CGA": forward, misfit adjoint, eps/sigma gradient, then the conjugate
gradient update of eps and sigma on the device); the problem's fields stay resident
between its solves.  A job is admitted
when a batch slot is free and its device footprint (dd_footprint_bytes plus its trace,
observation and gradient buffers) fits in the HBM budget; admitted solves join the
running batch at the next launch, so work of jobs of different sizes overlaps on the
device.  A job whose single step already fills the GPU (at least `solo_cells` cells per
step) gains nothing from sharing launches and is slower through the batch kernel: it runs
through the single-problem calls instead, on a stream of its own, issued by a host thread of
its own, so that it overlaps the batch on the device; two such jobs run at a time by default
(two large solves side by side fill each other's launch tails), and jobs are admitted in
arrival order.  The one-at-a-time server runs the same jobs in arrival order through the
single-problem calls, for comparison.

The device never waits for the host at a job boundary: admission (mesh set-up, the first
coefficients, the CGA run's state) runs on the caller's stream, the batch and every solve on
a stream of their own; a finished solve's CGA update, its step sizes (from the first gradient)
and the new coefficients are queued on the batch's stream without a host read; a finished
job's device memory is released only once an event shows its last work done, and its
completion time is taken then.

Failures: a DDError while a job is created, submitted or updated releases its slot and
budget; the job is queued again from its start (once by default) or rejected, and the other
jobs go on.  A DDError from a batch step does the same for every job of that batch, which
is replaced by a new one.

Requests are plain objects with `arrival` (s), `iterations` and `workload` (desc, sources,
initial eps / sigma, seed; `workload.extra["obs"]`, when present, gives the observations as a
host array [n_src][n_steps][n_det][3]).  Otherwise observations are seeded synthetic data of the
traces' shape: the cost of a solve does not depend on their values.
"""

import threading
import time

import numpy as np
import torch

from ._lib import DDError
from .batch import Batch
from .cga import CGA, CGAParams
from .solver import Problem


# coefficient box of the reconstruction (eq. epsilon_sigma_constraint)
EPS_MAX, SIG_MAX = 20.0, 3.0
# the first update moves eps by at most STEP_EPS and sigma by at most STEP_SIG
STEP_EPS, STEP_SIG = 0.5, 0.1


def cell_steps(desc, n_src):
    """Cells (outer nodes + FEM-owned nodes) x (forward + adjoint steps) x sources of one solve."""
    n_own = int(np.prod([max(int(c) - 1, 0) for c in desc.fem_cells]))
    n_grid = int(np.prod([int(v) for v in desc.n_outer]))
    return (n_grid + n_own) * 2 * int(desc.n_steps) * n_src


class _Job:
    """A request's problem, iterate, observations and CGA run, set up on the current stream."""

    def __init__(self, req, dev):
        w = req.workload
        self.req = req
        self.problem = Problem(w.desc)
        self.eps = torch.tensor(w.eps, dtype=torch.float32, device=dev)
        self.sigma = torch.tensor(w.sigma, dtype=torch.float32, device=dev)
        shape = (len(w.sources), w.desc.n_steps, self.problem.n_det, 3)
        obs = w.extra.get("obs") if isinstance(getattr(w, "extra", None), dict) else None
        if obs is not None:
            self.obs = torch.tensor(np.asarray(obs, dtype=np.float32).reshape(shape), device=dev)
        else:
            g = torch.Generator(device=dev)
            g.manual_seed(int(w.seed))
            self.obs = 1e-3 * torch.randn(shape, generator=g, device=dev, dtype=torch.float32)
        self.done_iters = 0
        self.footprint = 0
        self.problem.set_coefficients(self.eps, self.sigma)
        # the run's step sizes come from the first gradient (steps_from_gradient); these
        # placeholders are replaced before the first update
        prm = CGAParams(gamma_eps=1.0, gamma_sig=1.0, p=0.5, alpha_eps=0.0, alpha_sig=0.0, eps_max=EPS_MAX,
                        sig_max=SIG_MAX)
        self.cga = CGA(self.problem, w.sources, self.obs, self.eps, self.sigma, prm)
        self.updates = 0

    def update(self, g_eps, g_sigma):
        """CGA steps 2-6 and the next coefficients, queued on the current stream (no host read)."""
        if self.updates == 0:
            self.cga.steps_from_gradient(g_eps, g_sigma, STEP_EPS, STEP_SIG)
        self.cga.update(g_eps, g_sigma)
        self.problem.set_coefficients(self.cga.eps, self.cga.sigma, wait=False)
        self.updates += 1

    def close(self):
        self.cga.close()
        self.problem.close()


def job_footprint(req):
    w = req.workload
    n_src = len(w.sources)
    traces = n_src * int(w.desc.n_steps) * _n_det(w.desc) * 3 * 4
    # the problem (its CGA run included), traces and observations, gradients (FP64), the
    # iterate (float32) and the run's copy of it
    return Problem.footprint_bytes(w.desc, n_src) + 2 * traces + (16 + 8 + 8) * w.desc.n_fem_nodes()


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
    """All iterations of one job through the single-problem calls (queued on the current stream)."""
    req = job.req
    for _ in range(req.iterations):
        tr = job.problem.forward(req.workload.sources, save=True)
        job.problem.adjoint_misfit(tr, job.obs)
        ge, gs = job.problem.gradient()
        job.update(ge, gs)
        job.done_iters += 1


class _Finisher:
    """Jobs whose last work is queued.  A job's completion time is that of an event recorded
    after its last work (device clock, against an event recorded at the start of the run);
    once the event has completed (polled, never waited for in the loop) the job's device memory
    is released and `release(job)` is called."""

    def __init__(self, t0, keep, release=None):
        torch.cuda.synchronize()
        self.t0 = t0
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev0.record(torch.cuda.current_stream())
        self.keep, self.release = keep, release
        self.items = []
        self.lat, self.records = [], []

    def add(self, job, stream):
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        self.items.append((ev, job))

    def sweep(self, wait=False):
        left = []
        for ev, job in self.items:
            if wait:
                ev.synchronize()
            if ev.query():
                t_done = self.ev0.elapsed_time(ev) / 1e3
                req = job.req
                self.lat.append(t_done - req.arrival)
                self.records.append({"rid": req.rid, "arrival": req.arrival, "done": t_done,
                                     "iterations": job.done_iters, **(_final(job) if self.keep else {})})
                job.close()
                if self.release is not None:
                    self.release(job)
            else:
                left.append((ev, job))
        self.items = left

    def __len__(self):
        return len(self.items)


def serve_batched(requests, max_slots=16, hbm_budget=None, chunk=256, time_fn=time.perf_counter, keep=False,
                  solo_cells=3_000_000, fill_cells=None, retries=1, solo_overlap=True, solo_slots=2):
    """Continuous batching: returns a summary dict and per-job records (with each job's final
    eps and sigma when keep is set).  Jobs of at least solo_cells cells per step run through
    the single-problem calls (None: every job is batched): beside the batch on a stream and a
    host thread of their own (solo_overlap; up to solo_slots such jobs at once, each on its
    own stream), or alone once the batch has drained.
    fill_cells: the batch's fill target per launch (None: the library's default).  retries:
    how often a failed job is queued again before it is rejected."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if hbm_budget is None:
        free, _ = torch.cuda.mem_get_info()
        hbm_budget = int(0.9 * free)
    pending = sorted(requests, key=lambda r: r.arrival)
    admit = torch.cuda.current_stream()
    run = torch.cuda.Stream(device=dev)
    if not solo_overlap:
        solo_slots = 1
    slots = [{"stream": torch.cuda.Stream(device=dev) if solo_overlap else run, "thread": None, "job": None,
              "error": None} for _ in range(solo_slots)]
    batch = Batch(max_slots, fill_cells=fill_cells)
    active = {}           # job id in the batch -> _Job
    in_use = 0
    failures = {}         # rid -> failed attempts
    rejected = []
    solves = 0
    work = 0
    peak_bytes = peak_jobs = 0
    torch.cuda.synchronize()
    t0 = time_fn()

    def release(job):
        nonlocal in_use
        in_use -= job.footprint

    fin = _Finisher(t0, keep, release)

    def fail(req, job, err, stream=None):
        """Release the job's slot and budget, then queue it again or reject it."""
        nonlocal in_use
        if job is not None:
            in_use -= job.footprint
            fin_ev = torch.cuda.Event()
            fin_ev.record(run if stream is None else stream)
            fin_ev.synchronize()            # nothing of it may still run when its memory goes
            job.close()
        n = failures.get(req.rid, 0) + 1
        failures[req.rid] = n
        if n <= retries:
            pending.append(req)
            pending.sort(key=lambda r: r.arrival)
        else:
            rejected.append({"rid": req.rid, "arrival": req.arrival, "error": str(err)})

    def solo_worker(slot, job):
        try:
            with torch.cuda.stream(slot["stream"]):
                _run_alone(job)
        except DDError as e:
            slot["error"] = e

    def solo_finished():
        """Account for each thread's job once its launches are all issued."""
        nonlocal solves, work
        for slot in slots:
            th, job = slot["thread"], slot["job"]
            if th is None or th.is_alive():
                continue
            th.join()
            slot["thread"] = slot["job"] = None
            if slot["error"] is not None:
                err, slot["error"] = slot["error"], None
                fail(job.req, job, err, slot["stream"])
                continue
            solves += job.req.iterations
            work += cell_steps(job.req.workload.desc, len(job.req.workload.sources)) * job.req.iterations
            fin.add(job, slot["stream"])

    def solo_busy():
        return [sl for sl in slots if sl["thread"] is not None]

    while pending or active or solo_busy():
        fin.sweep()
        solo_finished()
        now = time_fn() - t0
        # admission: arrived, a slot free, the footprint fits
        while pending and pending[0].arrival <= now and len(active) < max_slots:
            fp = job_footprint(pending[0])
            if fp > hbm_budget:
                raise ValueError(f"request {pending[0].rid} needs {fp} bytes, over the HBM budget of {hbm_budget}")
            alone = solo_cells is not None and step_cells(pending[0].workload.desc) >= solo_cells
            free_slot = next((sl for sl in slots if sl["thread"] is None), None)
            if alone and (free_slot is None or (active and not solo_overlap)):
                break                    # solo_slots such jobs at a time (arrival order is kept)
            if in_use + fp > hbm_budget:
                break                    # room comes back as finished jobs are released
            req = pending.pop(0)
            try:
                job = _Job(req, dev)
            except DDError as e:
                fail(req, None, e)
                continue
            job.footprint = fp
            in_use += fp
            peak_bytes = max(peak_bytes, in_use)
            if alone:
                peak_jobs = max(peak_jobs, len(active) + len(solo_busy()) + 1)
                free_slot["stream"].wait_stream(admit)
                free_slot["job"] = job
                free_slot["thread"] = threading.Thread(target=solo_worker, args=(free_slot, job), daemon=True)
                free_slot["thread"].start()
                if not solo_overlap:
                    free_slot["thread"].join()
                    solo_finished()
                now = time_fn() - t0
                continue
            try:
                run.wait_stream(admit)
                with torch.cuda.stream(run):
                    jid = batch.submit(job.problem, req.workload.sources, obs=job.obs)
            except DDError as e:
                fail(req, job, e)
                continue
            active[jid] = job
            peak_jobs = max(peak_jobs, len(active))
        if not active:
            busy = solo_busy()
            if not pending and not busy:
                break            # the last jobs ran alone
            # idle until the next arrival, until finished jobs free room, or until a job
            # beside the batch has issued its work
            wait = 0.01 if not pending else min(0.01, pending[0].arrival - now)
            if busy:
                busy[0]["thread"].join(timeout=max(0.0005, wait))
            else:
                time.sleep(max(0.0005, wait))
            continue
        try:
            with torch.cuda.stream(run):
                batch.step(chunk)
        except DDError as e:
            # the batch's state is unknown: every job in it starts again (or is rejected)
            for j in list(active.values()):
                fail(j.req, j, e)
            active.clear()
            batch.close()
            batch = Batch(max_slots, fill_cells=fill_cells)
            continue
        finished, _ = batch.poll()
        for rec in finished:
            job = active.pop(rec["id"])
            try:
                with torch.cuda.stream(run):
                    job.update(rec["g_eps"], rec["g_sigma"])
                    solves += 1
                    work += cell_steps(job.req.workload.desc, len(job.req.workload.sources))
                    job.done_iters += 1
                    if job.done_iters < job.req.iterations:
                        jid = batch.submit(job.problem, job.req.workload.sources, obs=job.obs)
                        active[jid] = job
                        continue
            except DDError as e:
                fail(job.req, job, e)
                continue
            fin.add(job, run)
    run.synchronize()
    for sl in slots:
        sl["stream"].synchronize()
    fin.sweep(wait=True)
    makespan = time_fn() - t0
    batch.close()
    out = _summary(fin.lat, solves, makespan, work)
    out.update(hbm_budget_bytes=hbm_budget, peak_admitted_bytes=peak_bytes, peak_concurrent_jobs=peak_jobs,
               rejected=len(rejected), retried=sum(1 for n in failures.values() if n >= 1) - len(rejected),
               in_use_end_bytes=in_use)
    records = fin.records + [dict(r, rejected=True) for r in rejected]
    return out, records


def serve_serial(requests, time_fn=time.perf_counter, keep=False):
    """One solve at a time, jobs in arrival order, through the single-problem calls."""
    dev = torch.device("cuda", torch.cuda.current_device())
    solves = 0
    work = 0
    torch.cuda.synchronize()
    t0 = time_fn()
    fin = _Finisher(t0, keep)
    for req in sorted(requests, key=lambda r: r.arrival):
        now = time_fn() - t0
        if req.arrival > now:
            fin.sweep()
            time.sleep(req.arrival - now)
        job = _Job(req, dev)
        _run_alone(job)
        solves += req.iterations
        work += cell_steps(req.workload.desc, len(req.workload.sources)) * req.iterations
        fin.add(job, torch.cuda.current_stream())
        fin.sweep()
    torch.cuda.synchronize()
    fin.sweep(wait=True)
    makespan = time_fn() - t0
    return _summary(fin.lat, solves, makespan, work), fin.records
