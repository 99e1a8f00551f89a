"""Profiling helpers: copy-kernel calibration and rocprofv3 summaries.

  python -m paper_2508_07780_amd.profiling copy [MiB]        plain device copy of a known size
  python -m paper_2508_07780_amd.profiling stats CSV          kernel-trace stats -> markdown table
  python -m paper_2508_07780_amd.profiling pmc DIR COUNTER    average counter per dispatch per kernel
  python -m paper_2508_07780_amd.profiling hash [FILE ...]    hash of the step kernel sources (or of
                                                             the named files under csrc/)
  python -m paper_2508_07780_amd.profiling batch [STEPS]      two small mix problems batched, then alone
  python -m paper_2508_07780_amd.profiling grid DIR [GRID...]  kernel-trace durations per kernel and
                                                             grid size (only the given grid sizes)

The committed summaries under profiles/ record the HBM traffic of the fused step
kernel together with the hash of the kernel sources it was measured on; bench.py
only reports that traffic while the hash still matches.
"""

import collections
import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash(names=("kernels.hip", "dd_common.hpp")):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def copy_probe(mib=1024, reps=5):
    """Plain elementwise copy (one read and one write of `mib` MiB per dispatch)."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps} with an elementwise kernel", flush=True)


def batch_probe(steps=400):
    """Two small problems of the 16-problem mix (outer 112^3 / FEM 64^3 hexes, and 96^3 / 48^3),
    `steps` steps each, forward + misfit adjoint + gradient: first as one batch, whose steps
    share batched launches (batch_step_kernel), then one problem at a time (step_kernel), so
    that one kernel trace or counter run holds both."""
    import torch
    import synth
    from . import Problem
    from .batch import Batch
    mix = synth.batch_mix()
    ws = [synth.with_steps(mix[i], steps) for i in (2, 11)]

    def setup(w):
        p = Problem(w.desc)
        p.set_coefficients(torch.tensor(w.eps_true, dtype=torch.float32, device="cuda"),
                           torch.tensor(w.sigma_true, dtype=torch.float32, device="cuda"))
        obs = torch.zeros((len(w.sources), steps, p.n_det, 3), dtype=torch.float32, device="cuda")
        return p, obs

    probs = [setup(w) for w in ws]
    b = Batch(4)
    for (p, obs), w in zip(probs, ws):
        b.submit(p, w.sources, obs=obs)
    b.run_to_completion(chunk=64)
    torch.cuda.synchronize()
    b.close()
    print(f"batched: {[w.name for w in ws]}, {steps} steps", flush=True)
    for (p, obs), w in zip(probs, ws):
        tr = p.forward(w.sources, save=True)
        p.adjoint_misfit(tr, obs)
        p.gradient()
    torch.cuda.synchronize()
    print("one at a time", flush=True)
    for p, _ in probs:
        p.close()


def _rows(path_or_dir, suffix):
    files = [path_or_dir] if os.path.isfile(path_or_dir) else \
        glob.glob(os.path.join(path_or_dir, "**", "*" + suffix), recursive=True)
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _short(name):
    name = name.replace("(anonymous namespace)::", "").split("(")[0]
    return name.replace("void ", "").strip()


def stats_table(path):
    rows = _rows(path, "kernel_stats.csv")
    out = ["| kernel | calls | total ms | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append("| %s | %s | %.2f | %.2f | %.2f | %.2f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def grid_table(path, grids=()):
    """Average / min / max duration per (kernel, grid size) of a kernel trace: launches of one
    kernel on problems of different sizes apart."""
    dur = collections.defaultdict(list)
    for r in _rows(path, "kernel_trace.csv"):
        g = r["Grid_Size_X"]
        if grids and g not in grids:
            continue
        dur[(_short(r["Kernel_Name"]), g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| kernel | grid size (work-items) | calls | average us | min us | max us |", "|---|---|---|---|---|---|"]
    for (k, g), v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        out.append("| %s | %s | %d | %.2f | %.2f | %.2f |" % (k, g, len(v), sum(v) / len(v), min(v), max(v)))
    return "\n".join(out)


def pmc_average(path, counter, pattern=""):
    rows = _rows(path, "counter_collection.csv")
    tot = collections.defaultdict(float)
    cnt = collections.Counter()
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        k = _short(r.get("Kernel_Name", ""))
        if pattern and pattern not in k:
            continue
        tot[k] += float(r["Counter_Value"])
        cnt[k] += 1
    return {k: (tot[k] / cnt[k], cnt[k]) for k in tot}


def main(argv):
    if not argv:
        print(__doc__)
        return 1
    cmd = argv[0]
    if cmd == "copy":
        copy_probe(int(argv[1]) if len(argv) > 1 else 1024)
    elif cmd == "stats":
        print(stats_table(argv[1]))
    elif cmd == "pmc":
        for k, (v, n) in sorted(pmc_average(argv[1], argv[2], argv[3] if len(argv) > 3 else "").items()):
            print(f"{k}\t{argv[2]}\t{v:.1f}\tdispatches={n}")
    elif cmd == "hash":
        print(kernel_source_hash(argv[1:]) if len(argv) > 1 else kernel_source_hash())
    elif cmd == "grid":
        print(grid_table(argv[1], tuple(argv[2:])))
    elif cmd == "batch":
        batch_probe(int(argv[1]) if len(argv) > 1 else 400)
    else:
        print(__doc__)
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
