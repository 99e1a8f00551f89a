"""Write the full-size layered-skin oracle reference (tests/golden/c2_oracle_sample.npz).

Runs only the FP64 oracle on the full 160^3 / 64^3-hex / 2000-step layered-skin
workload with its true medium (float32-rounded, as the GPU receives it):
forward traces, then the adjoint and gradient for a seeded cotangent that the
GPU test regenerates from the same input generator.  Stores a seeded sample of
trace entries and gradient entries plus per-step trace norms and the gradient
norms, so the GPU result at full size can be compared without the full arrays.

Also stores the paper-formula variant of the eps gradient (eq. gradeps with the
grad(eps~).E term dropped) at the same sampled nodes, and its norm.

Usage: python tests/golden/make_c2_golden.py [n_steps [out_path]]   (about 80 min, 20 GB RAM)
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.discretization import Discretization  # noqa: E402
from oracle.solver import adjoint_gradient, forward  # noqa: E402

COT_SCALE = 1e-3
N_SAMPLE = 8192


def cotangent(shape, seed):
    return (COT_SCALE * synth.noise(shape, seed + 17)).astype(np.float32)


def main():
    n_steps = int(sys.argv[1]) if len(sys.argv) > 1 else 2000
    w = synth.c2(n_steps=n_steps)
    eps = w.eps_true.astype(np.float32).astype(np.float64)
    sig = w.sigma_true.astype(np.float32).astype(np.float64)
    t0 = time.time()
    d = Discretization(w.desc).set_coefficients(eps, sig)
    print(f"setup {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    fw = forward(d, w.sources[0])
    print(f"forward {time.time() - t0:.1f} s", flush=True)
    tr = fw["traces"]
    cot = cotangent(tr.shape, w.seed)
    t0 = time.time()
    ag = adjoint_gradient(d, cot.astype(np.float64), fw)
    print(f"adjoint {time.time() - t0:.1f} s", flush=True)
    rng = np.random.Generator(np.random.PCG64(w.seed + 99))
    ts = rng.integers(0, tr.shape[0], N_SAMPLE)
    ds = rng.integers(0, tr.shape[1], N_SAMPLE)
    free = np.nonzero(d.fem_free)[0]
    gs = np.sort(rng.choice(free, N_SAMPLE, replace=False))
    out = sys.argv[2] if len(sys.argv) > 2 else \
        os.path.join(os.path.dirname(os.path.abspath(__file__)), f"c2_oracle_sample_{n_steps}.npz")
    np.savez_compressed(
        out, n_steps=n_steps, t_idx=ts, d_idx=ds, traces=tr[ts, ds, :],
        trace_row_norm=np.sqrt(np.sum(tr * tr, axis=(1, 2))),
        g_idx=gs, g_eps=ag["g_eps"][gs], g_sigma=ag["g_sigma"][gs],
        g_eps_norm=np.linalg.norm(ag["g_eps"]), g_sigma_norm=np.linalg.norm(ag["g_sigma"]),
        g_eps_paper=ag["g_eps_paper"][gs], g_eps_paper_norm=np.linalg.norm(ag["g_eps_paper"]),
        energy=fw["energy"])
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
