"""Write the oracle reference of the streaming-regime case (tests/golden/s224_oracle_sample.npz).

Runs only the FP64 oracle on the 224^3 / 96^3-hex layered-skin case with one point dipole
above the FEM box (synth.stream224; its finite-difference fields exceed the last-level cache,
so the GPU runs its streaming tile variant there): forward traces and energy, then the
adjoint and gradient for the misfit J = 1/2 sum |T - E_obs|^2 with seeded synthetic
observations E_obs = OBS_SCALE * rms(T) * noise, which the GPU test regenerates from the
same input generator (the GPU forms T - E_obs inside its adjoint kernels).  Stores a seeded
sample of trace and free-node gradient entries, per-step trace norms, the gradient norms and
the energy history.

Usage: python tests/golden/make_s224_golden.py [n_steps [out_path]]   (about an hour, ~25 GB RAM)
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

OBS_SCALE = 0.3
N_SAMPLE = 8192


def observations(shape, seed, scale):
    """Seeded synthetic observations, float32 (the GPU test draws the same array)."""
    return (scale * synth.noise(shape, seed + 23)).astype(np.float32)


def main():
    n_steps = int(sys.argv[1]) if len(sys.argv) > 1 else 420
    w = synth.stream224(n_steps=n_steps)
    eps = w.eps_true.astype(np.float32).astype(np.float64)
    sig = w.sigma_true.astype(np.float32).astype(np.float64)
    t0 = time.time()
    d = Discretization(w.desc).set_coefficients(eps, sig)
    print(f"setup {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    fw = forward(d, w.sources[0])
    print(f"forward {time.time() - t0:.1f} s", flush=True)
    tr = fw["traces"]
    scale = OBS_SCALE * float(np.sqrt(np.mean(tr * tr)))
    obs = observations(tr.shape, w.seed, scale)
    cot = tr - obs.astype(np.float64)
    del fw["balance"]
    t0 = time.time()
    ag = adjoint_gradient(d, cot, fw)
    print(f"adjoint {time.time() - t0:.1f} s", flush=True)
    rng = np.random.Generator(np.random.PCG64(w.seed + 99))
    ts = rng.integers(0, tr.shape[0], N_SAMPLE)
    ds = rng.integers(0, tr.shape[1], N_SAMPLE)
    free = np.nonzero(d.fem_free)[0]
    gs = np.sort(rng.choice(free, N_SAMPLE, replace=False))
    out = sys.argv[2] if len(sys.argv) > 2 else \
        os.path.join(os.path.dirname(os.path.abspath(__file__)), f"s224_oracle_sample_{n_steps}.npz")
    np.savez_compressed(
        out, n_steps=n_steps, obs_scale=scale, t_idx=ts, d_idx=ds, traces=tr[ts, ds, :],
        trace_row_norm=np.sqrt(np.sum(tr * tr, axis=(1, 2))),
        g_idx=gs, g_eps=ag["g_eps"][gs], g_sigma=ag["g_sigma"][gs],
        g_eps_norm=np.linalg.norm(ag["g_eps"]), g_sigma_norm=np.linalg.norm(ag["g_sigma"]),
        energy=fw["energy"])
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
