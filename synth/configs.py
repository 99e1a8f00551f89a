"""Problem descriptions and seeded media for the hybrid FE/FD Maxwell solver.

Geometry follows the model problem of the paper's numerical section: a box
shaped outer domain discretised by a structured grid, with a cube of
tetrahedral finite elements inside it (Fig. "meshes", section "Numerical
results").  All lengths are in units where the FEM cube side is 1 (the paper's
10 mm cube), except for the first configuration, whose geometry is given
explicitly.

Conventions used everywhere in this repository:

* Outer-grid node (i, j, k) sits at origin + h * (i, j, k); arrays over the
  outer grid are in lexicographic order with x fastest.
* The FEM box covers hex cells [fem_lo, fem_lo + fem_cells) of the outer
  grid; its nodes have local indices l in [0, fem_cells] per axis and arrays
  over them (eps, sigma, gradients) are lexicographic with x fastest.
* A FEM node's layer is min over axes of min(l, fem_cells - l).  Layer 0 is
  owned by the finite-difference region, layer 1 is the first FEM-owned layer
  and layers >= 2 are free (eps and sigma may differ from 1 and 0 there).
* Face bits: top (z max, the paper's backscatter boundary) = 1,
  bottom (z min) = 2, x min = 4, x max = 8, y min = 16, y max = 32.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

FACE_TOP = 1
FACE_BOTTOM = 2
FACE_XMIN = 4
FACE_XMAX = 8
FACE_YMIN = 16
FACE_YMAX = 32
FACE_ALL = 63

SRC_SINE1 = 1       # one period of sin(omega t) (paper eq. "f")
SRC_GAUSS_SINE = 2  # Gaussian-modulated sine
SRC_DIPOLE = 3      # point dipole at a node (time function as GAUSS_SINE)

SEED_BASE = 2508077800


@dataclass
class ProblemDesc:
    n_outer: tuple          # outer grid nodes per axis (Nx, Ny, Nz)
    h: float                # grid spacing
    origin: tuple           # coordinates of node (0, 0, 0)
    fem_lo: tuple           # outer-grid index of the FEM box's lower corner node
    fem_cells: tuple        # hex cells of the FEM box per axis
    dt: float               # time step (fixed input, never derived from eps)
    n_steps: int            # number of time steps N_t
    ckpt_every: int = 64    # forward checkpoint interval K for the adjoint
    detector_faces: int = FACE_TOP
    absorbing_faces: int = FACE_TOP | FACE_BOTTOM
    t_switch: float = 0.0   # top face: source for t <= t_switch, absorbing after
    overlap: int = 2        # node layers shared by the FD and FEM regions
    s_stab: float = 1.0     # weight of the div-div stabiliser
    ckpt_mode: int = 0      # 0: FEM checkpoints + interface history, 1: every level kept

    def fem_shape(self):
        return tuple(int(c) + 1 for c in self.fem_cells)

    def n_fem_nodes(self):
        s = self.fem_shape()
        return s[0] * s[1] * s[2]

    def n_grid(self):
        return int(self.n_outer[0]) * int(self.n_outer[1]) * int(self.n_outer[2])

    def n_fem_owned(self):
        return int(np.prod([max(int(c) - 1, 0) for c in self.fem_cells]))

    def validate(self):
        for a in range(3):
            n, lo, c = int(self.n_outer[a]), int(self.fem_lo[a]), int(self.fem_cells[a])
            if n < 4:
                raise ValueError("outer grid needs at least 4 nodes per axis")
            if c < 2:
                raise ValueError("FEM box needs at least 2 cells per axis")
            if lo < 1 or lo + c > n - 2:
                raise ValueError("FEM box must sit strictly inside the outer grid")
        if not (self.h > 0 and self.dt > 0 and self.n_steps >= 0):
            raise ValueError("h, dt must be positive and n_steps non-negative")
        return self


@dataclass
class Source:
    kind: int
    omega: float
    t0: float = 0.0
    width: float = 0.0
    amp: float = 1.0
    pol: tuple = (0.0, 1.0, 0.0)
    pos: tuple = (0, 0, 0)   # dipole: outer-grid node index
    dir: tuple = (0.0, 0.0, 0.0)   # plane wave: direction of travel (zero: normal incidence, -z)

    def support_end(self):
        """End of the pulse's time support (used as the top-face switch time)."""
        if self.kind == SRC_SINE1:
            return 2.0 * math.pi / self.omega
        return 2.0 * self.t0


@dataclass
class Workload:
    name: str
    desc: ProblemDesc
    eps: np.ndarray             # current model, FEM lattice, float64
    sigma: np.ndarray
    sources: List[Source]
    seed: int
    eps_true: Optional[np.ndarray] = None   # model that generates observed data
    sigma_true: Optional[np.ndarray] = None
    noise_level: float = 0.0
    extra: dict = field(default_factory=dict)


def gauss_sine(omega, amp=1.0, pol=(0.0, 1.0, 0.0)):
    tp = 2.0 * math.pi / omega
    return Source(kind=SRC_GAUSS_SINE, omega=omega, t0=1.5 * tp, width=0.5 * tp, amp=amp, pol=pol)


def oblique_wave(omega, theta, phi, psi=0.0, amp=1.0):
    """Gaussian-modulated sine plane wave travelling along k = (sin theta cos phi, sin theta sin phi,
    -cos theta) (theta from the downward normal of the top face), polarised perpendicular to k
    at the angle psi from the incidence plane."""
    k = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), -math.cos(theta)])
    e_perp = np.array([-math.sin(phi), math.cos(phi), 0.0])        # perpendicular to the incidence plane
    e_par = np.cross(e_perp, k)                                     # in the incidence plane, perpendicular to k
    pol = math.cos(psi) * e_par + math.sin(psi) * e_perp
    src = gauss_sine(omega, amp=amp, pol=tuple(float(v) for v in pol))
    src.dir = tuple(float(v) for v in k)
    return src


def plane_wave_switch(desc: ProblemDesc, src: Source) -> float:
    """Top-face switch time that keeps a plane-wave source on until it has crossed the whole face:
    the pulse's support plus the largest arrival delay over the top face."""
    v = np.asarray(src.dir, dtype=np.float64)
    nv = float(np.linalg.norm(v))
    tau = 0.0
    if nv > 0:
        k = v / nv
        span = desc.h * (np.asarray(desc.n_outer[:2], dtype=np.float64) - 1.0)
        tau = float(abs(k[0]) * span[0] + abs(k[1]) * span[1])
    return src.support_end() + tau


def fem_layers(desc: ProblemDesc) -> np.ndarray:
    """Layer index of every FEM node (lexicographic, x fastest)."""
    nx, ny, nz = desc.fem_shape()
    cx, cy, cz = desc.fem_cells
    lz, ly, lx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lay = np.minimum(np.minimum(lx, cx - lx), np.minimum(ly, cy - ly))
    lay = np.minimum(lay, np.minimum(lz, cz - lz))
    return lay.reshape(-1)


def fem_node_coords(desc: ProblemDesc) -> np.ndarray:
    nx, ny, nz = desc.fem_shape()
    lz, ly, lx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = np.stack([lx, ly, lz], axis=-1).reshape(-1, 3) + np.asarray(desc.fem_lo)
    return np.asarray(desc.origin, dtype=np.float64) + desc.h * idx


def _centered_desc(n_outer, n_f, n_steps, detector_faces=FACE_TOP, ckpt_every=64):
    """Cube FEM box of n_f cells centred in an n_outer^3 grid, FEM side = 1."""
    h = 1.0 / n_f
    lo = (n_outer - 1 - n_f) // 2
    origin = (-lo * h,) * 3
    return ProblemDesc(n_outer=(n_outer,) * 3, h=h, origin=origin, fem_lo=(lo,) * 3,
                       fem_cells=(n_f,) * 3, dt=0.5 * h / math.sqrt(3.0), n_steps=n_steps,
                       ckpt_every=ckpt_every, detector_faces=detector_faces)


def _free_mask(desc):
    return fem_layers(desc) >= 2


def sphere_media(desc, rng, radius, eps_in, sig_in, centre_range):
    """eps = 1 background plus a sphere; nodal sampling restricted to free nodes."""
    x = fem_node_coords(desc)
    c = np.asarray(desc.origin) + desc.h * (np.asarray(desc.fem_lo) + 0.5 * np.asarray(desc.fem_cells))
    c = c + rng.uniform(-centre_range, centre_range, size=3)
    inside = (np.sum((x - c) ** 2, axis=1) <= radius ** 2) & _free_mask(desc)
    eps = np.ones(len(x))
    sig = np.zeros(len(x))
    eps[inside] = eps_in
    sig[inside] = sig_in
    return eps, sig, c


def skin_media(desc, rng):
    """Layered skin with an ellipsoidal melanoma on the free FEM nodes.

    Layers (from the top of the free region down): epidermis (at least one node
    layer, 0.1 mm), dermis 3.5 mm, fat to the bottom; 1 mm = 0.1 length units.
    Values follow the test column of the paper's Table 1 in spirit: tissue
    sigma = 0, tumour eps 1.5-2.5x the dermis value and sigma in [0, 3].
    """
    x = fem_node_coords(desc)
    free = _free_mask(desc)
    h = desc.h
    nzc = desc.fem_cells[2]
    z_top_free = desc.origin[2] + h * (desc.fem_lo[2] + nzc - 2)
    depth = z_top_free - x[:, 2]
    n_epi = max(1, int(round(0.01 / h)))
    n_derm = max(1, int(round(0.35 / h)))
    eps_epi = rng.uniform(3.0, 5.0)
    eps_derm = rng.uniform(4.0, 8.0)
    eps_fat = rng.uniform(1.5, 2.5)
    tol = 1e-9 * h
    eps = np.ones(len(x))
    sig = np.zeros(len(x))
    epi = depth < n_epi * h - tol
    derm = (~epi) & (depth < (n_epi + n_derm) * h - tol)
    fat = ~(epi | derm)
    eps[epi] = eps_epi
    eps[derm] = eps_derm
    eps[fat] = eps_fat
    # ellipsoid: semi-axes (a, a, c), top touching the epidermis/dermis interface
    a = rng.uniform(0.1, 0.2)
    cz_ = rng.uniform(0.05, 0.15)
    lo = np.asarray(desc.origin) + h * np.asarray(desc.fem_lo)
    side = h * np.asarray(desc.fem_cells)
    cxy = lo[:2] + side[:2] * rng.uniform(0.25, 0.75, size=2)
    z_int = z_top_free - n_epi * h
    centre = np.array([cxy[0], cxy[1], z_int - cz_])
    r2 = ((x[:, 0] - centre[0]) / a) ** 2 + ((x[:, 1] - centre[1]) / a) ** 2 + ((x[:, 2] - centre[2]) / cz_) ** 2
    tum = (r2 <= 1.0) & (~epi)
    eps_tum = rng.uniform(1.5, 2.5) * eps_derm
    sig_tum = rng.uniform(0.0, 3.0)
    eps[tum] = eps_tum
    sig[tum] = sig_tum
    eps[~free] = 1.0
    sig[~free] = 0.0
    info = dict(eps_epi=eps_epi, eps_derm=eps_derm, eps_fat=eps_fat, eps_tum=eps_tum,
                sig_tum=sig_tum, semi_axes=(a, a, cz_), centre=tuple(centre))
    return eps, sig, info


def random_media(desc, rng, eps_max=5.0, sig_max=1.0):
    """Smooth-ish random media on free nodes (parity tests on small grids)."""
    x = fem_node_coords(desc)
    free = _free_mask(desc)
    k = rng.normal(size=(4, 3)) * (2.0 / (desc.h * max(desc.fem_cells)))
    ph = rng.uniform(0, 2 * np.pi, size=4)
    f = sum(np.sin(x @ k[i] + ph[i]) for i in range(4)) / 4.0
    g = rng.uniform(0, 1, size=len(x))
    eps = 1.0 + (eps_max - 1.0) * (0.5 + 0.5 * f) * (0.6 + 0.4 * g)
    sig = sig_max * (0.5 + 0.5 * np.cos(3 * f)) * g
    eps[~free] = 1.0
    sig[~free] = 0.0
    return eps, sig


def initial_pulses(desc: ProblemDesc, seed: int, n_pulses: int = 3):
    """Seeded smooth initial data (f_0, f_1) over the whole grid, each (N, 3), node index
    x + Nx (y + Ny z): sums of Gaussian bumps of width 3h..6h with random centres (inside the
    grid, several within the FEM box) and random polarisations; f_1 has its own bumps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = (int(v) for v in desc.n_outer)
    lz, ly, lx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([lx, ly, lz], axis=-1).reshape(-1, 3).astype(np.float64)
    lo = np.asarray(desc.fem_lo, dtype=np.float64)
    hi = lo + np.asarray(desc.fem_cells, dtype=np.float64)
    out = []
    for _ in range(2):
        f = np.zeros((pts.shape[0], 3))
        for b in range(n_pulses):
            if b % 2 == 0:
                c = rng.uniform(lo, hi)
            else:
                c = rng.uniform(0.0, 1.0, 3) * (np.array([nx, ny, nz]) - 1.0)
            w = rng.uniform(3.0, 6.0)
            pol = rng.standard_normal(3)
            r2 = np.sum((pts - c) ** 2, axis=1)
            f += np.exp(-0.5 * r2 / (w * w))[:, None] * pol[None, :]
        out.append(f)
    return out[0], out[1]


def noise(shape, seed):
    """Standard normal noise, PCG64 seeded."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)


def c1() -> Workload:
    """Plain forward solve: 25^3 nodes, h = 0.02 on [-0.24, 0.24]^3, 8^3 FEM hexes."""
    seed = SEED_BASE + 1
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 0.02
    desc = ProblemDesc(n_outer=(25, 25, 25), h=h, origin=(-0.24,) * 3, fem_lo=(8, 8, 8),
                       fem_cells=(8, 8, 8), dt=0.5 * h / math.sqrt(3.0), n_steps=300,
                       ckpt_every=64, detector_faces=FACE_ALL)
    src = gauss_sine(17.56)
    desc.t_switch = src.support_end()
    eps, sig, _ = sphere_media(desc, rng, 0.05, 4.0, 0.5, 0.02)
    return Workload("c1", desc, eps, sig, [src], seed, eps_true=eps, sigma_true=sig)


def _skin_workload(name, cfg_no, n_outer, n_f, n_steps, ckpt_every=64):
    seed = SEED_BASE + cfg_no
    rng = np.random.Generator(np.random.PCG64(seed))
    desc = _centered_desc(n_outer, n_f, n_steps, ckpt_every=ckpt_every)
    src = gauss_sine(2.0 * math.pi / 2.236)
    desc.t_switch = src.support_end()
    eps_t, sig_t, info = skin_media(desc, rng)
    n = desc.n_fem_nodes()
    return Workload(name, desc, np.ones(n), np.zeros(n), [src], seed,
                    eps_true=eps_t, sigma_true=sig_t, noise_level=0.03, extra=info)


def c2(n_steps=2000) -> Workload:
    """Layered skin, 160^3 outer nodes, 64^3 FEM hexes, 2000 steps."""
    return _skin_workload("c2", 2, 160, 64, n_steps)


def c3(n_steps=1500) -> Workload:
    """Differentiation case: 192^3 outer nodes, 96^3 FEM hexes, 1500 steps, K = 64."""
    return _skin_workload("c3", 3, 192, 96, n_steps, ckpt_every=64)


def probe288(n_steps=300) -> Workload:
    """Bandwidth probe: the layered-skin generator on a 288^3 outer grid (96^3 FEM hexes),
    whose per-step field set (E twice and V, 860 MB) exceeds the 256 MB last-level cache."""
    return _skin_workload("probe288", 6, 288, 96, n_steps, ckpt_every=n_steps)


_SMALL = {
    # name: (n_outer, h, fem_lo, fem_cells, n_steps, detector faces, ckpt_every)
    "tiny": ((12, 11, 13), 0.05, (3, 3, 4), (5, 4, 5), 40, FACE_ALL, 8),
    "ragged": ((37, 35, 41), 0.03, (11, 12, 13), (12, 10, 14), 120, FACE_TOP | FACE_XMIN | FACE_YMAX, 16),
    "skinlet": ((48, 48, 48), 1.0 / 24, (12, 12, 12), (24, 24, 24), 160, FACE_TOP, 32),
}


def small(name: str, seed_offset: int = 0) -> Workload:
    """Small parity cases the oracle finishes in seconds; several tiles, ragged tails."""
    n_outer, h, lo, cells, nt, det, ck = _SMALL[name]
    seed = SEED_BASE + 100 + sorted(_SMALL).index(name) + 1000 * seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    desc = ProblemDesc(n_outer=n_outer, h=h, origin=(-0.5 * h * (n_outer[0] - 1),) * 3,
                       fem_lo=lo, fem_cells=cells, dt=0.5 * h / math.sqrt(3.0), n_steps=nt,
                       ckpt_every=ck, detector_faces=det)
    omega = 2.0 * math.pi / (12.0 * h)
    src = gauss_sine(omega, pol=(0.3, 1.0, -0.2))
    desc.t_switch = src.support_end()
    if name == "skinlet":
        eps, sig, _ = skin_media(desc, rng)
    else:
        eps, sig = random_media(desc, rng)
    return Workload(name, desc, eps, sig, [src], seed, eps_true=eps, sigma_true=sig)


def aligned_box(n_steps=96, ckpt_every=16, seed=SEED_BASE + 8) -> Workload:
    """A grid whose FEM box starts on a 32-node boundary in x and on 16-node boundaries in y and
    z (outer 64 x 40 x 41, box 16 x 12 x 12 cells at (32, 16, 16)), random media: the finite-
    difference tiles next to the box end one node short of its faces."""
    h = 0.03
    n_outer = (64, 40, 41)
    desc = ProblemDesc(n_outer=n_outer, h=h, origin=(-0.5 * h * (n_outer[0] - 1),) * 3, fem_lo=(32, 16, 16),
                       fem_cells=(16, 12, 12), dt=0.5 * h / math.sqrt(3.0), n_steps=n_steps, ckpt_every=ckpt_every,
                       detector_faces=FACE_TOP | FACE_XMIN | FACE_YMAX)
    src = gauss_sine(2.0 * math.pi / (12.0 * h), pol=(0.3, 1.0, -0.2))
    desc.t_switch = src.support_end()
    rng = np.random.Generator(np.random.PCG64(seed))
    eps, sig = random_media(desc, rng)
    return Workload("aligned", desc, eps, sig, [src], seed, eps_true=eps, sigma_true=sig)


def batch_mix(n_problems=16, seed=SEED_BASE + 4, ckpt_every=64):
    """Uneven multi-problem mix: outer 96..224 nodes, FEM 32..96 cells (valid pairs), 1000-2500
    steps, layered-skin media; even problems get a plane wave of seeded incidence (theta ~
    U[0, 30] degrees from the downward normal, phi ~ U[0, 360)) polarised perpendicular to its
    direction, the top face switching once it has crossed the face; odd ones a point dipole of
    seeded moment 4 nodes above the FEM box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for p in range(n_problems):
        while True:
            no = int(rng.choice(np.arange(96, 225, 16)))
            nf = int(rng.choice([32, 48, 64, 80, 96]))
            if no >= nf + 2 * max(8, math.ceil(0.2 * nf)):
                break
        nt = int(rng.integers(1000, 2501))
        desc = _centered_desc(no, nf, nt, ckpt_every=ckpt_every)
        base = gauss_sine(2.0 * math.pi / 2.236)
        desc.t_switch = base.support_end()
        v = rng.normal(size=3)
        v = tuple(v / np.linalg.norm(v))
        if p % 2 == 0:
            theta, phi, psi = rng.uniform(0.0, math.pi / 6), rng.uniform(0.0, 2 * math.pi), rng.uniform(0, math.pi)
            src = oblique_wave(base.omega, theta, phi, psi)
            desc.t_switch = plane_wave_switch(desc, src)
        else:
            src = Source(kind=SRC_DIPOLE, omega=base.omega, t0=base.t0, width=base.width, pol=v,
                         pos=(no // 2, no // 2, desc.fem_lo[2] + nf + 4))
        eps, sig, _ = skin_media(desc, rng)
        out.append(Workload(f"mix{p}", desc, eps, sig, [src], seed + p, eps_true=eps, sigma_true=sig))
    return out


def with_steps(w: Workload, n_steps: int) -> Workload:
    return replace(w, desc=replace(w.desc, n_steps=n_steps))


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    workload: Workload
    iterations: int         # reconstruction iterations of the job (solve, update, solve, ...)


def serving_requests(n_requests, rate, seed=SEED_BASE + 5, outer=(64, 96, 128, 160, 224),
                     fem=(32, 48, 64, 96), sources=(1, 8), steps=(500, 2000), iterations=(3, 10)):
    """Poisson arrivals (rate per second) of reconstruction jobs of uneven size.

    Each job draws an outer grid and a FEM box (valid pairs: outer >= fem + 2 max(8, 0.2 fem)),
    1-8 sources (plane waves of varying polarisation, every third one a point dipole above
    the FEM box), a step count and a number of iterations; media from the layered-skin
    generator.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        while True:
            no = int(rng.choice(outer))
            nf = int(rng.choice(fem))
            if no >= nf + 2 * max(8, math.ceil(0.2 * nf)):
                break
        nt = int(rng.integers(steps[0], steps[1] + 1))
        desc = _centered_desc(no, nf, nt)
        base = gauss_sine(2.0 * math.pi / 2.236)
        desc.t_switch = base.support_end()
        srcs = []
        for k in range(int(rng.integers(sources[0], sources[1] + 1))):
            pol = tuple(rng.normal(size=3) * np.array([1.0, 1.0, 0.2]))
            if k % 3 == 2:
                z = min(no - 2, desc.fem_lo[2] + nf + 4)
                srcs.append(Source(kind=SRC_DIPOLE, omega=base.omega, t0=base.t0, width=base.width,
                                   pol=pol, pos=(no // 2, no // 2, z)))
            else:
                srcs.append(gauss_sine(base.omega, pol=pol))
        eps, sig, _ = skin_media(desc, rng)
        n = desc.n_fem_nodes()
        w = Workload(f"req{r}", desc, np.ones(n), np.zeros(n), srcs, seed + 1000 + r,
                     eps_true=eps, sigma_true=sig, noise_level=0.03)
        out.append(Request(r, t, w, int(rng.integers(iterations[0], iterations[1] + 1))))
    return out


def stream224(n_steps=420) -> Workload:
    """Streaming-regime parity case: the layered-skin generator on a 224^3 outer grid with a
    96^3-hex FEM box, whose two levels of E (270 MB) exceed the 256 MB last-level cache, so the
    finite-difference tiles take their streaming variant by default.  One point dipole of seeded
    moment 4 nodes above the FEM box with a short pulse (period 16 h), so that within a few
    hundred steps the wave reaches both the FEM box and the top-face detectors; K = 64."""
    seed = SEED_BASE + 7
    rng = np.random.Generator(np.random.PCG64(seed))
    desc = _centered_desc(224, 96, n_steps, ckpt_every=64)
    h = desc.h
    base = gauss_sine(2.0 * math.pi / (16.0 * h))
    desc.t_switch = base.support_end()
    v = rng.normal(size=3)
    v = tuple(v / np.linalg.norm(v))
    src = Source(kind=SRC_DIPOLE, omega=base.omega, t0=base.t0, width=base.width, pol=v,
                 pos=(112, 100, desc.fem_lo[2] + 96 + 4))
    eps, sig, info = skin_media(desc, rng)
    return Workload("stream224", desc, eps, sig, [src], seed, eps_true=eps, sigma_true=sig, extra=info)


def meshref_marks(desc: ProblemDesc, eps: np.ndarray, beta: float) -> np.ndarray:
    """Cells of the FEM box (lexicographic, x fastest) marked for refinement by the rule of the
    paper's eq. meshref on the uniform starting mesh: |h eps| >= beta max |h eps| at any of the
    cell's corners (h the same everywhere, so the rule compares |eps|), among cells whose corners
    are all FEM-owned (layer >= 1), so that the overlap layers keep their lattice elements."""
    cx, cy, cz = (int(c) for c in desc.fem_cells)
    fx, fy = cx + 1, cy + 1
    e = np.abs(np.asarray(eps, dtype=np.float64))
    lay = fem_layers(desc)
    thr = beta * e.max()
    marks = np.zeros(cx * cy * cz, dtype=bool)
    for k in range(cz):
        for j in range(cy):
            for i in range(cx):
                corners = [(i + a) + fx * ((j + b) + fy * (k + c)) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                if lay[corners].min() >= 1 and e[corners].max() >= thr:
                    marks[i + cx * (j + cy * k)] = True
    return marks


def refined_mesh(desc: ProblemDesc, marks: np.ndarray):
    """A conforming tetrahedral mesh of the FEM box: the Kuhn split (six tetrahedra per cell, one per
    axis permutation, from the cell's lowest corner to its highest), where every marked cell gets
    its centre as a new node and each of its six tetrahedra is bisected across the cell's main
    diagonal into two (the cell's faces are not split, so neighbours stay conforming).  Returns
    (extra_xyz, tets): the centres (in the order of the marked cells) and the tetrahedra in
    FEM-node indices (lattice nodes first, lexicographic; then the centres)."""
    cx, cy, cz = (int(c) for c in desc.fem_cells)
    fx, fy, fz = cx + 1, cy + 1, cz + 1
    n_lat = fx * fy * fz
    lo = np.asarray(desc.origin, dtype=np.float64) + desc.h * np.asarray(desc.fem_lo, dtype=np.float64)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    extra, tets = [], []
    for k in range(cz):
        for j in range(cy):
            for i in range(cx):
                marked = bool(marks[i + cx * (j + cy * k)])
                if marked:
                    c_id = n_lat + len(extra)
                    extra.append(lo + desc.h * np.array([i + 0.5, j + 0.5, k + 0.5]))
                for perm in perms:
                    p = [i, j, k]
                    v = [p[0] + fx * (p[1] + fy * p[2])]
                    for a in perm:
                        p[a] += 1
                        v.append(p[0] + fx * (p[1] + fy * p[2]))
                    if marked:
                        tets.append((v[0], v[1], v[2], c_id))
                        tets.append((c_id, v[1], v[2], v[3]))
                    else:
                        tets.append(tuple(v))
    return np.asarray(extra, dtype=np.float64).reshape(-1, 3), np.asarray(tets, dtype=np.int32)


def refined_values(desc: ProblemDesc, marks: np.ndarray, lattice_values: np.ndarray) -> np.ndarray:
    """Nodal values on the refined mesh: the lattice values, then at each centre the mean of its
    cell's eight corners (the trilinear value there)."""
    cx, cy, cz = (int(c) for c in desc.fem_cells)
    fx, fy = cx + 1, cy + 1
    v = np.asarray(lattice_values, dtype=np.float64)
    out = [v]
    add = []
    for idx in np.nonzero(marks)[0]:
        i, j, k = idx % cx, (idx // cx) % cy, idx // (cx * cy)
        corners = [(i + a) + fx * ((j + b) + fy * (k + c)) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
        add.append(v[corners].mean())
    out.append(np.asarray(add, dtype=np.float64))
    return np.concatenate(out)
