"""Pins of the oracle's point-dipole source (the DD_SRC_DIPOLE branch of oracle.solver.forcing).

With eps = 1 and sigma = 0 the discrete scheme is M (E^{n+1} - 2E^n + E^{n-1}) / dt^2 + K E^n = F^n,
with M = h^3 on interior nodes and K = h times the 7-point stencil, so each component obeys
E_tt - Delta_h E = F / h^3: a force F = P(t) pol at one node is a discrete point source of
strength P(t) pol.  In free space the continuous solution is pol P(t - r) / (4 pi r) (the
retarded Green's function of the scalar wave equation).  The box's mirror-Neumann faces
(weights of the cells inside, lumped masses h^3 2^-b) are the even fold of an unbounded grid
about the boundary node planes, so inside a box with no absorbing face the exact solution is
the sum of that Green's function over the source's mirror images in every face plane (a
source on a face, edge or corner coincides with 1, 3 or 7 of its images: its folded force
counts 2, 4 or 8 times).

Pinned here: second-order convergence of the traces to that image sum (index order, force
scale and time function of the branch), the same sum for sources on a face, an edge and a
corner (the boundary mass factor), and reciprocity (a source at a seen at b equals a source
at b seen at a) under the symmetric div-div form R2, which is exact for any symmetric
operator; planted mistakes in the branch fail these pins.
"""

import math

import numpy as np
import pytest

from oracle import solver as osolver
from oracle.discretization import Discretization
from synth.configs import FACE_ALL, FACE_BOTTOM, FACE_TOP, SRC_DIPOLE, ProblemDesc, Source


def gauss_sine_pulse(t, omega, t0, width, amp=1.0):
    """The Gaussian-modulated sine of the dipole kind, sin(omega (t - t0)) exp(-((t - t0)/width)^2 / 2)
    on [0, 2 t0] (zero elsewhere), vectorised over t."""
    t = np.asarray(t, dtype=np.float64)
    u = (t - t0) / width
    p = amp * np.sin(omega * (t - t0)) * np.exp(-0.5 * u * u)
    return np.where((t >= 0.0) & (t <= 2.0 * t0), p, 0.0)


def image_sum(src_x, rec_x, t, pulse, box):
    """sum over the mirror images s' of the source in the faces of [0, box]^3 of
    pulse(t - |x - s'|) / (4 pi |x - s'|): (len(t), len(rec_x))."""
    reach = float(t[-1])
    m = int(math.ceil(reach / (2.0 * box))) + 1
    axes = []
    for a in range(3):
        axes.append(np.array([s * src_x[a] + 2.0 * k * box for k in range(-m, m + 1) for s in (1.0, -1.0)]))
    imgs = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    out = np.zeros((len(t), len(rec_x)))
    for q, x in enumerate(rec_x):
        r = np.linalg.norm(imgs - x[None, :], axis=1)
        for rr in r[r <= reach]:
            out[:, q] += pulse(t - rr) / (4.0 * math.pi * rr)
    return out


BOX = 1.0
TP = 0.5            # pulse period: 8, 16, 32 nodes per wavelength on the three grids
T_END = 1.0


def _dipole_run(n, src_frac, pol=(0.0, 1.0, 0.0), fd_only=True):
    """The oracle's traces on the top face of [0, 1]^3 (n nodes per axis, no absorbing face) for a
    dipole at src_frac * (n - 1), and the image sum at the same nodes and times."""
    h = BOX / (n - 1)
    dt = 0.5 * h / math.sqrt(3.0)
    nt = int(round(T_END / dt))
    desc = ProblemDesc(n_outer=(n, n, n), h=h, origin=(0.0, 0.0, 0.0), fem_lo=(1, 1, 1), fem_cells=(2, 2, 2),
                       dt=dt, n_steps=nt, ckpt_every=nt, detector_faces=FACE_TOP, absorbing_faces=0, t_switch=0.0)
    pos = tuple(int(round(f * (n - 1))) for f in src_frac)
    assert np.allclose(np.array(pos) * h, np.array(src_frac) * BOX)
    omega = 2.0 * math.pi / TP
    src = Source(kind=SRC_DIPOLE, omega=omega, t0=1.5 * TP, width=0.5 * TP, amp=1.0, pol=pol, pos=pos)
    d = Discretization(desc, fd_only=fd_only).set_coefficients(np.ones(27), np.zeros(27))
    tr = osolver.forward(d, src)["traces"]
    x_det = d.x[d.det]
    t = dt * np.arange(1, nt + 1)
    return tr, x_det, t, np.array(pos) * h, (omega, 1.5 * TP, 0.5 * TP)


_RUNS = {}


def _green_error(n, src_frac, min_r=0.2, pol=(0.0, 1.0, 0.0), fd_only=True, cached=True):
    """Relative L2 error, over the top-face nodes of the 1/16 lattice within 0.25 of the face centre
    and at least min_r from the source, of every traced component against pol * image sum.
    Runs of the unmodified oracle are shared between tests (cached); planted mistakes run anew."""
    key = (n, tuple(src_frac), tuple(pol), fd_only)
    if cached and key in _RUNS:
        run = _RUNS[key]
    else:
        run = _dipole_run(n, src_frac, pol, fd_only)
        if cached:
            _RUNS[key] = run
    tr, x_det, t, sx, (omega, t0, width) = run
    g = x_det * 16.0
    sel = np.all(np.abs(g - np.round(g)) < 1e-9, axis=1)
    sel &= (np.abs(x_det[:, 0] - 0.5) <= 0.25 + 1e-12) & (np.abs(x_det[:, 1] - 0.5) <= 0.25 + 1e-12)
    sel &= np.linalg.norm(x_det - sx[None, :], axis=1) >= min_r - 1e-12
    ex = image_sum(sx, x_det[sel], t, lambda s: gauss_sine_pulse(s, omega, t0, width), BOX)
    exact = ex[:, :, None] * np.asarray(pol)[None, None, :]
    num = tr[:, sel, :]
    return float(np.linalg.norm(num - exact) / np.linalg.norm(exact))


INTERIOR = (7 / 16, 6 / 16, 12 / 16)


def test_dipole_green_function_second_order():
    errs = [_green_error(n, INTERIOR) for n in (17, 33, 65)]
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert errs[2] < 1e-2, errs
    for r in ratios:
        assert 3.5 <= r <= 4.5, (errs, ratios)


def test_dipole_green_function_hybrid_and_polarisation():
    """The hybrid discretisation (a FEM box at eps = 1) and an oblique moment give the same sum."""
    pol = (0.48, -0.6, 0.64)
    e_fd = _green_error(33, INTERIOR, pol=pol, fd_only=True)
    e_hy = _green_error(33, INTERIOR, pol=pol, fd_only=False)
    assert e_fd < 3e-2 and abs(e_hy - e_fd) < 1e-12


@pytest.mark.parametrize("where,frac", [
    ("face", (7 / 16, 6 / 16, 1.0)),
    ("edge", (0.0, 6 / 16, 1.0)),
    ("corner", (0.0, 0.0, 1.0)),
])
def test_dipole_on_the_boundary_counts_its_images(where, frac):
    """A source on the top face, the top / x-min edge and a top corner (lumped mass h^3/2, h^3/4,
    h^3/8): the traces follow the image sum, in which the source coincides with 1, 3 or 7 images."""
    e33 = _green_error(33, frac)
    e65 = _green_error(65, frac)
    assert e65 < 1.5e-2, (where, e33, e65)
    assert 3.3 <= e33 / e65 <= 4.7, (where, e33, e65)


def _reciprocity(form, seed=7):
    """Max |G_ab - G_ba| / max |G| for two dipoles on detector faces with moments e_p, e_q."""
    rng = np.random.default_rng(seed)
    n = (14, 13, 15)
    h = 0.05
    desc = ProblemDesc(n_outer=n, h=h, origin=(0.0, 0.0, 0.0), fem_lo=(3, 3, 4), fem_cells=(7, 6, 6),
                       dt=0.5 * h / math.sqrt(3.0), n_steps=60, ckpt_every=60, detector_faces=FACE_ALL,
                       absorbing_faces=FACE_BOTTOM, t_switch=0.0)
    d = Discretization(desc, divdiv_form=form)
    free = d.fem_free
    eps = np.where(free, 1.0 + 4.0 * rng.uniform(size=d.n_fem), 1.0)
    sig = np.where(free, 2.0 * rng.uniform(size=d.n_fem), 0.0)
    d.set_coefficients(eps, sig)
    a, b = (2, 5, n[2] - 1), (n[0] - 1, 8, 9)     # top face, x-max face
    p, q = 0, 2
    omega = 2.0 * math.pi / (8 * h)
    tp = 2.0 * math.pi / omega

    def run(pos, c):
        pol = [0.0, 0.0, 0.0]
        pol[c] = 1.0
        src = Source(kind=SRC_DIPOLE, omega=omega, t0=1.5 * tp, width=0.5 * tp, pol=tuple(pol), pos=pos)
        return osolver.forward(d, src)["traces"]

    def node(pos):
        g = pos[0] + n[0] * (pos[1] + n[1] * pos[2])
        return int(np.nonzero(d.det == g)[0][0])

    tr_a = run(a, p)
    tr_b = run(b, q)
    g_ab = tr_a[:, node(b), q]
    g_ba = tr_b[:, node(a), p]
    scale = max(np.max(np.abs(g_ab)), np.max(np.abs(g_ba)))
    assert scale > 0
    return float(np.max(np.abs(g_ab - g_ba)) / scale)


def test_dipole_reciprocity_under_the_symmetric_form():
    assert _reciprocity("R2") <= 1e-12


def test_reciprocity_needs_a_symmetric_operator():
    """R1 (the nodal product inside the divergence) is not symmetric where eps varies: the same
    exchange then differs, which shows the reciprocity pin can fail."""
    assert _reciprocity("R1") > 1e-6


# ---- planted mistakes in the dipole branch (monkeypatched copies of forcing, on the CPU) ----------

def _forcing_with(mutation):
    def forcing(d, src, n):
        F = np.zeros((d.N, 3))
        t = n * d.dt
        if mutation == "late":
            t = (n + 1) * d.dt                      # time function one step late
        p = osolver.source_time_function(src, t)
        if p == 0.0:
            return F
        i, j, k = (int(v) for v in src.pos)
        if mutation == "index":
            g = k + d.nvec[2] * (j + d.nvec[1] * i)    # z fastest instead of x fastest
        else:
            g = i + d.nvec[0] * (j + d.nvec[1] * k)
        scale = d.m[g] / d.h ** 3 if mutation == "mass" else 1.0   # force scaled by the mass fraction
        F[g] = p * scale * np.asarray(src.pol, dtype=np.float64)
        return F
    return forcing


@pytest.mark.parametrize("mutation,frac,n", [
    ("index", INTERIOR, 33),
    ("mass", (7 / 16, 6 / 16, 1.0), 33),
    ("late", INTERIOR, 65),
])
def test_dipole_mutations_are_caught(monkeypatch, mutation, frac, n):
    base = _green_error(n, frac)
    monkeypatch.setattr(osolver, "forcing", _forcing_with(mutation))
    bad = _green_error(n, frac, cached=False)
    assert bad > 5.0 * base and bad > 0.03, (mutation, base, bad)


def test_unmutated_copy_of_the_branch_is_unchanged(monkeypatch):
    """The copy used for the mutations equals the oracle's branch when nothing is planted."""
    base = _green_error(33, INTERIOR)
    monkeypatch.setattr(osolver, "forcing", _forcing_with(None))
    assert abs(_green_error(33, INTERIOR, cached=False) - base) <= 1e-15
