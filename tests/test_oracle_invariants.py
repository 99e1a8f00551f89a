"""Pins of the oracle's time stepping, adjoint and gradient.

* Closed form: a normally incident plane wave in eps = 1 (model problem
  eq. model1 with the source of eq. f) has the top-face trace
  E_2(t) = Q(t), Q = int_0^t P; the discrete trace converges at second order.
* Special case: with eps = 1 the hybrid FE/FD scheme equals the pure 7-point
  finite-difference scheme (the FEM rows of the Kuhn split are 7-point rows).
* Invariant: the discrete energy W^{n+1/2} is conserved without damping and
  source, and obeys the exact balance identity with conductivity, absorbing
  faces and the source on.
* Invariant: the adjoint recursion is the exact transpose of the forward one
  (dot-product test sum_k r^k . T^k = -sum_n lambda^n . F^n).
* Brute force: the eps / sigma gradient (eq. gradeps, taken on the discrete
  scheme) matches central differences of the loss on a tiny grid.
* Identity: the mass term of the eps gradient equals its summation-by-parts
  form, the discrete -int lambda_t . E_t of eq. gradeps.
* Invariants: linearity in the forcing and the initial data (superposition),
  time-shift invariance when the damping does not change in time, and mirror symmetry of a
  symmetric grid, box and medium (eps = 1), each <= 1e-12.
"""

import math

import numpy as np
from scipy.integrate import quad

import synth
from oracle.discretization import Discretization
from oracle.solver import adjoint_gradient, forward, loss_and_cotangent, source_time_function


def _plane_wave_error(h, src, L=2.5, T=4.0):
    nz = int(round(L / h)) + 1
    dt = 0.5 * h / math.sqrt(3.0)
    desc = synth.ProblemDesc(n_outer=(6, 6, nz), h=h, origin=(0, 0, 0), fem_lo=(1, 1, nz // 3),
                             fem_cells=(2, 2, nz // 3), dt=dt, n_steps=int(round(T / dt)),
                             detector_faces=synth.FACE_TOP, absorbing_faces=synth.FACE_TOP | synth.FACE_BOTTOM,
                             t_switch=src.support_end())
    n = desc.n_fem_nodes()
    d = Discretization(desc).set_coefficients(np.ones(n), np.zeros(n))
    f = forward(d, src)
    tr = f["traces"][:, :, 1]
    tn = dt * np.arange(1, desc.n_steps + 1)
    q = np.array([quad(lambda s: source_time_function(src, s), 0.0, min(t, src.support_end()), limit=200)[0] for t in tn])
    assert np.abs(f["traces"][:, :, 0]).max() == 0.0 and np.abs(f["traces"][:, :, 2]).max() == 0.0
    assert np.abs(tr - tr[:, :1]).max() <= 1e-13     # uniform across the top face
    return np.linalg.norm(tr[:, 0] - q) / np.linalg.norm(q)


def test_plane_wave_second_order():
    src = synth.configs.gauss_sine(2 * math.pi)
    errs = [_plane_wave_error(h, src) for h in (0.1, 0.05, 0.025)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.6 and 3.6 < r2 < 4.4, errs
    assert errs[2] < 4e-3


def test_plane_wave_sine1_source():
    src = synth.Source(kind=synth.SRC_SINE1, omega=2 * math.pi)
    e1, e2 = _plane_wave_error(0.05, src), _plane_wave_error(0.025, src)
    assert e2 < e1 and e2 < 2e-2


def test_hybrid_equals_finite_difference_when_eps_is_one():
    for name in ("tiny", "ragged"):
        w = synth.with_steps(synth.small(name), 60)
        n = w.desc.n_fem_nodes()
        f1 = forward(Discretization(w.desc).set_coefficients(np.ones(n), np.zeros(n)), w.sources[0])
        f2 = forward(Discretization(w.desc, fd_only=True).set_coefficients(np.ones(n), np.zeros(n)), w.sources[0])
        assert np.abs(f1["traces"]).max() > 0
        assert np.abs(f1["traces"] - f2["traces"]).max() <= 1e-13 * np.abs(f2["traces"]).max()


def test_energy_conserved_closed_box():
    w = synth.small("tiny")
    desc = w.desc
    desc.absorbing_faces = 0
    desc.n_steps = 200
    n = desc.n_fem_nodes()
    f = forward(Discretization(desc).set_coefficients(np.ones(n), np.zeros(n)), w.sources[0])
    off = int(desc.t_switch / desc.dt) + 2
    W = f["energy"][off:]
    assert W.max() > 0
    assert (W.max() - W.min()) <= 1e-12 * W.max()


def test_energy_balance_with_damping_and_source():
    w = synth.with_steps(synth.small("ragged"), 300)
    n = w.desc.n_fem_nodes()
    d = Discretization(w.desc)
    sig = np.where(d.fem_free, 0.8, 0.0)
    f = forward(d.set_coefficients(np.ones(n), sig), w.sources[0])
    assert np.abs(f["balance"]).max() <= 1e-12 * np.abs(f["energy"]).max()
    # the damping actually removes energy after the source switched off
    off = int(w.desc.t_switch / w.desc.dt) + 2
    assert f["energy"][-1] < 0.9 * f["energy"][off]


def test_adjoint_dot_product():
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    rng = np.random.default_rng(11)
    nt = 30
    F = rng.standard_normal((nt, d.N, 3))
    fw = forward(d, force=lambda k: F[k], n_steps=nt)
    R = rng.standard_normal((nt, len(d.det), 3))
    ag = adjoint_gradient(d, R, fw, keep_lambda=True)
    lhs = np.sum(R * fw["traces"])
    rhs = -np.sum(ag["lambda"] * F)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_dot_product_across_absorbing_switch():
    # the top face switches from source to absorbing mid-run: S^{k-1} != S^{k+1}
    w = synth.small("tiny")
    w.desc.t_switch = 10.5 * w.desc.dt
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    rng = np.random.default_rng(12)
    nt = 25
    F = rng.standard_normal((nt, d.N, 3))
    fw = forward(d, force=lambda k: F[k], n_steps=nt)
    R = rng.standard_normal((nt, len(d.det), 3))
    ag = adjoint_gradient(d, R, fw, keep_lambda=True)
    assert abs(np.sum(R * fw["traces"]) + np.sum(ag["lambda"] * F)) <= 1e-12 * abs(np.sum(R * fw["traces"]))


def test_gradient_matches_central_differences():
    w = synth.small("tiny")
    desc = w.desc
    d = Discretization(desc).set_coefficients(w.eps, w.sigma)
    src = w.sources[0]
    eobs = forward(d, src)["traces"] * 0.9
    fw = forward(d, src)
    _, cot = loss_and_cotangent(fw["traces"], eobs)
    ag = adjoint_gradient(d, cot, fw)

    def J(eps, sig):
        dd = Discretization(desc).set_coefficients(eps, sig)
        return loss_and_cotangent(forward(dd, src)["traces"], eobs)[0]

    free = np.nonzero(d.fem_free)[0]
    assert len(free) >= 4
    delta = 1e-5
    for i in free:
        for which in ("eps", "sig"):
            e, s = w.eps.copy(), w.sigma.copy()
            arr = e if which == "eps" else s
            arr[i] += delta
            jp = J(e, s)
            arr[i] -= 2 * delta
            jm = J(e, s)
            fd = (jp - jm) / (2 * delta)
            g = ag["g_eps" if which == "eps" else "g_sigma"][i]
            assert abs(g - fd) <= 1e-4 * abs(fd), (i, which, g, fd)
    assert np.all(ag["g_eps"][~d.fem_free] == 0) and np.all(ag["g_sigma"][~d.fem_free] == 0)


def test_mass_term_summation_by_parts():
    w = synth.small("ragged")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    fw = forward(d, w.sources[0])
    rng = np.random.default_rng(3)
    cot = rng.standard_normal(fw["traces"].shape) * 1e-3
    ag = adjoint_gradient(d, cot, fw)
    scale = np.abs(ag["g_mass"]).max()
    assert scale > 0
    assert np.abs(ag["g_mass"] - ag["g_mass_sbp"]).max() <= 1e-12 * scale
    # the sigma term likewise: sum_n (lambda^n + lambda^{n+1}) . V^{n+1} (no boundary row from rest)
    ss = np.abs(ag["g_sigma"]).max()
    assert ss > 0 and np.abs(ag["g_sigma"] - ag["g_sigma_sbp"]).max() <= 1e-12 * ss


def test_superposition_of_sources_and_initial_data():
    """The scheme is linear in (f_0, f_1, F): the traces of a combination are the combination
    of the traces (<= 1e-12)."""
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    rng = np.random.default_rng(11)
    nt = 30
    Fa, Fb = rng.standard_normal((nt, d.N, 3)), rng.standard_normal((nt, d.N, 3))
    ia = synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 64)
    ib = synth.initial_pulses(w.desc, synth.configs.SEED_BASE + 65)
    a, b = 0.7, -1.9
    ta = forward(d, force=lambda k: Fa[k], n_steps=nt, initial=ia)["traces"]
    tb = forward(d, force=lambda k: Fb[k], n_steps=nt, initial=ib)["traces"]
    tc = forward(d, force=lambda k: a * Fa[k] + b * Fb[k], n_steps=nt,
                 initial=(a * ia[0] + b * ib[0], a * ia[1] + b * ib[1]))["traces"]
    assert np.abs(tc - (a * ta + b * tb)).max() <= 1e-12 * np.abs(tc).max()


def test_time_shift_invariance():
    """With damping that does not change in time (no top-face switch), delaying the forcing by
    m steps delays the traces by m steps."""
    w = synth.small("tiny")
    w.desc.absorbing_faces = synth.FACE_BOTTOM
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    rng = np.random.default_rng(12)
    nt, m = 40, 7
    F = rng.standard_normal((nt, d.N, 3))
    F[12:] = 0.0
    t0 = forward(d, force=lambda k: F[k], n_steps=nt)["traces"]
    t1 = forward(d, force=lambda k: F[k - m] if k >= m else np.zeros((d.N, 3)), n_steps=nt)["traces"]
    assert np.all(t1[:m] == 0.0)
    assert np.abs(t1[m:] - t0[:nt - m]).max() <= 1e-12 * np.abs(t0).max()


def test_mirror_symmetry():
    """The tiny grid and its FEM box are symmetric under x -> N_x - 1 - x.  With eps = 1 (the
    Kuhn split then carries the 7-point rows, which have no orientation, and the components
    decouple) and an x-symmetric sigma, the top plane wave (uniform in x) gives traces that
    are even under the mirror, component by component."""
    w = synth.small("tiny")
    desc = w.desc
    nx = desc.n_outer[0]
    assert desc.fem_lo[0] + desc.fem_cells[0] == nx - 1 - desc.fem_lo[0]
    d0 = Discretization(desc)
    # sigma symmetric in x: average each FEM node with its mirror image
    fs = desc.fem_shape()
    sl = synth.noise(d0.n_fem, 13).reshape(fs[2], fs[1], fs[0]) ** 2
    sl = 0.5 * (sl + sl[:, :, ::-1])
    sig = np.where(d0.fem_free, sl.ravel(), 0.0)
    d = d0.set_coefficients(np.ones(d0.n_fem), sig)
    tr = forward(d, w.sources[0])["traces"]
    det = np.asarray(d.det)
    gx = det % nx
    rest = det // nx
    mirrored = (nx - 1 - gx) + nx * rest
    pos = {int(g): i for i, g in enumerate(det)}
    perm = np.array([pos[int(g)] for g in mirrored])
    assert np.abs(tr).max() > 0
    assert np.abs(tr[:, perm, :] - tr).max() <= 1e-12 * np.abs(tr).max()
    # not symmetric by construction: an x-asymmetric sigma breaks it
    sig2 = np.where(d0.fem_free, synth.noise(d0.n_fem, 14) ** 2, 0.0)
    tr2 = forward(Discretization(desc).set_coefficients(np.ones(d0.n_fem), sig2), w.sources[0])["traces"]
    assert np.abs(tr2[:, perm, :] - tr2).max() > 1e-6 * np.abs(tr2).max()


def test_adjoint_without_the_lambda_history_gives_the_same_gradient():
    """sbp=False only skips the summed-by-parts diagnostics (and the lambda history they need):
    the gradient is the same, bit for bit."""
    import numpy as np
    import synth
    from oracle.discretization import Discretization
    from oracle.solver import adjoint_gradient, forward
    w = synth.small("tiny")
    d = Discretization(w.desc).set_coefficients(w.eps, w.sigma)
    fw = forward(d, w.sources[0], n_steps=30)
    cot = np.random.default_rng(4).standard_normal(fw["traces"].shape)
    a = adjoint_gradient(d, cot, fw)
    b = adjoint_gradient(d, cot, fw, sbp=False)
    for k in ("g_eps", "g_sigma", "g_eps_paper", "g_mass", "g_divdiv"):
        assert np.array_equal(a[k], b[k]), k
