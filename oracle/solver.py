"""Oracle time loops: forward, adjoint and gradient in FP64 (plain three-level form).

Forward (box "Forward problem" with the model problem eq. model1):
    D+^n E^{n+1} = (2 M_eps/dt^2 - A) E^n - D-^n E^{n-1} + F^n,
    D+-^n = M_eps/dt^2 +- (M_sigma + S^n)/(2 dt).
The model problem starts from rest, E^0 = E^{-1} = 0.  General initial data (eq.
forward_initial_cond, E(0) = f_0, dE/dt(0) = f_1) gives the two starting levels
E^0 = f_0 and E^{-1} = f_0 - dt f_1 (the one-sided difference of dE/dt at t = 0), so the
starting increment is V^0 = E^0 - E^{-1} = dt f_1; both levels are independent of eps and
sigma.
Traces T^n = E^n on the detector nodes for n = 1..N_t.

Loss: J = 1/2 sum_n sum_detectors |T^n - E_obs^n|^2 (eq. tikhonov_functional with
the observation indicator on the detector faces, smoothing z = 1, no
Tikhonov term).

Adjoint (box "Adjoint problem"), exact transpose of the forward recursion with
the Lagrangian L = J + sum_n lambda^n . R^n:
    D+^{k-1} lambda^{k-1} = -r^k + (2 M_eps/dt^2 - A^T) lambda^k - D-^{k+1} lambda^{k+1},
    k = N_t .. 1,  lambda^{N_t} = lambda^{N_t+1} = 0,  r^k = dJ/dT^k on the detectors.

Gradient (eq. gradeps and dL/deps, dL/dsigma of the optimality conditions,
taken exactly on the discrete scheme):
    dJ/deps_i   = sum_{n=0}^{N_t-1} [ m_i lambda^n_i . (E^{n+1} - 2E^n + E^{n-1})_i / dt^2
                                      + sum_{K ∋ i} |K| div_K(lambda^n) (grad phi_i . E^n_i) ],
    dJ/dsigma_i = sum_{n=0}^{N_t-1} m_i lambda^n_i . (E^{n+1} - E^{n-1})_i / (2 dt),
on free FEM nodes (layer >= 2), zero elsewhere.  The -lambda(x, 0) f_1 term of eq. gradeps
is the n = 0 row of the mass term, where E^{-1} = E^0 - V^0 with V^0 = dt f_1: summed by
parts,
    sum_n lambda^n . (V^{n+1} - V^n) = -sum_n (lambda^{n+1} - lambda^n) . V^{n+1} - lambda^0 . V^0
(lambda^{N_t} = 0), the discrete -int lambda_t . E_t plus the boundary term
-lambda^0 . V^0 = -dt lambda^0 . f_1.
It vanishes when the problem starts from rest.

The paper's own gradient formula (eq. gradeps with div((eps~) E) ~ eps~ div E) replaces
the div-div term by
    sum_{n} sum_{K ∋ i} (|K| / 4) div_K(lambda^n) div_K(E^n)
(|K|/4 = the integral of phi_i over K); it is returned as a variant.  For the symmetric
div-div form R2 it is the exact derivative, and the R2 discretisation uses it as such.
"""

from __future__ import annotations

import math

import numpy as np

SRC_SINE1, SRC_GAUSS_SINE, SRC_DIPOLE = 1, 2, 3


def source_time_function(src, t):
    """P(t): eq. f (one sine period) or a Gaussian-modulated sine on [0, 2 t0]."""
    if src.kind == SRC_SINE1:
        return src.amp * math.sin(src.omega * t) if 0.0 < t < 2.0 * math.pi / src.omega else 0.0
    if src.kind in (SRC_GAUSS_SINE, SRC_DIPOLE):
        if t < 0.0 or t > 2.0 * src.t0:
            return 0.0
        s = (t - src.t0) / src.width
        return src.amp * math.sin(src.omega * (t - src.t0)) * math.exp(-0.5 * s * s)
    raise ValueError("unknown source kind")


def incidence(src):
    """Unit direction k of a plane wave's travel, or None for normal incidence (k = -e_z, the
    model problem of eq. model1): src.dir, normalised; zero (or absent) means normal incidence.
    The wave enters through the top face, so k_z < 0."""
    v = np.asarray(getattr(src, "dir", (0.0, 0.0, 0.0)), dtype=np.float64)
    nv = float(np.linalg.norm(v))
    if nv == 0.0:
        return None
    k = v / nv
    if not k[2] < 0.0:
        raise ValueError("a plane wave enters through the top face: dir must point down (dir_z < 0)")
    return k


def arrival_delays(d, k):
    """tau_i = k . (x_i - x_ref) on the top-face nodes, with x_ref the top-face node the wave
    front reaches first (the smallest k . x), so every delay is >= 0."""
    top = d.face_mass[1] > 0.0
    proj = d.x[top] @ k
    return top, proj - proj.min()


def forcing(d, src, n):
    """F^n over the grid, shape (N, 3)."""
    F = np.zeros((d.N, 3))
    t = n * d.dt
    pol = np.asarray(src.pol, dtype=np.float64)
    if src.kind == SRC_DIPOLE:
        p = source_time_function(src, t)
        if p == 0.0:
            return F
        i, j, k = (int(v) for v in src.pos)
        g = i + d.nvec[0] * (j + d.nvec[1] * k)
        F[g] = p * pol
        return F
    if t > float(d.desc.t_switch):
        return F
    # Gamma_{1,1}: d_n E = P on the top face; a wave arriving from direction k reaches top-face
    # node i at the delay tau_i, so there d_n E = P(t - tau_i)
    k = incidence(src)
    if k is None:
        p = source_time_function(src, t)
        if p != 0.0:
            F += (d.face_mass[1] * p)[:, None] * pol[None, :]
        return F
    top, tau = arrival_delays(d, k)
    pv = np.array([source_time_function(src, t - ti) for ti in tau])
    F[top] += (d.face_mass[1][top] * pv)[:, None] * pol[None, :]
    return F


def forward(d, src=None, n_steps=None, force=None, keep_full=False, initial=None):
    """Run the forward recursion.

    ``src`` is a synth Source, or ``force`` a callable n -> F^n (N, 3).  ``initial`` is
    None (start from rest) or (f_0, f_1), each (N, 3) over the grid: E^0 = f_0,
    E^{-1} = f_0 - dt f_1.
    Returns a dict with traces (N_t, n_det, 3), energy W^{n+1/2} (N_t,),
    balance residual (N_t,), E on FEM nodes for levels -1..N_t (N_t+2, n_fem, 3)
    and, if ``keep_full``, E on the whole grid for levels -1..N_t.
    """
    nt = int(d.desc.n_steps if n_steps is None else n_steps)
    dt = d.dt
    Me = d.M_eps[:, None]
    E_prev = np.zeros((d.N, 3))
    E_cur = np.zeros((d.N, 3))
    w_prev = 0.0
    if initial is not None:
        E_cur = np.array(initial[0], dtype=np.float64).reshape(d.N, 3)
        V0 = dt * np.asarray(initial[1], dtype=np.float64).reshape(d.N, 3)
        E_prev = E_cur - V0
        # W^{-1/2}: the energy of the starting pair, in the form of W^{n+1/2} below
        w_prev = 0.5 * np.sum(Me * V0 * V0) / dt ** 2 + 0.5 * np.sum(E_cur * d.apply_A(E_prev))
    traces = np.zeros((nt, len(d.det), 3))
    energy = np.zeros(nt)
    balance = np.zeros(nt)
    fem_hist = np.zeros((nt + 2, d.n_fem, 3))
    fem_hist[0] = E_prev[d.fem_grid]
    fem_hist[1] = E_cur[d.fem_grid]
    full = [E_prev.copy(), E_cur.copy()] if keep_full else None
    for n in range(nt):
        F = force(n) if force is not None else forcing(d, src, n)
        C = (d.M_sig + d.damping(n))[:, None]
        AE = d.apply_A(E_cur)
        rhs = (2.0 * Me / dt ** 2) * E_cur - AE - (Me / dt ** 2 - C / (2 * dt)) * E_prev + F
        E_next = rhs / (Me / dt ** 2 + C / (2 * dt))
        traces[n] = E_next[d.det]
        V = E_next - E_cur
        w = 0.5 * np.sum(Me * V * V) / dt ** 2 + 0.5 * np.sum(E_next * AE)
        D = E_next - E_prev
        balance[n] = (w - w_prev) - 0.5 * np.sum(D * (F - C * D / (2 * dt)))
        energy[n] = w
        w_prev = w
        fem_hist[n + 2] = E_next[d.fem_grid]
        if keep_full:
            full.append(E_next.copy())
        E_prev, E_cur = E_cur, E_next
    out = dict(traces=traces, energy=energy, balance=balance, fem_hist=fem_hist)
    if keep_full:
        out["full"] = np.stack(full)
    return out


def taper(n_steps, dt, delta):
    """Smoothing function z of eq. tikhonov_functional at the trace rows (row n holds time
    level n + 1, t = (n + 1) dt): 1 up to T - delta, then a cosine ramp to 0 at T = n_steps dt,
    z(t) = (1 + cos(pi (t - T + delta) / delta)) / 2.  delta <= 0 gives z = 1."""
    T = n_steps * dt
    t = dt * np.arange(1, n_steps + 1)
    if delta <= 0:
        return np.ones(n_steps)
    s = np.clip((t - (T - delta)) / delta, 0.0, 1.0)
    return 0.5 * (1.0 + np.cos(np.pi * s))


def loss_and_cotangent(traces, eobs, z=None):
    """J = 1/2 sum_n z_n sum_det |T^n - E_obs^n|^2 (z = 1 when not given) and dJ/dT.
    traces / eobs: [n_steps][n_det][3], or with a leading source axis."""
    r = traces - eobs
    if z is None:
        return 0.5 * float(np.sum(r * r)), r
    w = np.asarray(z, dtype=np.float64).reshape((-1, 1, 1))
    return 0.5 * float(np.sum(w * r * r)), w * r


def adjoint_gradient(d, cot, fwd, keep_lambda=False, sbp=True):
    """Adjoint recursion backward in time and the eps / sigma gradient.

    ``cot`` is dJ/dT with the shape of the traces; ``fwd`` the forward result
    (its FEM history).  Returns dict(g_eps, g_sigma) over the FEM lattice, the
    mass term in both the plain and the summed-by-parts form (the latter, and the
    sigma term summed by parts, only with ``sbp``: they keep lambda^n on the FEM nodes
    for every n), and optionally lambda^n (n = 0..N_t-1) on the whole grid.
    """
    nt = cot.shape[0]
    dt = d.dt
    Me = d.M_eps[:, None]
    Eh = fwd["fem_hist"]                      # level n at index n + 1
    m = d.m[d.fem_grid]
    lam_next = np.zeros((d.N, 3))            # lambda^{k+1}
    lam_cur = np.zeros((d.N, 3))             # lambda^k
    g_mass = np.zeros(d.n_fem)
    g_dd = np.zeros(d.n_fem)
    g_dd_paper = np.zeros(d.n_fem)
    g_sig = np.zeros(d.n_fem)
    lam_f = np.zeros((nt + 1, d.n_fem, 3)) if sbp else None   # lambda^n on FEM nodes, n = 0..N_t
    lams = np.zeros((nt, d.N, 3)) if keep_lambda else None
    for k in range(nt, 0, -1):
        r = np.zeros((d.N, 3))
        r[d.det] = cot[k - 1]
        Cm = (d.M_sig + d.damping(k - 1))[:, None]
        Cp = (d.M_sig + d.damping(k + 1))[:, None]
        rhs = -r + (2.0 * Me / dt ** 2) * lam_cur - d.apply_AT(lam_cur) - (Me / dt ** 2 - Cp / (2 * dt)) * lam_next
        lam_prev = rhs / (Me / dt ** 2 + Cm / (2 * dt))
        n = k - 1
        lf = lam_prev[d.fem_grid]
        if sbp:
            lam_f[n] = lf
        e_p, e_c, e_m = Eh[n + 2], Eh[n + 1], Eh[n]
        g_mass += m * np.sum(lf * (e_p - 2.0 * e_c + e_m), axis=1) / dt ** 2
        g_sig += m * np.sum(lf * (e_p - e_m), axis=1) / (2.0 * dt)
        # div-div term: sum_K |K| div_K(lambda^n restricted to FEM rows) (grad phi_i . E^n_i)
        lr = lf.copy()
        lr[~d.fem_owned] = 0.0
        div = np.einsum("tac,tac->t", d.grad, lr[d.tets])
        ge = np.einsum("tac,tac->ta", d.grad, e_c[d.tets])
        g_dd += np.bincount(d.tets.ravel(), weights=((d.vol * div)[:, None] * ge).ravel(), minlength=d.n_fem)
        # paper formula: sum_K (|K| / 4) div_K(lambda^n) div_K(E^n) on the four vertices of K
        div_e = np.einsum("tac,tac->t", d.grad, e_c[d.tets])
        g_dd_paper += np.bincount(d.tets.ravel(), weights=np.repeat(0.25 * d.vol * div * div_e, 4),
                                  minlength=d.n_fem)
        if keep_lambda:
            lams[n] = lam_prev
        lam_next, lam_cur = lam_cur, lam_prev
    # summation by parts of the mass term: -sum_n m (lambda^{n+1} - lambda^n) . (E^{n+1} - E^n) / dt^2
    # plus the boundary term -m lambda^0 . V^0 / dt^2 of the starting levels (zero from rest)
    g_mass_sbp = np.zeros(d.n_fem)
    g_sig_sbp = np.zeros(d.n_fem)
    for n in range(nt if sbp else 0):
        g_mass_sbp -= m * np.sum((lam_f[n + 1] - lam_f[n]) * (Eh[n + 2] - Eh[n + 1]), axis=1) / dt ** 2
    if sbp:
        g_mass_sbp -= m * np.sum(lam_f[0] * (Eh[1] - Eh[0]), axis=1) / dt ** 2
    # the sigma term summed by parts: sum_n m (lambda^n + lambda^{n+1}) . (E^{n+1} - E^n) / (2 dt)
    # plus the boundary row m lambda^0 . V^0 / (2 dt) of the starting levels (zero from rest)
    for n in range(nt if sbp else 0):
        g_sig_sbp += m * np.sum((lam_f[n] + lam_f[n + 1]) * (Eh[n + 2] - Eh[n + 1]), axis=1) / (2.0 * dt)
    if sbp:
        g_sig_sbp += m * np.sum(lam_f[0] * (Eh[1] - Eh[0]), axis=1) / (2.0 * dt)
    free = d.fem_free
    g_eps_paper = np.where(free, g_mass + g_dd_paper, 0.0)
    if getattr(d, "divdiv_form", "R1") == "R2":
        g_dd = g_dd_paper           # exact for the element-mean form
    g_eps = np.where(free, g_mass + g_dd, 0.0)
    g_sigma = np.where(free, g_sig, 0.0)
    out = dict(g_eps=g_eps, g_sigma=g_sigma, g_mass=np.where(free, g_mass, 0.0),
               g_mass_sbp=np.where(free, g_mass_sbp, 0.0), g_sigma_sbp=np.where(free, g_sig_sbp, 0.0),
               g_divdiv=np.where(free, g_dd, 0.0),
               g_eps_paper=g_eps_paper)
    if keep_lambda:
        out["lambda"] = lams
    return out


def energy_balance_residual(fwd):
    return fwd["balance"]
