"""Pins of the oracle's semi-implicit step (oracle.si_step) against what the
mathematics fixes, independent of its own formulas:

* MPDATA (eq. MPDATA's explicit operator): conservation of sum(G psi) by the
  flux form; exact translation by one cell at unit effective Courant number;
  second-order convergence to the exact solution of the transport equation
  in longitude, in latitude (where the Jacobian G = cos(lat) varies) and in
  both (which needs the cross terms of the antidiffusive velocity), against
  a donor-cell control that converges at first order only.
* The step (eqs. SWE1-SWE3, RSWE2-RSWE3, rhslin, Qexpr, Elliptic): a fluid at
  rest stays at rest; the trapezoidal relaxation of the polar absorber has a
  closed form; mass sum(G Phi) is conserved; the step commutes with the
  equatorial mirror (f, tan(lat) odd, Q_y changes sign) and with a shift in
  longitude; the gradient-wind-balanced zonal jet stays balanced to
  truncation error, which shrinks at third order per step when dx and dt
  halve, while a dropped or flipped metric term or a flipped Coriolis sign
  breaks it; and Q^{n+1} satisfies the implicit momentum equation that eq.
  Qexpr inverts.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import si_step as si
from oracle.gcr import gcr
from oracle.operator import Grid, absorber_profile, OMEGA, RADIUS, GRAVITY
import workloads


# bounds of the GPU step's parity tests (float64 explicit part, solve to
# rtol 1e-12): fractions of max|Phi| and of max|Q_x|
TOL_PHI = 1e-11
TOL_Q = 1e-10


def direct(op, rhs, x0):
    return np.linalg.solve(op.dense(), rhs.ravel()).reshape(rhs.shape)


def iterative(op, rhs, x0):
    res = gcr(op, rhs, x0, rtol=1e-13, max_iters=400)
    return res.x


def mp(g, psi, cx, cy):
    return si.mpdata(g, psi, cx, cy, 1.0)


def up(g, psi, cx, cy):
    return si._upwind(g, psi, cx, cy)


# ---------------------------------------------------------------- MPDATA

def test_mpdata_conserves_the_integral():
    rng = np.random.default_rng(1)
    nx, ny = 32, 16
    g = Grid(nx, ny)
    G = np.cos(g.lat)[:, None]
    psi = rng.uniform(0.5, 2.0, (ny, nx))
    cx = rng.uniform(-0.3, 0.3, (ny, nx)) * G
    cy = np.zeros((ny + 1, nx))
    cy[1:-1] = rng.uniform(-0.3, 0.3, (ny - 1, nx)) * np.cos(g.lat_n)[:, None]
    for sign in (1.0, -1.0):
        out = si.mpdata(g, psi, cx, cy, sign)
        assert abs((G * out).sum() - (G * psi).sum()) <= 1e-13 * (G * psi).sum()


def test_mpdata_translates_exactly_at_unit_courant():
    # C^x = G in every row: one cell east per step, antidiffusion vanishes
    rng = np.random.default_rng(2)
    nx, ny = 16, 8
    g = Grid(nx, ny)
    psi = rng.uniform(1.0, 3.0, (ny, nx))
    cx = np.cos(g.lat)[:, None] * np.ones((1, nx))
    cy = np.zeros((ny + 1, nx))
    out = mp(g, psi, cx, cy)
    assert np.allclose(out, np.roll(psi, 1, axis=1), rtol=0, atol=1e-13)


def test_mpdata_is_identity_without_flow():
    rng = np.random.default_rng(3)
    g = Grid(16, 8)
    psi = rng.normal(size=(8, 16))
    out = si.mpdata(g, psi, np.zeros((8, 16)), np.zeros((9, 16)), -1.0)
    assert np.array_equal(out, psi)


def _order(errs):
    errs = np.asarray(errs)
    return np.log2(errs[:-1] / errs[1:])


def _zonal_errors(scheme):
    # psi_t + c psi_lambda = 0 (per-row C^x = c G): exact translation
    errs = []
    for nx in (32, 64, 128, 256):
        g = Grid(nx, 4)
        cx = 0.25 * np.cos(g.lat)[:, None] * np.ones((1, nx))
        cy = np.zeros((5, nx))
        f0 = lambda lam: np.exp(np.sin(lam))
        psi = np.repeat(f0(g.lam)[None, :], 4, axis=0)
        for _ in range(nx):
            psi = scheme(g, psi, cx, cy)
        errs.append(np.abs(psi - f0(g.lam - 0.25 * nx * g.dlam)[None, :]).max())
    return errs


def _characteristic(f0, lam, lat, sx, sy):
    # G psi_t + (U G psi)_lambda + (V G psi)_lat = 0 with constant U, V:
    # psi cos(lat) is carried along lambda - U t, lat - V t
    return f0(lam - sx, lat - sy) * np.cos(lat - sy) / np.cos(lat)


def _meridional_errors(scheme, sizes=(32, 64, 128, 256)):
    errs = []
    for ny in sizes:
        nx = 8
        g = Grid(nx, ny)
        cy = np.zeros((ny + 1, nx))
        cy[1:-1] = 0.25 * np.cos(g.lat_n)[:, None]
        cx = np.zeros((ny, nx))
        f0 = lambda lam, p: np.exp(-((p + 0.35) / 0.2) ** 2) + 0.0 * lam
        L, P = np.meshgrid(g.lam, g.lat)
        psi = f0(L, P)
        n = ny // 2
        for _ in range(n):
            psi = scheme(g, psi, cx, cy)
        errs.append(np.abs(psi - _characteristic(f0, L, P, 0.0, n * 0.25 * g.dphi)).max())
    return errs


def _oblique_errors(scheme, sizes=(32, 64, 128, 256)):
    errs = []
    for ny in sizes:
        nx = 2 * ny
        g = Grid(nx, ny)
        cx = 0.5 * np.cos(g.lat)[:, None] * np.ones((1, nx))
        cy = np.zeros((ny + 1, nx))
        cy[1:-1] = 0.25 * np.cos(g.lat_n)[:, None]
        f0 = lambda lam, p: np.exp(-((p + 0.35) / 0.25) ** 2) * np.exp(np.sin(lam))
        L, P = np.meshgrid(g.lam, g.lat)
        psi = f0(L, P)
        n = ny // 2
        for _ in range(n):
            psi = scheme(g, psi, cx, cy)
        errs.append(np.abs(psi - _characteristic(f0, L, P, n * 0.5 * g.dlam, n * 0.25 * g.dphi)).max())
    return errs


def test_mpdata_second_order_in_longitude():
    assert _order(_zonal_errors(mp))[-1] > 1.85
    assert _order(_zonal_errors(up))[-1] < 1.2      # the control: donor cell alone


def test_mpdata_second_order_in_latitude():
    assert _order(_meridional_errors(mp))[-1] > 1.85
    assert _order(_meridional_errors(up))[-1] < 1.2


def test_mpdata_second_order_oblique():
    # the cross terms of the antidiffusive velocity are needed here: without
    # them the order stays near 1.5
    o = _order(_oblique_errors(mp))
    assert o[-1] > 1.85, o
    assert _order(_oblique_errors(up, sizes=(64, 128, 256)))[-1] < 1.2


# ---------------------------------------------------------------- the step

def _rand_state(nx, ny, seed):
    rng = np.random.default_rng(seed)
    st = workloads.zonal_flow_state(nx, ny, u0=30.0, pert_amp=40.0, pert_lmax=6, seed_instance=seed)
    phi = st["phi"]
    qx = st["qx"] * (1.0 + 0.1 * rng.uniform(-1, 1, (ny, nx)))
    qy = phi * rng.uniform(-5.0, 5.0, (ny, nx))
    return si.State(phi, qx, qy)


def _orography(nx, ny, seed):
    rng = np.random.default_rng(100 + seed)
    g = Grid(nx, ny)
    L, P = np.meshgrid(g.lam, g.lat)
    return 500.0 * (1 + np.sin(2 * L + rng.uniform(0, 6)) * np.cos(P) ** 2)


def test_rest_state_is_steady():
    nx, ny = 32, 16
    z = np.zeros((ny, nx))
    s = si.State(np.full((ny, nx), 8000.0), z.copy(), z.copy())
    new, _ = si.si_step(nx, ny, s, s, z, (z, z), si.Params(dt=900.0, absorber=1e-4), direct)
    assert np.abs(new.phi - 8000.0).max() <= 1e-12 * 8000.0
    # momentum scale of a 1 m/s flow: 8000 m^2/s
    assert np.abs(new.qx).max() <= 1e-12 * 8000.0
    assert np.abs(new.qy).max() <= 1e-12 * 8000.0


def test_absorber_relaxation_closed_form():
    # flat, at rest, no rotation, relaxation towards a uniform zonal Qbar:
    # Q^{n+1} (1 + d alpha) = Qhat + d alpha Qbar, Qhat = d alpha Qbar, so
    # Q_x^{n+1} = 2 d alpha Qbar / (1 + d alpha), Phi and Q_y unchanged
    nx, ny = 32, 16
    z = np.zeros((ny, nx))
    s = si.State(np.full((ny, nx), 8000.0), z.copy(), z.copy())
    p = si.Params(dt=900.0, absorber=2e-4, omega=0.0)
    qbar = np.full((ny, nx), 500.0)
    new, _ = si.si_step(nx, ny, s, s, z, (qbar, z), p, direct)
    d = 0.5 * p.dt
    alpha = absorber_profile(Grid(nx, ny).lat, p.absorber)[:, None]
    expect = 2.0 * d * alpha / (1.0 + d * alpha) * 500.0
    assert alpha.max() > 0 and (alpha == 0).any()
    assert np.abs(new.qx - expect).max() <= 1e-11 * 500.0
    assert np.abs(new.qy).max() <= 1e-11 * 500.0
    assert np.abs(new.phi - 8000.0).max() <= 1e-12 * 8000.0


def test_mass_is_conserved():
    nx, ny = 32, 16
    s = _rand_state(nx, ny, 4)
    s_old = _rand_state(nx, ny, 5)
    h0 = _orography(nx, ny, 4)
    rng = np.random.default_rng(6)
    qbar = (rng.normal(size=(ny, nx)) * 1e4, rng.normal(size=(ny, nx)) * 1e4)
    new, _ = si.si_step(nx, ny, s, s_old, h0, qbar, si.Params(dt=1200.0, absorber=1e-4), direct)
    G = np.cos(Grid(nx, ny).lat)[:, None]
    m0, m1 = (G * s.phi).sum(), (G * new.phi).sum()
    assert abs(m1 - m0) <= 1e-12 * m0
    assert np.abs(new.phi - s.phi).max() > 1e-3     # the state did change


def _mirror(f, sign=1.0):
    return sign * f[::-1].copy()


def test_equatorial_mirror_symmetry():
    nx, ny = 32, 16
    s = _rand_state(nx, ny, 7)
    s_old = _rand_state(nx, ny, 8)
    h0 = _orography(nx, ny, 7) * (1 + 0.3 * np.random.default_rng(9).uniform(size=(ny, nx)))
    rng = np.random.default_rng(10)
    qbar = (rng.normal(size=(ny, nx)) * 1e4, rng.normal(size=(ny, nx)) * 1e4)
    p = si.Params(dt=900.0, absorber=1e-4)
    a, _ = si.si_step(nx, ny, s, s_old, h0, qbar, p, direct)
    ms = si.State(_mirror(s.phi), _mirror(s.qx), _mirror(s.qy, -1.0))
    mo = si.State(_mirror(s_old.phi), _mirror(s_old.qx), _mirror(s_old.qy, -1.0))
    b, _ = si.si_step(nx, ny, ms, mo, _mirror(h0), (_mirror(qbar[0]), _mirror(qbar[1], -1.0)), p, direct)
    assert np.allclose(b.phi, _mirror(a.phi), rtol=1e-12, atol=0)
    qs = np.abs(a.qx).max()
    assert np.abs(b.qx - _mirror(a.qx)).max() <= 1e-10 * qs
    assert np.abs(b.qy - _mirror(a.qy, -1.0)).max() <= 1e-10 * qs
    assert np.abs(a.qy).max() > 1e-3 * qs           # not trivially symmetric


def test_longitude_shift_equivariance():
    nx, ny = 32, 16
    s = _rand_state(nx, ny, 11)
    h0 = _orography(nx, ny, 11)
    z = np.zeros((ny, nx))
    p = si.Params(dt=900.0)
    a, _ = si.si_step(nx, ny, s, s, h0, (z, z), p, direct)
    r = lambda f: np.roll(f, 5, axis=1)
    b, _ = si.si_step(nx, ny, si.State(r(s.phi), r(s.qx), r(s.qy)), si.State(r(s.phi), r(s.qx), r(s.qy)), r(h0),
                      (z, z), p, direct)
    assert np.allclose(b.phi, r(a.phi), rtol=1e-12, atol=0)
    qs = np.abs(a.qx).max()
    assert np.abs(b.qx - r(a.qx)).max() <= 1e-10 * qs
    assert np.abs(b.qy - r(a.qy)).max() <= 1e-10 * qs


def _jet_step(nx, ny, dt, omega=OMEGA):
    st = workloads.zonal_flow_state(nx, ny)
    z = np.zeros((ny, nx))
    s = si.State(st["phi"], st["qx"], st["qy"])
    new, _ = si.si_step(nx, ny, s, s, z, (z, z), si.Params(dt=dt, omega=omega), iterative)
    return s, new


def test_zonal_jet_stays_balanced():
    # the depth of the jet is in gradient-wind balance with u = u0 cos(lat):
    # pressure gradient, Coriolis and metric force cancel, so one step
    # leaves Q_y at truncation level (a dropped metric term gives ~ 400 here,
    # a flipped Coriolis sign ~ 2e4)
    s, new = _jet_step(128, 64, 450.0)
    assert np.abs(new.qy).max() < 40.0
    assert np.abs(new.qx - s.qx).max() < 2.0
    s, flipped = _jet_step(128, 64, 450.0, omega=-OMEGA)
    assert np.abs(flipped.qy).max() > 1e3


def test_zonal_jet_imbalance_converges():
    # dx and dt halve together: the one-step error dt * O(dx^2) drops ~8x
    errs = [np.abs(_jet_step(nx, nx // 2, 900.0 * 64 / nx)[1].qy).max() for nx in (64, 128, 256)]
    assert errs[0] / errs[1] > 6.0 and errs[1] / errs[2] > 6.0, errs


def test_momentum_satisfies_the_implicit_equation():
    # eq. Qexpr inverts Q^{n+1} = Qhat + dt/2 (f k x Q^{n+1} - alpha (Q^{n+1} - Qbar)
    # + 2 M^n - M^{n-1} - g/h (Phi grad(Phi + H0))_lin): check that residual
    nx, ny = 32, 16
    s = _rand_state(nx, ny, 12)
    s_old = _rand_state(nx, ny, 13)
    h0 = _orography(nx, ny, 12)
    rng = np.random.default_rng(14)
    qbar = (rng.normal(size=(ny, nx)) * 1e4, rng.normal(size=(ny, nx)) * 1e4)
    p = si.Params(dt=900.0, absorber=1e-4)
    new, ex = si.si_step(nx, ny, s, s_old, h0, qbar, p, direct)
    g = Grid(nx, ny)
    d = 0.5 * p.dt
    cos = np.cos(g.lat)[:, None]
    f = 2 * p.omega * np.sin(g.lat)[:, None]
    alpha = absorber_profile(g.lat, p.absorber)[:, None]
    # Qhat from the building blocks
    rx, ry = si.forcing(g, s, h0, qbar, p)
    vx, vy = si.cell_velocity(g, s, p.radius)
    vx0, vy0 = si.cell_velocity(g, s_old, p.radius)
    cx, cy = si.courant(g, 1.5 * vx - 0.5 * vx0, 1.5 * vy - 0.5 * vy0, p.dt)
    qhx = si.mpdata(g, s.qx + d * rx, cx, cy, -1.0)
    qhy = si.mpdata(g, s.qy + d * ry, cx, cy, -1.0)
    mx, my = si.metric(g, s, p.radius)
    mx0, my0 = si.metric(g, s_old, p.radius)
    ps = ex.phistar
    h0x, h0y = si._grad(g, h0)
    hx, hy = si._grad(g, ps + h0)
    px, py = si._grad(g, new.phi)
    prx = 0.5 * (ps * h0x + new.phi * hx + ps * px)
    pry = 0.5 * (ps * h0y + new.phi * hy + ps * py)
    resx = new.qx - qhx - d * (f * new.qy - alpha * (new.qx - qbar[0]) + 2 * mx - mx0 - p.g / (p.radius * cos) * prx)
    resy = new.qy - qhy - d * (-f * new.qx - alpha * (new.qy - qbar[1]) + 2 * my - my0 - p.g / p.radius * pry)
    scale = np.abs(new.qx).max()
    assert np.abs(resx).max() <= 1e-12 * scale
    assert np.abs(resy).max() <= 1e-12 * scale


def test_gpu_step_bounds_bite():
    # a dropped metric term in the oracle moves the new state far beyond the
    # bounds of the GPU step's parity tests
    nx, ny = 64, 32
    s, so, h0 = _rand_state(nx, ny, 94), _rand_state(nx, ny, 95), _orography(nx, ny, 94)
    z = np.zeros((ny, nx))
    p = si.Params(dt=900.0, absorber=1e-4)
    ref, _ = si.si_step(nx, ny, s, so, h0, (z, z), p, direct)
    orig = si.metric
    try:
        si.metric = lambda g, s, r=si.RADIUS: (0.0 * s.qx, 0.0 * s.qx)
        bad, _ = si.si_step(nx, ny, s, so, h0, (z, z), p, direct)
    finally:
        si.metric = orig
    assert np.abs(bad.phi - ref.phi).max() > 100 * TOL_PHI * np.abs(ref.phi).max()
    assert np.abs(bad.qy - ref.qy).max() > 100 * TOL_Q * np.abs(ref.qx).max()


def _linearised_step(nx, ny, p, depth=8000.0):
    """Jacobian of the step map (Phi^n, Q^n, Phi^{n-1}, Q^{n-1}) ->
    (Phi^{n+1}, Q^{n+1}, Phi^n, Q^n) about a fluid at rest over a flat
    surface, by one-sided differences (the map is smooth there to second
    order: MPDATA's |C| terms multiply differences of a uniform field)."""
    n = nx * ny
    z = np.zeros((ny, nx))

    def step(vec):
        f = vec.reshape(6, ny, nx)
        s = si.State(depth + f[0], f[1], f[2])
        so = si.State(depth + f[3], f[4], f[5])
        new, _ = si.si_step(nx, ny, s, so, z, (z, z), p, direct)
        return np.concatenate([(new.phi - depth).ravel(), new.qx.ravel(), new.qy.ravel(), f[0].ravel(),
                               f[1].ravel(), f[2].ravel()])

    base = step(np.zeros(6 * n))
    jac = np.empty((6 * n, 6 * n))
    for k in range(6 * n):
        e = np.zeros(6 * n)
        e[k] = 1e-4 if k % (3 * n) < n else 1e-4 * depth
        jac[:, k] = (step(e) - base) / e[k]
    return jac


def test_linear_gravity_waves_are_neutral_at_moderate_courant():
    # the trapezoidal integral of linear gravity waves (and of implicit
    # Coriolis) neither grows nor decays: spectral radius 1 while the
    # gravity-wave Courant number at the pole rows stays below ~1
    # (16x8, dt 1000 s: ~0.6)
    jac = _linearised_step(16, 8, si.Params(dt=1000.0, absorber=0.0))
    rho = np.abs(np.linalg.eigvals(jac)).max()
    assert abs(rho - 1.0) < 1e-6, rho


def test_half_weight_linearisation_grows_at_large_courant():
    # eq. rhslin puts half of the n+1 pressure gradient on the explicit
    # predictor Phi*; at a gravity-wave Courant number ~11 at the pole rows
    # (dt 20000 s on 16x8) the linearised step amplifies, as a Fourier
    # analysis of the linearised one-dimensional scheme predicts (growth
    # factors up to ~7 per step once c dt k exceeds ~3)
    jac = _linearised_step(16, 8, si.Params(dt=20000.0, omega=0.0, absorber=0.0))
    assert np.abs(np.linalg.eigvals(jac)).max() > 2.0
