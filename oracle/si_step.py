"""One semi-implicit time step of the shallow-water model around the
elliptic solve (oracle), paper Sections 2.1-2.2: eqs. SWE1-SWE3 (generalised
transport form), RSWE2-RSWE3 (forcings), MPDATA (trapezoidal integral with
the MPDATA operator as its explicit part), rhslin (linearised pressure
gradient), Qexpr (pointwise inversion), Elliptic / L_Operator and vadv.

Test infrastructure: only the tests use this module.

Variables on the collocated grid of oracle.operator: fluid thickness Phi (m),
momenta Q_x = Phi xdot h_x and Q_y = Phi ydot h_y (Phi times the zonal and
meridional velocity, m^2/s), orography H0, and the relaxation target Qbar
with the inverse time scale alpha of the polar absorber.  h_x = a cos(lat),
h_y = a, G = h_x h_y; the advective velocity (eq. vadv) is
v = (Q_x h_y, Q_y h_x) / Phi, and v Phi = (a Q_x, a cos(lat) Q_y) is the mass
flux of eq. SWE1.

A step n -> n+1 (`si_step`):
1. the forcings R^n of eqs. RSWE2-RSWE3 at the cell centres;
2. the advective velocity at n + 1/2 by linear extrapolation from n and n-1
   (an O(dt^2) explicit predictor), averaged to the cell faces as Courant
   numbers;
3. the explicit part: Phi* = MPDATA(Phi^n) (eq. rhslin's predictor) and
   Qhat = MPDATA(Q^n + dt/2 R^n) (eq. MPDATA's first term);
4. the implicit part of eq. MPDATA with the pressure gradient of eq. rhslin,
   Coriolis and relaxation at n+1 and the metric forces extrapolated from n
   and n-1, inverted pointwise (eq. Qexpr): Q^{n+1} = Qhathat + A grad Phi^{n+1}
   + B Phi^{n+1};
5. the trapezoidal integral of eq. SWE1 with (4) substituted: the elliptic
   problem L(Phi^{n+1}) = R (oracle.operator's L with Phi* and H0), whose
   right-hand side is R = D(F^n) + D(Fhathat) - C Phi^n, F the mass flux and D
   the discrete divergence of the operator's face fluxes;
6. Q^{n+1} from (4) with the solved Phi^{n+1} (eq. Qexpr), and so v^{n+1}.

Readings (the paper cites MPDATA and its predictors but prints neither):
* MPDATA: one donor-cell pass and one corrective pass with the standard
  two-dimensional antidiffusive pseudo-velocity in Courant-number form with
  the Jacobian (Smolarkiewicz 1984; Smolarkiewicz & Margolin 1998), using |psi|
  in the ratios (the variant for fields of either sign); no non-oscillatory
  limiter.  G is normalised by a^2 (G = cos(lat)), Courant numbers are
  C^x = v_x dt / (a^2 dlam), C^y = v_y dt / (a^2 dphi).
* Face velocities are the means of the two cell values; no flux through the
  pole faces.  Across a pole the momenta change sign (the row beyond the
  pole, seen from the other side, moves the other way); Phi does not.
* Cell-centred gradients are central differences (rows across the poles as
  in the operator); the face fluxes of the explicit momenta in (5) are the
  means of the two cell values, as the operator averages Phi* at faces.
* The metric forces are extrapolated as 2 M^n - M^{n-1}; Qbar is given.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .operator import EllipticOperator, Grid, across_pole_extend, absorber_profile, RADIUS, GRAVITY, OMEGA

EPS_RATIO = 1e-300     # keeps the MPDATA ratios finite where |psi| vanishes


@dataclass
class State:
    phi: np.ndarray        # [ny][nx]
    qx: np.ndarray
    qy: np.ndarray


def _ext(f, sign):
    """[ny+2][nx]: rows beyond the poles seen across the pole, times `sign`."""
    e = across_pole_extend(f)
    e[0] *= sign
    e[-1] *= sign
    return e


def cell_velocity(grid: Grid, s: State, radius=RADIUS):
    """eq. vadv divided by a^2: (Q_x / (a Phi), cos(lat) Q_y / (a Phi))."""
    cos = np.cos(grid.lat)[:, None]
    return s.qx / (radius * s.phi), cos * s.qy / (radius * s.phi)


def courant(grid: Grid, vx, vy, dt):
    """Face Courant numbers: x faces [ny][nx] (face i+1/2), y faces [ny+1][nx]
    (face j-1/2, the first and last are the poles and carry zero)."""
    cx = 0.5 * (vx + np.roll(vx, -1, axis=1)) * dt / grid.dlam
    cy = np.zeros((grid.ny + 1, grid.nx))
    cy[1:-1] = 0.5 * (vy[:-1] + vy[1:]) * dt / grid.dphi
    return cx, cy


def _upwind(grid: Grid, psi, cx, cy):
    """Donor-cell pass of G psi_t + div(v psi) = 0 in flux form."""
    g = np.cos(grid.lat)[:, None]
    fx = np.maximum(cx, 0.0) * psi + np.minimum(cx, 0.0) * np.roll(psi, -1, axis=1)
    fy = np.zeros((grid.ny + 1, grid.nx))
    fy[1:-1] = np.maximum(cy[1:-1], 0.0) * psi[:-1] + np.minimum(cy[1:-1], 0.0) * psi[1:]
    return psi - ((fx - np.roll(fx, 1, axis=1)) + (fy[1:] - fy[:-1])) / g


def _antidiffusive(grid: Grid, psi, cx, cy, sign):
    """Antidiffusive Courant numbers of the corrective pass."""
    g = np.cos(grid.lat)
    gy = np.zeros(grid.ny + 1)
    gy[1:-1] = np.cos(grid.lat_n)
    a = np.abs(_ext(psi, sign))                      # |psi| on rows -1 .. ny
    c = a[1:-1]
    east = np.roll(c, -1, axis=1)
    ax = (east - c) / (east + c + EPS_RATIO)
    up, dn = a[2:], a[:-2]                           # rows j+1, j-1
    num = (up + np.roll(up, -1, axis=1)) - (dn + np.roll(dn, -1, axis=1))
    den = (up + np.roll(up, -1, axis=1)) + (dn + np.roll(dn, -1, axis=1))
    bx = 0.5 * num / (den + EPS_RATIO)
    cyb = 0.25 * (cy[1:] + np.roll(cy[1:], -1, axis=1) + cy[:-1] + np.roll(cy[:-1], -1, axis=1))
    gx = g[:, None]
    acx = (np.abs(cx) - cx * cx / gx) * ax - cx * cyb / gx * bx
    # y faces j+1/2 between rows j and j+1 (interior faces only)
    lo, hi = c[:-1], c[1:]
    ay = (hi - lo) / (hi + lo + EPS_RATIO)
    num = (np.roll(hi, -1, axis=1) + np.roll(lo, -1, axis=1)) - (np.roll(hi, 1, axis=1) + np.roll(lo, 1, axis=1))
    den = (np.roll(hi, -1, axis=1) + np.roll(lo, -1, axis=1)) + (np.roll(hi, 1, axis=1) + np.roll(lo, 1, axis=1))
    by = 0.5 * num / (den + EPS_RATIO)
    cxb = 0.25 * (cx[:-1] + np.roll(cx[:-1], 1, axis=1) + cx[1:] + np.roll(cx[1:], 1, axis=1))
    cyi = cy[1:-1]
    gyi = gy[1:-1][:, None]
    acy = np.zeros_like(cy)
    acy[1:-1] = (np.abs(cyi) - cyi * cyi / gyi) * ay - cyi * cxb / gyi * by
    return acx, acy


def mpdata(grid: Grid, psi, cx, cy, sign=1.0):
    """MPDATA: donor cell, then one corrective pass with the antidiffusive
    Courant numbers of the first pass's result.  sign: -1 for a momentum
    component (it changes sign across a pole)."""
    p1 = _upwind(grid, psi, cx, cy)
    acx, acy = _antidiffusive(grid, p1, cx, cy, sign)
    return _upwind(grid, p1, acx, acy)


def _grad(grid: Grid, f, sign=1.0):
    """Central-difference gradient at cell centres (d/dlam, d/dlat)."""
    e = _ext(f, sign)
    return ((np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)) / (2.0 * grid.dlam),
            (e[2:] - e[:-2]) / (2.0 * grid.dphi))


@dataclass
class Params:
    dt: float
    g: float = GRAVITY
    omega: float = OMEGA
    radius: float = RADIUS
    absorber: float = 0.0          # alpha_max of the polar absorber (also in the operator)


def metric(grid: Grid, s: State, radius=RADIUS):
    """Metric forces of eqs. RSWE2-RSWE3 with h_y = a, dh_x/dlat = -a sin(lat):
    (tan(lat) Q_x Q_y, -tan(lat) Q_x^2) / (a Phi)."""
    t = np.tan(grid.lat)[:, None]
    return t * s.qx * s.qy / (radius * s.phi), -t * s.qx * s.qx / (radius * s.phi)


def forcing(grid: Grid, s: State, h0, qbar, p: Params):
    """R^n of eqs. RSWE2-RSWE3 at the cell centres."""
    cos = np.cos(grid.lat)[:, None]
    f = 2.0 * p.omega * np.sin(grid.lat)[:, None]
    alpha = absorber_profile(grid.lat, p.absorber)[:, None]
    hx, hy = _grad(grid, s.phi + h0)
    mx, my = metric(grid, s, p.radius)
    rx = -p.g / (p.radius * cos) * s.phi * hx + f * s.qy + mx - alpha * (s.qx - qbar[0])
    ry = -p.g / p.radius * s.phi * hy - f * s.qx + my - alpha * (s.qy - qbar[1])
    return rx, ry


def mass_flux_divergence(grid: Grid, qx, qy, radius=RADIUS):
    """D(F) of the mass flux F = (a Q_x, a cos(lat) Q_y) with face values the
    means of the two cells and no flux through the poles."""
    fx = radius * 0.5 * (qx + np.roll(qx, -1, axis=1))
    fy = np.zeros((grid.ny + 1, grid.nx))
    fy[1:-1] = radius * np.cos(grid.lat_n)[:, None] * 0.5 * (qy[:-1] + qy[1:])
    return (fx - np.roll(fx, 1, axis=1)) / grid.dlam + (fy[1:] - fy[:-1]) / grid.dphi


@dataclass
class Explicit:
    phistar: np.ndarray
    qhh: tuple             # Qhathat (x, y)
    rhs: np.ndarray        # R of the elliptic problem
    op: EllipticOperator


def explicit_part(grid_nx, grid_ny, s: State, s_old: State, h0, qbar, p: Params) -> Explicit:
    """Steps 1-5: Phi*, Qhathat and the elliptic problem (operator and R)."""
    grid = Grid(grid_nx, grid_ny)
    cos = np.cos(grid.lat)[:, None]
    d = 0.5 * p.dt
    rx, ry = forcing(grid, s, h0, qbar, p)
    vx, vy = cell_velocity(grid, s, p.radius)
    vx0, vy0 = cell_velocity(grid, s_old, p.radius)
    cx, cy = courant(grid, 1.5 * vx - 0.5 * vx0, 1.5 * vy - 0.5 * vy0, p.dt)
    phistar = mpdata(grid, s.phi, cx, cy, 1.0)
    qhx = mpdata(grid, s.qx + d * rx, cx, cy, -1.0)
    qhy = mpdata(grid, s.qy + d * ry, cx, cy, -1.0)
    # implicit part: Coriolis and relaxation at n+1, metric extrapolated, the
    # known half of the linearised pressure gradient (Phi* grad H0)
    alpha = absorber_profile(grid.lat, p.absorber)[:, None]
    gam = 1.0 + d * alpha
    b = d * 2.0 * p.omega * np.sin(grid.lat)[:, None]
    D = gam * gam + b * b
    mx, my = metric(grid, s, p.radius)
    mx0, my0 = metric(grid, s_old, p.radius)
    h0x, h0y = _grad(grid, h0)
    ex = qhx + d * (alpha * qbar[0] + 2.0 * mx - mx0) - d * p.g / (p.radius * cos) * 0.5 * phistar * h0x
    ey = qhy + d * (alpha * qbar[1] + 2.0 * my - my0) - d * p.g / p.radius * 0.5 * phistar * h0y
    qhh = ((gam * ex + b * ey) / D, (-b * ex + gam * ey) / D)
    op = EllipticOperator(grid_nx, grid_ny, phistar, p.dt, orography=h0, absorber=p.absorber, g=p.g,
                          omega=p.omega, radius=p.radius)
    rhs = (mass_flux_divergence(grid, s.qx, s.qy, p.radius) + mass_flux_divergence(grid, *qhh, p.radius)
           - op.c[:, None] * s.phi)
    return Explicit(phistar, qhh, rhs, op)


def recover_momentum(grid_nx, grid_ny, ex: Explicit, phi_new, h0, p: Params):
    """Step 6, eq. Qexpr: Q^{n+1} = Qhathat + A grad Phi^{n+1} + B Phi^{n+1}."""
    grid = Grid(grid_nx, grid_ny)
    cos = np.cos(grid.lat)[:, None]
    d = 0.5 * p.dt
    alpha = absorber_profile(grid.lat, p.absorber)[:, None]
    gam = 1.0 + d * alpha
    b = d * 2.0 * p.omega * np.sin(grid.lat)[:, None]
    D = gam * gam + b * b
    px, py = _grad(grid, phi_new)
    hx, hy = _grad(grid, ex.phistar + h0)
    # the unknown half of eq. rhslin: Phi^{n+1} grad H* + Phi* grad Phi^{n+1}
    ux = -d * p.g / (p.radius * cos) * 0.5 * (phi_new * hx + ex.phistar * px)
    uy = -d * p.g / p.radius * 0.5 * (phi_new * hy + ex.phistar * py)
    return (ex.qhh[0] + (gam * ux + b * uy) / D, ex.qhh[1] + (-b * ux + gam * uy) / D)


def si_step(nx, ny, s: State, s_old: State, h0, qbar, p: Params, solve):
    """One step: returns (State at n+1, Explicit).  `solve(op, rhs, x0)` solves
    L(x) = rhs (the oracle's GCR, or any solver under test)."""
    ex = explicit_part(nx, ny, s, s_old, h0, qbar, p)
    phi_new = solve(ex.op, ex.rhs, s.phi)
    qx, qy = recover_momentum(nx, ny, ex, phi_new, h0, p)
    return State(phi_new, qx, qy), ex
