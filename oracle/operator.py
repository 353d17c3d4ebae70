"""Elliptic operator of the semi-implicit shallow-water depth problem (oracle).

Paper, Section 2.1-2.2: the continuity equation in generalised transport form
(eq. SWE1) with h_x = a cos(lat), h_y = a, G = h_x h_y; the momentum forcings
(eqs. RSWE2, RSWE3); trapezoidal time integration (eq. MPDATA); the
linearised pressure gradient (eq. rhslin); the pointwise 2x2 inversion giving
Q = Qhathat + A grad(Phi) + B Phi (eq. Qexpr); and the resulting Helmholtz
problem L(Phi) - R = 0 (eq. Elliptic) with the generalised Laplacian

    L(Phi) = sum_I d_I ( sum_J A^IJ d_J Phi + B^I Phi ) - C Phi     (eq. L_Operator)

and residual r = L(Phi) - R (eq. Residual).

Coefficients (substituting the implicit momentum into the trapezoidal
continuity equation and multiplying by -2/dt).  With delta = dt/2,
gamma = 1 + delta*alpha, b = delta*f, D = gamma^2 + b^2, H* = Phi* + H0 and
kappa = delta*g*Phi*/(2 D):

    A^xx = kappa*gamma/cos(lat)      A^xy = kappa*b
    A^yx = -kappa*b                  A^yy = kappa*gamma*cos(lat)
    B^x  = delta*g/(2D) * ( gamma/cos(lat) dH*/dlon + b dH*/dlat )
    B^y  = delta*g/(2D) * ( -b dH*/dlon + gamma*cos(lat) dH*/dlat )
    C    = 2 a^2 cos(lat) / dt

The paper prints no discrete stencil.  Reading used here (compact flux form
on the collocated grid):

* fluxes live on cell faces; coefficient factors that depend on latitude
  (cos, f, alpha) are evaluated analytically at the face latitude, Phi* and
  H* are averaged across the face, face gradients of H* use the same
  differences as those of Phi;
* east-face flux  F^x = A^xx dPhi/dlon + A^xy <dPhi/dlat> + B^x <Phi>,
  north-face flux F^y = A^yy dPhi/dlat + A^yx <dPhi/dlon> + B^y <Phi>,
  where <d/dlat> at an east face averages the two central differences of the
  adjacent columns (and <d/dlon> likewise at a north face), giving a 9-point
  stencil;
* longitude is periodic; the rows beyond the poles are the polar rows seen
  across the pole, i.e. shifted by NX/2 in longitude; the meridional flux
  through each pole (a point, h_x = 0) is zero.

Units are SI throughout: Phi in m, dt in s, a in m.
"""
from __future__ import annotations

import numpy as np

RADIUS = 6.371e6        # m; reproduces the pole-row spacings printed in Section 3.2
GRAVITY = 9.80616       # m s^-2; sqrt(g * 8 km) = 280 m/s as quoted in Section 3.2
OMEGA = 7.292e-5        # s^-1; Earth's rotation rate (f = 2 Omega sin(lat))


def absorber_profile(lat, alpha_max):
    """Polar absorber inverse time scale (Section 3.2): zero at angular
    distance >= 3*pi/64 from a pole, rising linearly to alpha_max at the pole."""
    dist = 0.5 * np.pi - np.abs(lat)
    width = 3.0 * np.pi / 64.0
    return alpha_max * np.maximum(0.0, 1.0 - dist / width)


class Grid:
    """Regular collocated lon/lat grid with cell-centred rows (no point on a pole)."""

    def __init__(self, nx: int, ny: int):
        if nx < 4 or nx % 2:
            raise ValueError("nx must be even and >= 4")
        if ny < 2:
            raise ValueError("ny must be >= 2")
        self.nx, self.ny = nx, ny
        self.dlam = 2.0 * np.pi / nx
        self.dphi = np.pi / ny
        self.lam = np.arange(nx) * self.dlam
        self.lat = -0.5 * np.pi + (np.arange(ny) + 0.5) * self.dphi
        # interior north faces j+1/2, j = 0..ny-2
        self.lat_n = -0.5 * np.pi + (np.arange(ny - 1) + 1.0) * self.dphi

    def pole_row_spacing(self, radius=RADIUS):
        """Zonal grid length in the rows next to the poles, a*dlam*cos(lat_0)."""
        return radius * self.dlam * np.cos(self.lat[0])


def across_pole_extend(f):
    """[ny][nx] -> [ny+2][nx]: row -1 is row 0 and row ny is row ny-1, each
    seen across the pole (shifted by NX/2 in longitude)."""
    nx = f.shape[1]
    south = np.roll(f[0], nx // 2)
    north = np.roll(f[-1], nx // 2)
    return np.vstack([south[None, :], f, north[None, :]])


def _dlat_at_east(f, dphi):
    """<dF/dlat> at east faces (i+1/2, j): mean of the central differences of
    columns i and i+1, ghost rows across the poles."""
    e = across_pole_extend(f)
    d = e[2:] - e[:-2]
    return (d + np.roll(d, -1, axis=1)) / (4.0 * dphi)


def _dlon_at_north(f, dlam):
    """<dF/dlon> at interior north faces (i, j+1/2): mean of the central
    differences of rows j and j+1.  Shape [ny-1][nx]."""
    d = np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)
    return (d[:-1] + d[1:]) / (4.0 * dlam)


class EllipticOperator:
    """Discrete L of eq. L_Operator for one solve, built from the explicit depth
    predictor Phi* (eq. rhslin), orography H0 and the physical parameters."""

    def __init__(self, nx, ny, depth, dt, orography=None, absorber=0.0,
                 g=GRAVITY, omega=OMEGA, radius=RADIUS, b_terms=True):
        grid = Grid(nx, ny)
        self.grid = grid
        self.dt, self.g, self.omega, self.radius = float(dt), float(g), float(omega), float(radius)
        depth = np.asarray(depth, dtype=np.float64).reshape(ny, nx)
        h0 = np.zeros_like(depth) if orography is None else np.asarray(orography, np.float64).reshape(ny, nx)
        hstar = depth + h0
        delta = 0.5 * self.dt

        def latitude_factors(lat):
            gamma = 1.0 + delta * absorber_profile(lat, absorber)
            b = delta * 2.0 * omega * np.sin(lat)
            return gamma, b, gamma * gamma + b * b

        # east faces: latitude of the row
        gam, b, D = latitude_factors(grid.lat)
        cos = np.cos(grid.lat)
        phistar_e = 0.5 * (depth + np.roll(depth, -1, axis=1))
        kappa_e = delta * g * phistar_e / (2.0 * D[:, None])
        self.axx_e = kappa_e * (gam / cos)[:, None]
        self.axy_e = kappa_e * b[:, None]
        if b_terms:
            dhl = (np.roll(hstar, -1, axis=1) - hstar) / grid.dlam
            dhp = _dlat_at_east(hstar, grid.dphi)
            self.bx_e = (delta * g / (2.0 * D))[:, None] * ((gam / cos)[:, None] * dhl + b[:, None] * dhp)
        else:
            self.bx_e = np.zeros_like(depth)

        # interior north faces
        gam_n, b_n, D_n = latitude_factors(grid.lat_n)
        cos_n = np.cos(grid.lat_n)
        phistar_n = 0.5 * (depth[:-1] + depth[1:])
        kappa_n = delta * g * phistar_n / (2.0 * D_n[:, None])
        self.ayy_n = kappa_n * (gam_n * cos_n)[:, None]
        self.ayx_n = -kappa_n * b_n[:, None]
        if b_terms:
            dhp_n = (hstar[1:] - hstar[:-1]) / grid.dphi
            dhl_n = _dlon_at_north(hstar, grid.dlam)
            self.by_n = (delta * g / (2.0 * D_n))[:, None] * (-b_n[:, None] * dhl_n + (gam_n * cos_n)[:, None] * dhp_n)
        else:
            self.by_n = np.zeros((ny - 1, nx))

        self.c = 2.0 * radius * radius * cos / self.dt   # Helmholtz coefficient per row

    # ---- L --------------------------------------------------------------
    def fluxes(self, phi):
        g = self.grid
        fx = (self.axx_e * (np.roll(phi, -1, axis=1) - phi) / g.dlam
              + self.axy_e * _dlat_at_east(phi, g.dphi)
              + self.bx_e * 0.5 * (phi + np.roll(phi, -1, axis=1)))
        fy_int = (self.ayy_n * (phi[1:] - phi[:-1]) / g.dphi
                  + self.ayx_n * _dlon_at_north(phi, g.dlam)
                  + self.by_n * 0.5 * (phi[:-1] + phi[1:]))
        zero = np.zeros((1, g.nx))
        fy = np.vstack([zero, fy_int, zero])          # pole faces carry no flux
        return fx, fy

    def apply(self, phi):
        """L(phi) for phi[ny][nx] (float64)."""
        g = self.grid
        phi = np.asarray(phi, dtype=np.float64).reshape(g.ny, g.nx)
        fx, fy = self.fluxes(phi)
        return ((fx - np.roll(fx, 1, axis=1)) / g.dlam
                + (fy[1:] - fy[:-1]) / g.dphi
                - self.c[:, None] * phi)

    def residual(self, phi, rhs):
        """r = L(phi) - R (eq. Residual)."""
        return self.apply(phi) - rhs

    # ---- pieces used by the preconditioners -----------------------------
    def ayy_north_south(self):
        """A^yy on the north and south face of every cell, [ny][nx] each;
        the pole faces are zero."""
        ny, nx = self.grid.ny, self.grid.nx
        zero = np.zeros((1, nx))
        north = np.vstack([self.ayy_n, zero])
        south = np.vstack([zero, self.ayy_n])
        return north, south

    def diagonal(self):
        """Diagonal of L (coefficient of phi_ij in L(phi)_ij)."""
        g = self.grid
        axx_w = np.roll(self.axx_e, 1, axis=1)
        bx_w = np.roll(self.bx_e, 1, axis=1)
        ayy_n, ayy_s = self.ayy_north_south()
        zero = np.zeros((1, g.nx))
        by_n = np.vstack([self.by_n, zero])
        by_s = np.vstack([zero, self.by_n])
        return (-(self.axx_e + axx_w) / g.dlam ** 2
                - (ayy_n + ayy_s) / g.dphi ** 2
                + (self.bx_e - bx_w) / (2.0 * g.dlam)
                + (by_n - by_s) / (2.0 * g.dphi)
                - self.c[:, None])

    def dense(self):
        """Dense matrix of L by applying it to every unit vector (tiny grids)."""
        n = self.grid.nx * self.grid.ny
        m = np.empty((n, n))
        u = np.zeros(n)
        for col in range(n):
            u[col] = 1.0
            m[:, col] = self.apply(u).ravel()
            u[col] = 0.0
        return m
