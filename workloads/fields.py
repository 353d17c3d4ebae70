"""Random smooth fields on a regular longitude/latitude grid.

The paper's experiments run on regular lon/lat grids of NX x NY points
(128x64, 256x128, 512x256) with a mean depth of 8 km (Section 3).  Its test
cases (a Rossby-Haurwitz wave and flow over Earth orography) need data that is
not available here, so every workload is synthetic: real spherical-harmonic
series with standard-normal coefficients, which are smooth on the sphere
(no pole artefacts) and have a controlled spectral content.

Grid convention (shared with every consumer, restated independently by each):
longitude  lambda_i = i * 2*pi/NX,  latitude  phi_j = -pi/2 + (j + 1/2) * pi/NY,
arrays are [NY][NX] row-major, longitude contiguous, row 0 southernmost.
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y

CONFIG_SEED_BASE = 2103


def cell_centres(nx: int, ny: int):
    """Longitudes (nx,) and latitudes (ny,) of the cell centres, radians."""
    lam = np.arange(nx, dtype=np.float64) * (2.0 * np.pi / nx)
    phi = -0.5 * np.pi + (np.arange(ny, dtype=np.float64) + 0.5) * (np.pi / ny)
    return lam, phi


_LEGENDRE_CACHE = {}


def _legendre_table(ny, lmax):
    """Y_lm(colatitude, lambda = 0) for l <= lmax, m <= l at the row latitudes:
    the fully normalised associated Legendre functions (real for lambda = 0)."""
    key = (ny, lmax)
    tab = _LEGENDRE_CACHE.get(key)
    if tab is None:
        _, phi = cell_centres(2, ny)
        theta = 0.5 * np.pi - phi
        tab = np.zeros((lmax + 1, lmax + 1, ny))
        for l in range(lmax + 1):
            for m in range(l + 1):
                tab[l, m] = sph_harm_y(l, m, theta, 0.0).real
        _LEGENDRE_CACHE[key] = tab
    return tab


def harmonic_field(nx, ny, lmax, rng, lmin=0, amplitude=1.0, lam_shift=0.0):
    """Real spherical-harmonic series sum_{l=lmin..lmax} sum_m (a cos + b sin),
    coefficients N(0,1) drawn in (l up, m up, cos then sin) order, sampled at
    the cell centres and rescaled so that max|field| == amplitude.  The m > 0
    terms carry the factor sqrt(2) of the orthonormal real harmonics.

    ``lam_shift`` evaluates the same series at longitude (lambda - lam_shift),
    i.e. the pattern advected eastward by lam_shift radians.
    """
    lam, _ = cell_centres(nx, ny)
    lam = lam - lam_shift
    tab = _legendre_table(ny, lmax)
    # field = sum_m [ A_m(lat) cos(m lam) + B_m(lat) sin(m lam) ]
    A = np.zeros((lmax + 1, ny))
    Bc = np.zeros((lmax + 1, ny))
    for l in range(lmin, lmax + 1):
        for m in range(0, l + 1):
            a = rng.standard_normal()
            if m == 0:
                A[0] += a * tab[l, 0]
            else:
                b = rng.standard_normal()
                A[m] += np.sqrt(2.0) * a * tab[l, m]
                Bc[m] += np.sqrt(2.0) * b * tab[l, m]
    ms = np.arange(lmax + 1)[:, None]
    field = A.T @ np.cos(ms * lam[None, :]) + Bc.T @ np.sin(ms * lam[None, :])
    peak = np.max(np.abs(field))
    if peak == 0.0:
        return field
    return field * (amplitude / peak)


def _seed(config: int, instance: int) -> int:
    return CONFIG_SEED_BASE + 1000 * config + instance


def problem(config: int, nx: int, ny: int, instance: int = 0, dt: float | None = None,
            depth_mean=8000.0, depth_amp=500.0, depth_lmax=8, sol_lmax=12):
    """One solve of the configuration family: depth field, time step, and the
    field whose operator image becomes the right-hand side.

    Returns dict(nx, ny, dt, depth[ny,nx], x_true[ny,nx], seed).  The depth is
    depth_mean + depth_amp * (harmonic series of degree 1..depth_lmax with max 1);
    x_true is a degree 0..sol_lmax series with max|x_true| = 1.
    """
    seed = _seed(config, instance)
    rng = np.random.default_rng(seed)
    depth = depth_mean + harmonic_field(nx, ny, depth_lmax, rng, lmin=1, amplitude=depth_amp)
    x_true = harmonic_field(nx, ny, sol_lmax, rng, lmin=0, amplitude=1.0)
    return dict(nx=nx, ny=ny, dt=600.0 if dt is None else float(dt), depth=depth,
                x_true=x_true, seed=seed)


def batch_problems(config: int, count: int, grids=((128, 64), (256, 128), (512, 256)),
                   dt_range=(300.0, 1200.0), depth_range=(4000.0, 10000.0)):
    """Independent solves of uneven sizes: grid drawn uniformly from ``grids``,
    dt uniform in ``dt_range``, depth = mid + half-range * Psi_8 / max|Psi_8|
    so that it spans ``depth_range``; each member has its own x_true."""
    rng = np.random.default_rng(_seed(config, 999))
    out = []
    mid = 0.5 * (depth_range[0] + depth_range[1])
    half = 0.5 * (depth_range[1] - depth_range[0])
    for n in range(count):
        nx, ny = grids[int(rng.integers(len(grids)))]
        dt = float(rng.uniform(*dt_range))
        p = problem(config, nx, ny, instance=n, dt=dt, depth_mean=mid, depth_amp=half)
        out.append(p)
    return out


# Zonal jet used for the time-stepping sequence.  Earth constants are inputs of
# the workload here (they set the jet's balanced depth), not solver arithmetic.
_A = 6.371e6
_G = 9.80616
_OMEGA = 7.292e-5


def jet_sequence_depth(nx, ny, step, dt, u0=40.0, pert_amp=200.0, pert_lmax=16,
                       seed_instance=0, config=5):
    """Depth field of step ``step`` of a sequence: a zonal jet u = u0 cos(lat) in
    gradient-wind balance, h = 8000 - (a*Omega*u0 + u0^2/2) sin^2(lat) / g, plus a
    degree <= pert_lmax perturbation of amplitude pert_amp advected eastward at
    u0 (solid-body rotation by u0*step*dt/a radians)."""
    lam, phi = cell_centres(nx, ny)
    h = 8000.0 - (_A * _OMEGA * u0 + 0.5 * u0 * u0) * np.sin(phi) ** 2 / _G
    rng = np.random.default_rng(_seed(config, seed_instance))
    shift = u0 * step * dt / _A
    pert = harmonic_field(nx, ny, pert_lmax, rng, lmin=1, amplitude=pert_amp, lam_shift=shift)
    return h[:, None] + pert


def zonal_flow_state(nx, ny, u0=40.0, pert_amp=0.0, pert_lmax=16, seed_instance=0, config=6):
    """A state of the shallow-water model for the semi-implicit step: the
    zonal jet u = u0 cos(lat) with the depth of jet_sequence_depth (gradient-
    wind balance, plus a degree <= pert_lmax perturbation of amplitude
    pert_amp), v = 0.  Returns dict(phi, qx, qy) with Q = Phi * velocity."""
    lam, phi = cell_centres(nx, ny)
    h = 8000.0 - (_A * _OMEGA * u0 + 0.5 * u0 * u0) * np.sin(phi) ** 2 / _G
    depth = np.repeat(h[:, None], nx, axis=1)
    if pert_amp > 0:
        rng = np.random.default_rng(_seed(config, seed_instance))
        depth = depth + harmonic_field(nx, ny, pert_lmax, rng, lmin=1, amplitude=pert_amp)
    u = u0 * np.cos(phi)[:, None] * np.ones((1, nx))
    return dict(phi=depth, qx=depth * u, qy=np.zeros_like(depth))


def model_state(nx, ny, instance=0, u0=40.0, pert_amp=100.0, pert_lmax=16, oro_amp=2000.0, oro_lmax=8, config=7):
    """A state over synthetic mountains for the semi-implicit step: the zonal
    jet of zonal_flow_state with its balanced free surface, orography H0 =
    oro_amp * (degree <= oro_lmax series mapped onto [0, 1]) under it (the
    fluid thins over the mountains, Phi = surface - H0), plus a degree <=
    pert_lmax perturbation of the depth.  Returns dict(phi, qx, qy, orography)."""
    rng = np.random.default_rng(_seed(config, instance))
    base = zonal_flow_state(nx, ny, u0=u0)
    f = harmonic_field(nx, ny, oro_lmax, rng, lmin=1, amplitude=1.0)
    h0 = oro_amp * (f - f.min()) / (f.max() - f.min())
    depth = base["phi"] - h0 + harmonic_field(nx, ny, pert_lmax, rng, lmin=1, amplitude=pert_amp)
    u = base["qx"] / base["phi"]
    return dict(phi=depth, qx=depth * u, qy=np.zeros_like(depth), orography=h0)

