"""Emulated reduced precision (oracle), paper Sections 3.3 (reduced-precision
experiments), 4.2.1 (single-precision initial residual) and 4.3 (the
mixed-precision solver with half precision).

Test infrastructure: only the tests, the smoke check, the benchmark's CPU
baseline and the measurement drivers' comparisons use this package.

The paper emulates half precision in software: the significand keeps 10
explicit bits, as IEEE half does, but the exponent keeps double precision's 11
bits, so only the significand is rounded and the range stays that of
float64 (no overflow beyond 65504, no subnormals below 2^-14).
`rpe_round(x, 10)` does that on float64 values.

The half-precision mixed solver of Section 4.3, as emulated here
(`gcr_half`):
* step 1: r_0 in single precision with the split evaluation of Section
  4.2.1 (float32 base and correction, float64 polar bands);
* steps 1 and 3: the preconditioner and the operator L in half precision --
  every arithmetic result rounded to half -- except the last operation of L,
  the subtraction of C Phi (single precision), and the rows within `polar`
  rows of either pole, where both run in single precision;
* step 2: the residual update and the accumulation of the solver increments
  Delta Phi in single precision; global sums (beta, alpha, ||r||) in single
  precision;
* step 4: p_{nu+1} = e + sum alpha_l p_l in half precision, L(p_{nu+1}) in
  single precision;
* at exit Phi = Phi_0 + Delta Phi (float64) and its residual in float64.

Readings (the paper does not say):
* the emulator's tie rule: round to nearest, ties to even (IEEE's default);
* each arithmetic operation rounds its result ("half precision arithmetic");
  stored inputs (coefficients, fields) are rounded once when first used; the
  grid factors dlam, dphi are rounded like any other input;
* the order of operations is the operator's flux form: face fluxes
  A dPhi/dlam + <A dPhi/dlat> + B <Phi>, then their divergence (the oracle's
  `EllipticOperator.fluxes` and `apply`);
* the row systems are solved by the Thomas algorithm for a cyclic
  tridiagonal system (Sherman-Morrison correction of the two corner
  entries), the textbook direct method for such rows;
* single-precision global sums are float32 sums of float32 products (numpy's
  float32 summation).
With rounding switched off (`exact`) every function equals its float64
oracle counterpart up to float64 rounding: the pin of the formulas.
"""
from __future__ import annotations

import numpy as np

from .operator import EllipticOperator, across_pole_extend
from .gcr import GCRResult, CONVERGED, NOT_CONVERGED, STAGNATED
from .split import split_fields, base_differences, residual_split

HALF_BITS = 10      # explicit significand bits of half precision


def rpe_round(x, sbits=HALF_BITS):
    """Round float64 values to `sbits` explicit significand bits, ties to
    even, keeping float64's exponent range (zeros, infinities and NaN pass)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m * 2^e, 0.5 <= |m| < 1
    scale = float(2 ** (sbits + 1))          # m has sbits + 1 significant bits after rounding
    return np.ldexp(np.rint(m * scale) / scale, e)


def half(x):
    return rpe_round(x, HALF_BITS)


def single(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def exact(x):
    return np.asarray(x, dtype=np.float64)


def polar_mask(ny, polar):
    j = np.arange(ny)
    return (j < polar) | (j >= ny - polar)


def _select(a_in, a_pol, mask):
    out = np.array(a_in, copy=True)
    out[mask] = a_pol[mask]
    return out


def _divergence(op: EllipticOperator, phi, R, zonal=True):
    """sum of the flux divergences of L(phi) with every operation rounded by
    R: with zonal=False the A^xx part is left out (the meridional, cross and
    B terms: P^M without the Helmholtz term)."""
    g = op.grid
    dl, dp = R(g.dlam), R(g.dphi)
    four_dl, four_dp, hlf = R(4.0 * dl), R(4.0 * dp), R(0.5)
    phi = R(phi)
    east = np.roll(phi, -1, axis=1)
    ex = across_pole_extend(phi)
    d = R(ex[2:] - ex[:-2])
    lat_e = R(d + np.roll(d, -1, axis=1))
    fx = R(R(R(op.axy_e) * lat_e) / four_dp)
    if zonal:
        lon_e = R(east - phi)
        fx = R(R(R(R(op.axx_e) * lon_e) / dl) + fx)
    fx = R(fx + R(R(op.bx_e) * R(hlf * R(phi + east))))
    z = R(east - np.roll(phi, 1, axis=1))
    lon_n = R(z[:-1] + z[1:])
    lat_n = R(phi[1:] - phi[:-1])
    fy = R(R(R(R(op.ayy_n) * lat_n) / dp) + R(R(R(op.ayx_n) * lon_n) / four_dl))
    fy = R(fy + R(R(op.by_n) * R(hlf * R(phi[:-1] + phi[1:]))))
    zero = np.zeros((1, g.nx))
    fy = np.vstack([zero, fy, zero])
    return R(R(R(fx - np.roll(fx, 1, axis=1)) / dl) + R(R(fy[1:] - fy[:-1]) / dp))


def apply_emulated(op: EllipticOperator, phi, R, Rc):
    """L(phi): the divergence with rounding R, then C phi subtracted with
    rounding Rc."""
    div = _divergence(op, phi, R)
    return Rc(div - Rc(Rc(op.c)[:, None] * Rc(phi)))


def cyclic_thomas(lo, di, up, rhs, R):
    """Solve lo_i x_{i-1} + di_i x_i + up_i x_{i+1} = rhs_i (indices mod n)
    for every row (arrays [ny][n]) by the Thomas algorithm with the
    Sherman-Morrison correction of the corner couplings, every operation
    rounded by R."""
    ny, n = di.shape
    gam = R(-di[:, 0])
    b = di.copy()
    b[:, 0] = R(di[:, 0] - gam)
    b[:, n - 1] = R(di[:, n - 1] - R(R(lo[:, 0] * up[:, n - 1]) / gam))
    u = np.zeros((ny, n))
    u[:, 0] = gam
    u[:, n - 1] = up[:, n - 1]
    # forward sweep on the two right-hand sides (rhs and u) together
    rr = np.stack([rhs, u])
    cp = np.zeros((ny, n))
    dd = np.zeros((2, ny, n))
    cp[:, 0] = R(up[:, 0] / b[:, 0])
    dd[:, :, 0] = R(rr[:, :, 0] / b[:, 0])
    for i in range(1, n):
        m = R(b[:, i] - R(lo[:, i] * cp[:, i - 1]))
        cp[:, i] = R(up[:, i] / m)
        dd[:, :, i] = R(R(rr[:, :, i] - R(lo[:, i] * dd[:, :, i - 1])) / m)
    xs = np.zeros((2, ny, n))
    xs[:, :, n - 1] = dd[:, :, n - 1]
    for i in range(n - 2, -1, -1):
        xs[:, :, i] = R(dd[:, :, i] - R(cp[:, i] * xs[:, :, i + 1]))
    y, z = xs[0], xs[1]
    # v = (1, 0, ..., 0, lo_0 / gam): x = y - (v.y) / (1 + v.z) z
    vn = R(lo[:, 0] / gam)
    vy = R(y[:, 0] + R(vn * y[:, n - 1]))
    vz = R(z[:, 0] + R(vn * z[:, n - 1]))
    fac = R(vy / R(1.0 + vz))
    return R(y - R(fac[:, None] * z))


def precond_emulated(op: EllipticOperator, r, R, iterations=2):
    """Option 3 (eq. P_Operator) with every operation rounded by R:
    q_{mu+1} = T^{-1}(q_mu + eta (P^M q_mu - r)), q_0 = 0, T = I - eta (P^Z - P^H)."""
    g = op.grid
    ny, nx = g.ny, g.nx
    dl, dp = R(g.dlam), R(g.dphi)
    zero = np.zeros((1, nx))
    ayy = R(op.ayy_n)
    north = np.vstack([ayy, zero])
    south = np.vstack([zero, ayy])
    eta = R(R(dp * dp) / R(north + south))
    ae = R(R(op.axx_e) / R(dl * dl))
    aw = np.roll(ae, 1, axis=1)
    c = R(op.c)[:, None]
    lo = R(-R(eta * aw))
    up = R(-R(eta * ae))
    di = R(R(1.0 + R(eta * R(ae + aw))) + R(eta * c))
    r = R(r)
    q = cyclic_thomas(lo, di, up, R(-R(eta * r)), R)
    for _ in range(1, iterations):
        pm = _divergence(op, q, R, zonal=False)
        q = cyclic_thomas(lo, di, up, R(q + R(eta * R(pm - r))), R)
    return q


class HalfPrecisionParts:
    """The operator and the preconditioner of the half-precision solver:
    half precision with C Phi in single precision, single precision in the
    `polar` rows next to either pole (`rh`, `rs` replace half and single,
    e.g. by `exact` for the formula pins)."""

    def __init__(self, op: EllipticOperator, polar=3, iterations=2, rh=half, rs=single):
        self.op, self.iterations, self.rh, self.rs = op, iterations, rh, rs
        self.mask = polar_mask(op.grid.ny, polar)
        self.polar = polar

    def apply(self, phi):
        a = apply_emulated(self.op, phi, self.rh, self.rs)
        if not self.mask.any():
            return a
        return _select(a, apply_emulated(self.op, phi, self.rs, self.rs), self.mask)

    def precond(self, r):
        if not self.mask.any():
            return precond_emulated(self.op, r, self.rh, self.iterations)
        # the polar rows' systems run in single precision; their P^M reads the
        # neighbouring rows as the interior computed them, so the two
        # evaluations are merged after every Richardson iteration
        return self._merged(r)

    def _merged(self, r):
        op, rh, rs, mask = self.op, self.rh, self.rs, self.mask
        g = op.grid
        parts = {}
        for name, R in (("h", rh), ("s", rs)):
            dl, dp = R(g.dlam), R(g.dphi)
            zero = np.zeros((1, g.nx))
            ayy = R(op.ayy_n)
            eta = R(R(dp * dp) / R(np.vstack([ayy, zero]) + np.vstack([zero, ayy])))
            ae = R(R(op.axx_e) / R(dl * dl))
            aw = np.roll(ae, 1, axis=1)
            lo, up = R(-R(eta * aw)), R(-R(eta * ae))
            di = R(R(1.0 + R(eta * R(ae + aw))) + R(eta * R(op.c)[:, None]))
            parts[name] = (R, eta, lo, di, up)

        def step(q, first):
            out = {}
            for name, (R, eta, lo, di, up) in parts.items():
                rv = R(r)
                if first:
                    rhs = R(-R(eta * rv))
                else:
                    pm = _divergence(op, q, R, zonal=False)
                    rhs = R(R(q) + R(eta * R(pm - rv)))
                out[name] = cyclic_thomas(lo, di, up, rhs, R)
            return _select(out["h"], out["s"], mask)

        q = step(None, True)
        for _ in range(1, self.iterations):
            q = step(q, False)
        return q


def _dot32(a, b):
    return float(np.sum(np.asarray(a, np.float32) * np.asarray(b, np.float32), dtype=np.float32))


def gcr_half(op: EllipticOperator, rhs, x0=None, k=3, rtol=1e-8, polar=3, iterations=2, min_iters=None,
             max_iters=60, rh=half, rs=single):
    """The paper's mixed-precision GCR(k) with half precision (Section 4.3),
    emulated; returns a GCRResult whose history is the single-precision
    recursive residual and whose rel_res_true is the float64 residual of the
    final Phi_0 + Delta Phi."""
    if min_iters is None:
        min_iters = k + 1
    parts = HalfPrecisionParts(op, polar, iterations, rh, rs)
    rhs = np.asarray(rhs, dtype=np.float64)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    # step 1: r_0 in single precision, split evaluation with float64 polar bands
    if rs is exact:
        r = op.apply(x) - rhs
    else:
        hat, tilde = split_fields(x)
        r = single(residual_split(op, hat, base_differences(hat), tilde, rhs, polar=polar))
    dot = _dot32 if rs is single else (lambda a, b: float(np.sum(a * b)))
    sq = (lambda v: float(np.float32(np.sqrt(np.float32(v))))) if rs is single else np.sqrt
    rho0 = sq(dot(r, r))
    if rho0 == 0.0:
        return GCRResult(x, CONVERGED, 0, 0.0, 0.0, 0.0)
    dx = np.zeros_like(x)
    p = [None] * (k + 1)
    lp = [None] * (k + 1)
    p[0] = rh(parts.precond(r))
    lp[0] = rs(parts.apply(p[0]))
    history = [1.0]
    it, status, rn, done = 0, NOT_CONVERGED, rho0, False
    while not done:
        cycle_start = rn
        for nu in range(k):
            den = dot(lp[nu], lp[nu])
            beta = rs(-dot(r, lp[nu]) / den) if den != 0.0 else np.nan
            if not np.isfinite(beta):
                status, done = STAGNATED, True
                break
            dx = rs(dx + rs(beta * p[nu]))
            r = rs(r + rs(beta * lp[nu]))
            it += 1
            rn = sq(dot(r, r))
            history.append(rn / rho0)
            if it >= min_iters and rn <= rtol * rho0:
                status, done = CONVERGED, True
                break
            if it >= max_iters:
                status, done = NOT_CONVERGED, True
                break
            e = parts.precond(r)
            le = rs(parts.apply(e))
            pn, lpn = rh(e), le
            for l in range(nu + 1):
                alpha = rs(-dot(le, lp[l]) / dot(lp[l], lp[l]))
                pn = rh(pn + rh(alpha * p[l]))
                lpn = rs(lpn + rs(alpha * lp[l]))
            p[nu + 1], lp[nu + 1] = pn, lpn
        if done:
            break
        if rn >= cycle_start:
            status = STAGNATED
            break
        p[0], lp[0] = p[k], lp[k]
    xf = x + dx
    res = op.apply(xf) - rhs
    r0_64 = np.sqrt(float(np.sum((op.apply(x) - rhs) ** 2)))
    return GCRResult(xf, status, it, rho0, rn / rho0, float(np.sqrt(np.sum(res * res)) / r0_64), history)
