"""Split single-precision residual (oracle), paper Section 4.2.1, eq. L_Operator_SP.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

The depth is carried as two float32 fields, Phi ~ Phi_hat + Phi_tilde:
  Phi_hat   = fl32(Phi0)                 (the base, renewed only now and then)
  Phi_tilde = fl32(Phi0 - Phi_hat)       (the difference taken in float64)
In the operator the gradient terms take the differences of Phi_hat, computed
once and stored in float32, plus those of Phi_tilde; the B and C terms take
Phi_SP = Phi_hat + Phi_tilde, all in float32.  The rows within `polar` rows
of either pole use the float64 operator on Phi_hat + Phi_tilde instead (the
paper keeps three such bands in double precision).  The residual is
r = L_SP - R with R in float64; the float32 rows are returned rounded to
float32.

Readings:
* "differences of Phi_hat" are the undivided differences the discrete
  operator uses at each face (zonal and 4-point meridional at east faces,
  meridional and 4-point zonal at north faces), computed in float64 from the
  float32 values and rounded once to float32;
* the coefficients of the float32 rows are the float64 ones rounded to
  float32, and every operation of those rows is a float32 operation.
`dtype=np.float64` evaluates the same formula without rounding (it then
equals the float64 operator on Phi_hat + Phi_tilde): the pin of the formula.
"""
from __future__ import annotations

import numpy as np

from .operator import EllipticOperator, across_pole_extend


def split_fields(phi0):
    """(Phi_hat, Phi_tilde) as float32 arrays."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    hat = phi0.astype(np.float32)
    tilde = (phi0 - hat.astype(np.float64)).astype(np.float32)
    return hat, tilde


def face_differences(phi, dtype):
    """The undivided differences of the discrete operator's gradient terms:
    lon_e  phi[i+1,j] - phi[i,j]                                  (east faces)
    lat_e  phi[i,j+1] - phi[i,j-1] + phi[i+1,j+1] - phi[i+1,j-1]   (east faces)
    lat_n  phi[i,j+1] - phi[i,j]                          (interior north faces)
    lon_n  phi[i+1,j] - phi[i-1,j] + phi[i+1,j+1] - phi[i-1,j+1]   (north faces)
    with rows beyond the poles seen across the pole."""
    phi = np.asarray(phi, dtype=dtype)
    e = across_pole_extend(phi)
    d = e[2:] - e[:-2]
    z = np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)
    return {"lon_e": np.roll(phi, -1, axis=1) - phi,
            "lat_e": d + np.roll(d, -1, axis=1),
            "lat_n": phi[1:] - phi[:-1],
            "lon_n": z[:-1] + z[1:]}


def base_differences(phi_hat):
    """Stored float32 differences of Phi_hat (taken in float64, rounded once)."""
    return {k: v.astype(np.float32) for k, v in face_differences(np.asarray(phi_hat, np.float64),
                                                                 np.float64).items()}


def residual_split(op: EllipticOperator, phi_hat, dhat, phi_tilde, rhs, polar=3, dtype=np.float32):
    """r = L_SP(Phi_hat + Phi_tilde) - R (float64 array holding the float32
    results of the float32 rows)."""
    g = op.grid
    t = dtype
    ph = np.asarray(phi_hat).astype(t)
    pt = np.asarray(phi_tilde).astype(t)
    dt_ = face_differences(pt, t)
    dlon_e = dhat["lon_e"].astype(t) + dt_["lon_e"]
    dlat_e = dhat["lat_e"].astype(t) + dt_["lat_e"]
    dlat_n = dhat["lat_n"].astype(t) + dt_["lat_n"]
    dlon_n = dhat["lon_n"].astype(t) + dt_["lon_n"]
    psp = ph + pt
    dl, dp = t(g.dlam), t(g.dphi)
    fx = (op.axx_e.astype(t) * dlon_e / dl
          + op.axy_e.astype(t) * dlat_e / (t(4.0) * dp)
          + op.bx_e.astype(t) * t(0.5) * (psp + np.roll(psp, -1, axis=1)))
    fy_int = (op.ayy_n.astype(t) * dlat_n / dp
              + op.ayx_n.astype(t) * dlon_n / (t(4.0) * dl)
              + op.by_n.astype(t) * t(0.5) * (psp[:-1] + psp[1:]))
    zero = np.zeros((1, g.nx), dtype=t)
    fy = np.vstack([zero, fy_int, zero])
    lsp = (fx - np.roll(fx, 1, axis=1)) / dl + (fy[1:] - fy[:-1]) / dp - op.c.astype(t)[:, None] * psp
    r = (lsp.astype(np.float64) - np.asarray(rhs, np.float64)).astype(t).astype(np.float64)
    if polar > 0:
        full = op.apply(np.asarray(phi_hat, np.float64) + np.asarray(phi_tilde, np.float64)) - rhs
        rows = np.r_[0:min(polar, g.ny), max(g.ny - polar, 0):g.ny]
        r[rows] = full[rows]
    return r


def residual_naive_sp(op: EllipticOperator, phi, rhs):
    """The plain float32 evaluation of the operator on fl32(Phi), for
    comparison: r = fl32(L_32(fl32(Phi)) - R)."""
    hat = np.asarray(phi, np.float64).astype(np.float32)
    zero = np.zeros_like(hat)
    return residual_split(op, hat, {k: v.astype(np.float32) for k, v in face_differences(hat, np.float32).items()},
                          zero, rhs, polar=0)
