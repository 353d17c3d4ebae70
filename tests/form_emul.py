"""Rounding model of the solver's precision forms (test helper).

The parity tests of gcr_apply_operator_form / gcr_apply_precond_form compare
the GPU with this model element by element.  The model takes the float64
oracle's operator and preconditioner steps and rounds exactly the quantities
that a form stores in a narrower type, as the solver stores them (paper
Sections 4.2-4.3 list which quantity is held in which precision; the
solver's forms are described in include/mpgcr.h):

* mixed forms hold residuals in scaled units s r, s = dt / (2 a^2), and
  directions in physical units; vectors are float32;
* operator coefficients of GCR_MIXED / GCR_MIXED_FP64DOT and preconditioner
  coefficients of every mixed form with float16 intermediates are the face
  coefficients, divided by the grid factors of their differences and scaled
  by s, stored as float16 (float32 in the polar rows); the Helmholtz
  coefficient is float32;
* the float32 operator (GCR_MIXED_HALF_PC, GCR_SINGLE) and the float32
  preconditioner (GCR_SINGLE) form their coefficients from the float32 depth;
* the preconditioner intermediate between Richardson iterations is float16
  with one scale per row (its row maximum), or float32.

Everything else is float64 here, so the GPU differs from the model by float32
arithmetic only -- plus, where a float16 intermediate is stored, the rare
points where float32 arithmetic lands on the other side of a float16 rounding
boundary.  Nothing here comes from the HIP path.
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.operator import EllipticOperator
from oracle.precond import meridional_part, pseudo_timestep, row_systems

FP64, MIXED, MIXED_FP64DOT, MIXED_HALF_PC, SINGLE, SINGLE_POLAR64 = range(6)
U16 = 2.0 ** -11      # unit roundoff of float16
U32 = 2.0 ** -24      # unit roundoff of float32


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def f16(x):
    """float64 -> float16 as the assembly stores it: through float32."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def scale_of(op: EllipticOperator) -> float:
    return op.dt / (2.0 * op.radius ** 2)


def polar_rows(ny: int, polar: int = -1) -> np.ndarray:
    """Boolean [ny]: rows within `polar` rows of a pole (-1: max(1, log2(NY/32)))."""
    if polar < 0:   # max(1, ceil(log2(max(NY // 32, 1)))), the solver's default
        v, lg = max(ny // 32, 1), 0
        while (1 << lg) < v:
            lg += 1
        polar = max(1, lg)
    polar = min(polar, ny)
    j = np.arange(ny)
    return (j < polar) | (j >= ny - polar)


def stored_operator(op: EllipticOperator, rnd) -> EllipticOperator:
    """Copy of op whose coefficients are the values a form stores: each face
    coefficient divided by its grid factor, times s, rounded by `rnd`, and
    mapped back to physical units in float64; C as float32 s*C."""
    g = op.grid
    s = scale_of(op)
    out = copy.copy(op)

    def st(a, f):
        return rnd(s * a / f) * f / s

    out.axx_e = st(op.axx_e, g.dlam ** 2)
    out.axy_e = st(op.axy_e, 4.0 * g.dlam * g.dphi)
    out.bx_e = st(op.bx_e, 2.0 * g.dlam)
    out.ayy_n = st(op.ayy_n, g.dphi ** 2)
    out.ayx_n = st(op.ayx_n, 4.0 * g.dlam * g.dphi)
    out.by_n = st(op.by_n, 2.0 * g.dphi)
    out.c = f32(s * op.c) / s
    return out


def float32_depth_operator(nx, ny, depth, dt, orography=None, **kw) -> EllipticOperator:
    """The operator formed from the float32 depth pools (Phi* and H* = Phi* +
    H0 each rounded to float32), with float32 C."""
    d32 = f32(depth)
    oro = None
    if orography is not None:
        oro = f32(np.asarray(depth) + np.asarray(orography)) - d32   # H* = d32 + oro is float32 exactly
    op = EllipticOperator(nx, ny, d32, dt, orography=oro, **kw)
    op.c = f32(scale_of(op) * op.c) / scale_of(op)
    return op


def _rows(a, b, sel):
    """Rows of b where sel, else rows of a."""
    out = np.array(a, copy=True)
    out[sel] = b[sel]
    return out


class RowOps:
    """Per-row choice between two operators (interior rows from `inner`,
    rows where `sel` from `outer`); each row's stencil, pseudo time step and
    row system come from its own operator, as each GPU row reads one storage."""

    def __init__(self, inner, outer=None, sel=None):
        self.inner, self.outer = inner, outer
        self.sel = np.zeros(inner.grid.ny, bool) if sel is None else sel

    def apply(self, x):
        y = self.inner.apply(x)
        return y if self.outer is None else _rows(y, self.outer.apply(x), self.sel)

    def meridional(self, q):
        y = meridional_part(self.inner, q)
        return y if self.outer is None else _rows(y, meridional_part(self.outer, q), self.sel)

    def eta(self):
        e = pseudo_timestep(self.inner)
        return e if self.outer is None else _rows(e, pseudo_timestep(self.outer), self.sel)

    def systems(self):
        lo, di, up = row_systems(self.inner, pseudo_timestep(self.inner))
        if self.outer is not None:
            lo2, di2, up2 = row_systems(self.outer, pseudo_timestep(self.outer))
            lo, di, up = _rows(lo, lo2, self.sel), _rows(di, di2, self.sel), _rows(up, up2, self.sel)
        return lo, di, up


def _row_solver(lo, di, up):
    ny, nx = di.shape
    idx = np.arange(ny * nx).reshape(ny, nx)
    rows = np.concatenate([idx.ravel()] * 3)
    cols = np.concatenate([idx.ravel(), np.roll(idx, 1, 1).ravel(), np.roll(idx, -1, 1).ravel()])
    vals = np.concatenate([di.ravel(), lo.ravel(), up.ravel()])
    lu = spla.splu(sp.csc_matrix((vals, (rows, cols)), shape=(ny * nx, ny * nx)))
    return lambda rhs: lu.solve(np.ascontiguousarray(rhs).ravel()).reshape(ny, nx)


def operator_model(form, op, depth, orography=None, absorber=0.0, b_terms=True, polar=-1):
    """RowOps of the operator the solve of `form` applies to a direction."""
    g = op.grid
    sel = polar_rows(g.ny, polar)
    if form == FP64:
        return RowOps(op)
    if form in (MIXED, MIXED_FP64DOT):
        return RowOps(stored_operator(op, f16), stored_operator(op, f32), sel)
    op32 = float32_depth_operator(g.nx, g.ny, depth, op.dt, orography, absorber=absorber, b_terms=b_terms)
    if form in (MIXED_HALF_PC, SINGLE):
        return RowOps(op32)
    return RowOps(op32, op, sel)            # SINGLE_POLAR64: float64 polar rows


def precond_model(form, op, depth, orography=None, absorber=0.0, b_terms=True, polar=-1):
    """(RowOps of the preconditioner's coefficients, intermediate storage
    'half' or 'single' or 'double')."""
    g = op.grid
    sel = polar_rows(g.ny, polar)
    if form == FP64:
        return RowOps(op), "double"
    if form in (MIXED, MIXED_FP64DOT, MIXED_HALF_PC):
        return RowOps(stored_operator(op, f16), stored_operator(op, f32), sel), "half"
    op32 = float32_depth_operator(g.nx, g.ny, depth, op.dt, orography, absorber=absorber, b_terms=b_terms)
    if form == SINGLE:
        return RowOps(op32), "single"
    return RowOps(op32, op, sel), "single"


def store_intermediate(q, kind):
    """The preconditioner intermediate as the next Richardson iteration reads it."""
    if kind == "double":
        return q
    if kind == "single":
        return f32(q)
    sc = f32(np.max(np.abs(f32(q)), axis=1))
    sc = np.where(sc > 0, sc, 1.0)
    inv = f32(1.0 / sc)
    t = f32(f32(q) * inv[:, None])
    return f32(f16(t) * sc[:, None])


def emulate_operator(form, model: RowOps, x):
    """y = L(x) of the form in physical units (x rounded to the vector type)."""
    xv = x if form == FP64 else f32(x)
    return model.apply(xv)


def emulate_precond(form, model: RowOps, kind, r, s, iterations=2):
    """e = P^{-1}(r) of option 3 with `iterations` Richardson iterations, as
    the form computes it (r entering as the held residual, e as held)."""
    rv = r if form == FP64 else f32(s * r)
    units = 1.0 if form == FP64 else s       # coefficients are physical; residual held in units s
    eta = model.eta()
    solve = _row_solver(*model.systems())
    q = solve(-eta * rv / units)
    for _ in range(1, iterations):
        q = store_intermediate(q, kind)
        q = solve(q + eta * (model.meridional(q) - rv / units))
    return q


def row_condition(model: RowOps):
    """Per-row max-norm condition bound of the row systems: max_i di/(di - |lo| - |up|)."""
    lo, di, up = model.systems()
    return np.max(di / (di - np.abs(lo) - np.abs(up)), axis=1)


def b_term_magnitude(op: EllipticOperator, depth, orography=None):
    """Per point: an upper bound of sum |B face coefficient| / grid factor
    over the four faces, with every difference of H* in B^x, B^y replaced by
    the sum of the magnitudes of its terms (gamma / D <= 1 and b / D <= |b|
    taken as bounds).  Forming B from the float32 depth errs by a few float32
    ulps of this; the caller multiplies by the local max |x|."""
    g = op.grid
    hs = np.abs(np.asarray(depth) + (0.0 if orography is None else np.asarray(orography)))
    delta = 0.5 * op.dt
    lat, lat_n = g.lat, g.lat_n
    b = np.abs(delta * 2.0 * op.omega * np.sin(lat))
    bn = np.abs(delta * 2.0 * op.omega * np.sin(lat_n))
    gx = delta * op.g / 2.0            # gamma, D >= 1 make these upper bounds
    e = np.vstack([np.roll(hs[0], g.nx // 2)[None], hs, np.roll(hs[-1], g.nx // 2)[None]])
    m4 = (e[2:] + e[:-2]) + np.roll(e[2:] + e[:-2], -1, 1)
    bx = gx * (1.0 / np.cos(lat)[:, None] * (hs + np.roll(hs, -1, 1)) / g.dlam
               + b[:, None] * m4 / (4 * g.dphi))
    l4 = (np.roll(hs, -1, 1) + np.roll(hs, 1, 1))
    by = gx * (bn[:, None] * (l4[:-1] + l4[1:]) / (4 * g.dlam)
               + np.cos(lat_n)[:, None] * (hs[1:] + hs[:-1]) / g.dphi)
    zero = np.zeros((1, g.nx))
    tot = (bx + np.roll(bx, 1, 1)) / g.dlam + (np.vstack([by, zero]) + np.vstack([zero, by])) / g.dphi
    return tot


def stencil_magnitude(op, x):
    """Pointwise sum of |summands| of L(x), inflated by the conditioning of the
    latitude-dependent factors: a latitude computed with or without a fused
    multiply-add differs by ~1 ulp of pi/2, which changes cos(lat) by a
    relative ~ulp/cos(lat) -- large next to the poles, where A^xx ~ 1/cos.
    A small multiple of eps times this bounds the float64 rounding of any
    evaluation order."""
    g = op.grid
    ax = np.abs(x)
    m = ax
    mx = np.maximum.reduce([ax, np.roll(ax, 1, 1), np.roll(ax, -1, 1)])
    ext = np.vstack([np.roll(mx[0], g.nx // 2)[None], mx, np.roll(mx[-1], g.nx // 2)[None]])
    m3 = np.maximum.reduce([ext[:-2], ext[1:-1], ext[2:]])
    aw = np.roll(op.axx_e, 1, 1)
    north, south = op.ayy_north_south()
    zero = np.zeros((1, g.nx))
    cross = (np.abs(op.axy_e) + np.abs(np.roll(op.axy_e, 1, 1))) / (4 * g.dlam * g.dphi) * 4
    cross += (np.abs(np.vstack([op.ayx_n, zero])) + np.abs(np.vstack([zero, op.ayx_n]))) / (4 * g.dlam * g.dphi) * 4
    bterm = (np.abs(op.bx_e) + np.abs(np.roll(op.bx_e, 1, 1))) / g.dlam
    bterm += (np.abs(np.vstack([op.by_n, zero])) + np.abs(np.vstack([zero, op.by_n]))) / g.dphi
    cond = 1.0 + 1.0 / np.cos(g.lat)[:, None]
    return ((2 * (np.abs(op.axx_e) + np.abs(aw)) / g.dlam ** 2 + 2 * (north + south) / g.dphi ** 2
             + cross + bterm) * m3 + op.c[:, None] * m) * cond


def neighbourhood_max(x):
    """max |x| over each point's 3x3 stencil neighbourhood (across the poles too)."""
    nx = x.shape[1]
    ax = np.abs(x)
    mx = np.maximum.reduce([ax, np.roll(ax, 1, 1), np.roll(ax, -1, 1)])
    ext = np.vstack([np.roll(mx[0], nx // 2)[None], mx, np.roll(mx[-1], nx // 2)[None]])
    return np.maximum.reduce([ext[:-2], ext[1:-1], ext[2:]])


def rows_max3(a):
    """Per row, the max of |a| over the row and its two meridional neighbours
    (the rows across the poles are the polar rows themselves), shape [ny][1]."""
    m = np.max(np.abs(a), axis=1)
    ext = np.concatenate([m[:1], m, m[-1:]])
    return np.maximum.reduce([ext[:-2], ext[1:-1], ext[2:]])[:, None]


def meridional_magnitude(op):
    """Per point: the sum of |P^M coefficients| (meridional, cross and B
    terms of the stencil, without the zonal A^xx part and C), inflated by
    (1 + 1/cos(lat)) as in stencil_magnitude."""
    g = op.grid
    north, south = op.ayy_north_south()
    zero = np.zeros((1, g.nx))
    cross = (np.abs(op.axy_e) + np.abs(np.roll(op.axy_e, 1, 1))) / (4 * g.dlam * g.dphi) * 4
    cross += (np.abs(np.vstack([op.ayx_n, zero])) + np.abs(np.vstack([zero, op.ayx_n]))) / (4 * g.dlam * g.dphi) * 4
    bterm = (np.abs(op.bx_e) + np.abs(np.roll(op.bx_e, 1, 1))) / g.dlam
    bterm += (np.abs(np.vstack([op.by_n, zero])) + np.abs(np.vstack([zero, op.by_n]))) / g.dphi
    return (2 * (north + south) / g.dphi ** 2 + cross + bterm) * (1.0 + 1.0 / np.cos(g.lat)[:, None])


def richardson_bound(op, iters, local, u):
    """Pointwise rounding bound of the semi-implicit Richardson preconditioner
    (option 3) with unit roundoff u, 64 u per rounding step, relative to the
    local magnitude `local` of the iterates ([ny][1], rows j-1..j+1).  The row
    solve of each iteration rounds with at most the row systems' condition
    bound di / (di - |lo| - |up|) as amplification, the P^M evaluation with
    eta * sum|P^M summands| (inflated by the latitude conditioning as in
    stencil_magnitude); an error left by one iteration passes the next one
    through T^{-1} (norm <= 1: diagonally dominant with margin 1 + eta C)
    times (1 + eta |P^M|)."""
    lo, di, up = row_systems(op)
    cond = np.max(di / (di - np.abs(lo) - np.abs(up)), axis=1)[:, None]
    pm = pseudo_timestep(op) * meridional_magnitude(op)
    pm_infl = np.max(pm, axis=1)[:, None]
    rho = np.max(pm / (1.0 + 1.0 / np.cos(op.grid.lat))[:, None], axis=1)[:, None]
    c = 64 * u
    delta = c * (cond + 1.0) * local
    for _ in range(1, iters):
        delta = rows_max3(delta) * (1.0 + rho) + c * (cond + pm_infl) * local
    return delta
