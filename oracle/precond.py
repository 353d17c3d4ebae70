"""Preconditioners of the GCR solve (oracle), paper Section 2.3.

The preconditioner estimates the solution error q = P^{-1}(r) ~ L^{-1}(r) by a
stationary iteration started from q_0 = 0.  Options:

* 0: P = I, q = r.
* 1: P = diagonal of L, q = r / diag(L).
* 2: explicit Richardson iteration on the full L, preconditioned by its
  diagonal: q_{mu+1} = q_mu - diag(L)^{-1} (L q_mu - r).
* 3: the semi-implicit Richardson scheme of eq. P_Operator,
      [I - eta (P^Z - P^H)] q_{mu+1} = q_mu + eta (P^M q_mu - r),
  with P^Z the second-order zonal derivative part of L, P^H the Helmholtz
  term (C q) and P^M = L - (P^Z - P^H) the remainder (meridional, cross and
  B terms), lagged by one iteration.  The left-hand operator couples only
  points of one latitude row: a cyclic tridiagonal system per row.

Readings (the paper gives no discrete form):
* P^Z q = [A^xx_e (q_{i+1}-q_i) - A^xx_w (q_i-q_{i-1})] / dlam^2, exactly the
  zonal diagonal-coefficient part of the discrete L.
* eta is a pointwise pseudo-time step equal to the explicit stability bound
  of the meridional diffusion in P^M:  eta = dlat^2 / (A^yy_n + A^yy_s).
* Two Richardson iterations (two tridiagonal inversions, one P^M evaluation)
  unless told otherwise, as used for every experiment of the paper.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import EllipticOperator

PC_NONE, PC_DIAG, PC_RICHARDSON, PC_SEMI_IMPLICIT = 0, 1, 2, 3


def zonal_part(op: EllipticOperator, q):
    """P^Z q."""
    g = op.grid
    axx_w = np.roll(op.axx_e, 1, axis=1)
    return (op.axx_e * (np.roll(q, -1, axis=1) - q) - axx_w * (q - np.roll(q, 1, axis=1))) / g.dlam ** 2


def helmholtz_part(op: EllipticOperator, q):
    """P^H q = C q."""
    return op.c[:, None] * q


def meridional_part(op: EllipticOperator, q):
    """P^M q = L q - (P^Z q - P^H q)."""
    return op.apply(q) - zonal_part(op, q) + helmholtz_part(op, q)


def pseudo_timestep(op: EllipticOperator):
    """eta[ny][nx] = dlat^2 / (A^yy_n + A^yy_s)."""
    north, south = op.ayy_north_south()
    return op.grid.dphi ** 2 / (north + south)


def row_systems(op: EllipticOperator, eta=None):
    """Entries of T = I - eta (P^Z - P^H): per row j the cyclic tridiagonal
    system  lower_i q_{i-1} + diag_i q_i + upper_i q_{i+1}.  Returns
    (lower, diag, upper), each [ny][nx]."""
    g = op.grid
    if eta is None:
        eta = pseudo_timestep(op)
    ae = op.axx_e / g.dlam ** 2
    aw = np.roll(op.axx_e, 1, axis=1) / g.dlam ** 2
    lower = -eta * aw
    upper = -eta * ae
    diag = 1.0 + eta * (ae + aw) + eta * op.c[:, None]
    return lower, diag, upper


def row_matrix(lower, diag, upper):
    """Dense cyclic tridiagonal matrix of one row (for tests)."""
    n = diag.shape[0]
    m = np.zeros((n, n))
    for i in range(n):
        m[i, i] = diag[i]
        m[i, (i - 1) % n] += lower[i]
        m[i, (i + 1) % n] += upper[i]
    return m


class SemiImplicitRichardson:
    """Option 3, eq. P_Operator.  The block-diagonal T (one cyclic tridiagonal
    block per row) is factorised once with a sparse LU."""

    def __init__(self, op: EllipticOperator, iterations=2):
        self.op = op
        self.iterations = iterations
        self.eta = pseudo_timestep(op)
        lower, diag, upper = row_systems(op, self.eta)
        ny, nx = op.grid.ny, op.grid.nx
        idx = np.arange(ny * nx).reshape(ny, nx)
        west = np.roll(idx, 1, axis=1)
        east = np.roll(idx, -1, axis=1)
        rows = np.concatenate([idx.ravel(), idx.ravel(), idx.ravel()])
        cols = np.concatenate([idx.ravel(), west.ravel(), east.ravel()])
        vals = np.concatenate([diag.ravel(), lower.ravel(), upper.ravel()])
        self.T = sp.csc_matrix((vals, (rows, cols)), shape=(ny * nx, ny * nx))
        self._lu = spla.splu(self.T)

    def solve_rows(self, rhs):
        """T^{-1} rhs."""
        shape = rhs.shape
        return self._lu.solve(np.ascontiguousarray(rhs, dtype=np.float64).ravel()).reshape(shape)

    def __call__(self, r):
        q = np.zeros_like(r)
        for _ in range(self.iterations):
            q = self.solve_rows(q + self.eta * (meridional_part(self.op, q) - r))
        return q


class Preconditioner:
    """q = P^{-1}(r) for options 0-3."""

    def __init__(self, op: EllipticOperator, option=PC_SEMI_IMPLICIT, iterations=2):
        self.op, self.option, self.iterations = op, option, iterations
        if option == PC_SEMI_IMPLICIT:
            self._si = SemiImplicitRichardson(op, iterations)
        elif option in (PC_DIAG, PC_RICHARDSON):
            self._diag = op.diagonal()
        elif option != PC_NONE:
            raise ValueError(f"unknown preconditioner option {option}")

    def __call__(self, r):
        if self.option == PC_NONE:
            return r.copy()
        if self.option == PC_DIAG:
            return r / self._diag
        if self.option == PC_RICHARDSON:
            q = np.zeros_like(r)
            for _ in range(self.iterations):
                q = q - (self.op.apply(q) - r) / self._diag
            return q
        return self._si(r)
