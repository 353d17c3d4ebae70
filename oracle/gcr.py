"""Preconditioned GCR(k) (oracle), paper Section 2.3.

GCR minimises the Euclidean norm of the residual r = L(Phi) - R (eq.
Residual) over the preconditioned Krylov directions, re-optimising at every
iteration the coefficients of the current and up to k-1 past directions, and
converges monotonically for a non-self-adjoint L.  Steps as the paper names
them:

  step 1  r_0 = L(Phi_0) - R;  p_0 = P^{-1}(r_0);  L(p_0)
  step 2  beta = -<r L(p_nu)> / <L(p_nu) L(p_nu)>;  Phi += beta p_nu;
          r += beta L(p_nu);  exit test (eq. exitcondition)
  step 3  e = P^{-1}(r);  L(e)
  step 4  alpha_l = -<L(e) L(p_l)> / <L(p_l) L(p_l)>, l = 0..nu;
          p_{nu+1} = e + sum alpha_l p_l;  L(p_{nu+1}) = L(e) + sum alpha_l L(p_l)

After k iterations the window restarts from the last direction
(p_0, L(p_0)) := (p_k, L(p_k)).

Readings:
* <.,.> is the plain sum over all grid points (the Euclidean norm the exit
  condition names), not an area-weighted integral.
* Exit when ||r_{nu+1}||_2 <= eps ||r_0||_2, but never inside the first full
  GCR(3) cycle: the earliest exit is after iteration k+1, which makes 4 the
  minimum iteration count the paper reports.
* norm="linf": the same exit test with the maximum norm, the alternative exit
  condition the paper reports trying (Section 4.1 discussion); the iteration
  itself, the stagnation test and the reported residuals stay Euclidean.
* ||r_0|| is the initial residual of this solve, also for warm starts.
* Breakdown (<L(p) L(p)> == 0 or non-finite scalars) and a cycle without any
  decrease of ||r|| stop the iteration (stagnation).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .operator import EllipticOperator
from .precond import Preconditioner, PC_SEMI_IMPLICIT

CONVERGED, NOT_CONVERGED, STAGNATED = 0, 1, 2


def dot(a, b):
    return float(np.sum(a * b))


@dataclass
class GCRResult:
    x: np.ndarray
    status: int
    iterations: int
    r0_norm: float
    rel_res_recursive: float
    rel_res_true: float
    history: list = field(default_factory=list)        # ||r_nu|| / ||r_0||, recursive
    orth_log: list = field(default_factory=list)        # per iteration: max |<r, Lp_l>| / (|r| |Lp_l|)


def gcr(op: EllipticOperator, rhs, x0=None, k=3, rtol=1e-8, precond=PC_SEMI_IMPLICIT,
        richardson_iters=2, min_iters=None, max_iters=200, pc=None, track_orthogonality=False, norm="l2",
        r0=None):
    """Solve L(x) = rhs by preconditioned GCR(k).  `r0`: the initial residual
    as the caller evaluated it (e.g. the split single-precision residual of
    Section 4.2.1, oracle.split.residual_split); default L(x0) - rhs."""
    if norm not in ("l2", "linf"):
        raise ValueError(f"norm must be 'l2' or 'linf', got {norm!r}")
    if min_iters is None:
        min_iters = k + 1
    if pc is None:
        pc = Preconditioner(op, precond, richardson_iters)
    rhs = np.asarray(rhs, dtype=np.float64)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.float64, copy=True)

    # step 1
    r = op.apply(x) - rhs if r0 is None else np.array(r0, dtype=np.float64, copy=True)
    rho0 = np.sqrt(dot(r, r))
    rho0_inf = float(np.max(np.abs(r)))
    if rho0 == 0.0:
        return GCRResult(x, CONVERGED, 0, 0.0, 0.0, 0.0)
    p = [None] * (k + 1)
    lp = [None] * (k + 1)
    p[0] = pc(r)
    lp[0] = op.apply(p[0])

    history = [1.0]
    orth_log = []
    it = 0
    status = NOT_CONVERGED
    rn = rho0
    done = False
    while not done:
        cycle_start = rn
        for nu in range(k):
            # step 2
            den = dot(lp[nu], lp[nu])
            beta = -dot(r, lp[nu]) / den if den != 0.0 else np.nan
            if not np.isfinite(beta):
                status, done = STAGNATED, True
                break
            x += beta * p[nu]
            r += beta * lp[nu]
            it += 1
            rn = np.sqrt(dot(r, r))
            history.append(rn / rho0)
            if track_orthogonality:
                orth_log.append(max(abs(dot(r, lp[l])) / (rn * np.sqrt(dot(lp[l], lp[l])))
                                    for l in range(nu + 1)))
            small = rn <= rtol * rho0 if norm == "l2" else float(np.max(np.abs(r))) <= rtol * rho0_inf
            if it >= min_iters and small:
                status, done = CONVERGED, True
                break
            if it >= max_iters:
                status, done = NOT_CONVERGED, True
                break
            # step 3
            e = pc(r)
            le = op.apply(e)
            # step 4
            pn = e.copy()
            lpn = le.copy()
            for l in range(nu + 1):
                alpha = -dot(le, lp[l]) / dot(lp[l], lp[l])
                pn += alpha * p[l]
                lpn += alpha * lp[l]
            p[nu + 1] = pn
            lp[nu + 1] = lpn
        if done:
            break
        if rn >= cycle_start:
            status = STAGNATED
            break
        p[0], lp[0] = p[k], lp[k]

    true_res = np.sqrt(dot(op.apply(x) - rhs, op.apply(x) - rhs)) / rho0
    return GCRResult(x, status, it, rho0, rn / rho0, true_res, history, orth_log)
