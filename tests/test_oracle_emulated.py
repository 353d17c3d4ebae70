"""Pins of the emulated reduced-precision oracle (paper Sections 3.3, 4.3),
CPU only.

* The rounding: values worked by hand (ties to even, carries into the next
  binade), the range kept from float64 (no overflow at 65504, no
  subnormals), and agreement with IEEE half (numpy float16) wherever IEEE
  half has the same 10-bit significand, i.e. its normal range.
* The formulas: with rounding switched off the emulated operator, P^M,
  row solves, preconditioner and solver equal the float64 oracle's.
* The half-precision solver: with the paper's rounding points it stalls at a
  true relative residual of order 1e-5 (the paper reports about 1e-5 for
  RHW4 and 5e-5 for the orographic case, then a plateau) while its own
  recursive residual keeps falling; rounding the operator alone to half also
  in the polar rows costs accuracy there.
"""
import numpy as np
import pytest

from oracle import emulated as em
from oracle.gcr import gcr, CONVERGED
from oracle.operator import EllipticOperator
from oracle.precond import Preconditioner, meridional_part, row_matrix, row_systems
from workloads import problem


def test_rounding_by_hand():
    r = em.rpe_round
    one = 1.0
    u = 2.0 ** -10                                  # spacing of the significand in [1, 2)
    assert r(one + u / 2) == one                    # tie: to the even significand (1.0000000000)
    assert r(one + 3 * u / 2) == one + 2 * u        # tie: 1.0000000001 is odd, goes up to ...10
    assert r(one + u / 2 + 2.0 ** -30) == one + u   # just above the tie
    assert r(one + u / 2 - 2.0 ** -30) == one       # just below it
    assert r(2.0 - u / 2) == 2.0                    # tie at the top of the binade carries into 2
    assert r(-(one + 3 * u / 2)) == -(one + 2 * u)  # symmetric
    assert r(1000.0) == 1000.0                      # 1111101000b: 10 bits, exact
    assert r(1025.0) == 1025.0                      # 10000000001b: 11 significant bits, exact
    assert r(2049.0) == 2048.0                      # 12 bits needed, spacing 2: tie to even (...000)
    assert r(2051.0) == 2052.0                      # tie between 2050 (odd) and 2052 (even)
    assert r(np.pi) == 3.140625                     # 11.00100100 00111...: rounds down


def test_rounding_keeps_the_float64_range():
    r = em.rpe_round
    assert r(70000.0) == 70016.0                    # beyond IEEE half's 65504: still finite
    assert 70000.0 > float(np.finfo(np.float16).max)
    tiny = 2.0 ** -30 * (1 + 2.0 ** -12)
    assert r(tiny) == 2.0 ** -30                    # no subnormal flush below 2^-14
    assert r(3.0 * 2.0 ** 900 + 2.0 ** 890) == 3.0 * 2.0 ** 900
    assert r(0.0) == 0.0 and np.isinf(r(np.inf)) and np.isnan(r(np.nan))
    assert r(1e-300) > 0


def test_rounding_equals_ieee_half_in_its_normal_range():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, 200000) * 2.0 ** rng.integers(-14, 15, 200000)
    x = x[(np.abs(x) >= 2.0 ** -14) & (np.abs(x) <= 65504)]
    assert np.array_equal(em.rpe_round(x), x.astype(np.float16).astype(np.float64))
    assert np.array_equal(em.rpe_round(x, 23), x.astype(np.float32).astype(np.float64))


def _case(nx=64, ny=32, seed=0):
    pr = problem(2, nx, ny, instance=seed, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    return pr, op


@pytest.mark.parametrize("nx,ny", [(16, 8), (64, 32), (128, 64)])
def test_unrounded_parts_are_the_oracle(nx, ny):
    pr, op = _case(nx, ny)
    x = np.random.default_rng(1).standard_normal((ny, nx))
    scale = np.max(np.abs(op.apply(x)))
    assert np.max(np.abs(em.apply_emulated(op, x, em.exact, em.exact) - op.apply(x))) <= 1e-13 * scale
    pm = meridional_part(op, x)
    assert np.max(np.abs(em._divergence(op, x, em.exact, zonal=False) - pm)) <= 1e-13 * np.max(np.abs(pm))
    for it in (1, 2, 3):
        ref = Preconditioner(op, 3, it)(x)
        got = em.precond_emulated(op, x, em.exact, it)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the polar-row merge with no rounding is the same preconditioner
    parts = em.HalfPrecisionParts(op, polar=2, rh=em.exact, rs=em.exact)
    assert np.max(np.abs(parts.precond(x) - Preconditioner(op, 3, 2)(x))) <= 1e-12 * np.max(np.abs(ref))


def test_cyclic_thomas_is_a_dense_solve():
    rng = np.random.default_rng(2)
    ny, n = 5, 9
    lo, up = -rng.random((ny, n)), -rng.random((ny, n))
    di = 2.5 + rng.random((ny, n))
    b = rng.standard_normal((ny, n))
    x = em.cyclic_thomas(lo, di, up, b, em.exact)
    for j in range(ny):
        assert np.allclose(row_matrix(lo[j], di[j], up[j]) @ x[j], b[j], rtol=0, atol=1e-13)


def test_unrounded_solver_is_the_oracle():
    pr, op = _case(64, 32)
    rhs = op.apply(pr["x_true"])
    ref = gcr(op, rhs, rtol=1e-10)
    got = em.gcr_half(op, rhs, rtol=1e-10, rh=em.exact, rs=em.exact)
    assert got.status == CONVERGED and got.iterations == ref.iterations
    assert np.linalg.norm(got.x - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


def test_half_operator_error_is_half_sized():
    pr, op = _case(128, 64)
    x = pr["x_true"]
    exact = op.apply(x)
    h = em.apply_emulated(op, x, em.half, em.single)
    rel = np.abs(h - exact) / np.max(np.abs(exact))
    assert 1e-6 < np.max(rel) < 1e-2           # rounded to about half precision: well above float32
    parts = em.HalfPrecisionParts(op, polar=2)
    hp = parts.apply(x)
    # the polar bands run in single precision: float32-sized errors there
    relp = np.abs(hp - exact) / np.max(np.abs(exact))
    assert np.max(relp[:2]) < 1e-5 and np.max(relp[-2:]) < 1e-5
    assert np.max(relp[:2]) < 0.1 * np.max(rel[:2])


@pytest.mark.parametrize("nx,ny,polar", [(64, 32, 1), (128, 64, 2)])
def test_half_precision_solver_plateau(nx, ny, polar):
    pr, op = _case(nx, ny)
    rhs = op.apply(pr["x_true"])
    ref = gcr(op, rhs, rtol=1e-10)
    res = em.gcr_half(op, rhs, rtol=1e-8, polar=polar)
    # the recursive (single-precision) residual reaches the tolerance ...
    assert res.status == CONVERGED and res.rel_res_recursive <= 1e-8
    # ... but the solution stalls at a half-precision plateau, as the paper
    # reports (about 1e-5 relative for its test cases)
    assert 1e-7 < res.rel_res_true < 1e-3
    err = np.linalg.norm(res.x - ref.x) / np.linalg.norm(ref.x)
    assert 1e-8 < err < 1e-3
    # one full cycle at least, and no more iterations than the plateau needs
    assert 4 <= res.iterations <= 10
