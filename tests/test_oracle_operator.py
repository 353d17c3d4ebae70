"""Pins of the oracle's grid, coefficients and discrete operator L.

Each check ties the oracle to something other than itself: numbers printed in
the paper (Section 3.2), the paper's governing equations differentiated
symbolically (eqs. SWE1, RSWE2-3, MPDATA, rhslin, Qexpr), a closed-form
eigenfunction, and the algebraic properties of L (symmetry with rotation and
B terms off, negative definiteness).
"""
import json
import os

import numpy as np
import pytest
import sympy as sy

from oracle.operator import EllipticOperator, Grid, RADIUS, GRAVITY, OMEGA, absorber_profile


# --------------------------------------------------------------------------
# geometry: Section 3.2 prints the zonal grid length in the pole rows and the
# external-mode Courant number at 512x256, dt = 200 s
# --------------------------------------------------------------------------
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_geometry.json")))


@pytest.mark.parametrize("nx,ny,printed", GOLDEN["pole_row_zonal_spacing_m"]["grids"])
def test_pole_row_spacing_matches_paper(nx, ny, printed):
    dx = Grid(nx, ny).pole_row_spacing()
    assert abs(dx - printed) < 0.5, dx


def test_external_mode_courant_number_matches_paper():
    # sqrt(g H_o) with H_o = 8 km is quoted as 280 m/s; the maximal Courant
    # numbers reported at 512x256 with dt = 200 s are 116 and 118
    cel = GOLDEN["external_mode_celerity_m_per_s"]
    c = np.sqrt(GRAVITY * cel["depth_m"])
    assert abs(c - cel["value"]) < 0.5
    cou = GOLDEN["max_external_courant"]
    courant = c * cou["dt_s"] / Grid(*cou["grid"]).pole_row_spacing()
    assert min(cou["values"]) - 1.0 < courant < max(cou["values"]) + 1.0


@pytest.mark.parametrize("nx,ny,dt", GOLDEN["time_steps_s"]["grids"])
def test_paper_time_steps_far_exceed_explicit_limit(nx, ny, dt):
    # the explicit scheme would need dt ~ 40, 10, 2.5 s; the paper's steps are
    # 20x-80x longer, so the zonal pole-row problem must be handled implicitly
    c = np.sqrt(GRAVITY * 8000.0)
    assert c * dt / Grid(nx, ny).pole_row_spacing() > 20.0


def test_absorber_profile_shape():
    amax = 1.0 / (200.0 * 200.0)
    assert absorber_profile(np.array([np.pi / 2]), amax)[0] == pytest.approx(amax)
    assert absorber_profile(np.array([np.pi / 2 - 3 * np.pi / 64]), amax)[0] == pytest.approx(0.0)
    assert absorber_profile(np.array([-(np.pi / 2 - 1.5 * np.pi / 64)]), amax)[0] == pytest.approx(0.5 * amax)
    assert absorber_profile(np.array([0.3]), amax)[0] == 0.0


# --------------------------------------------------------------------------
# the operator derived symbolically from the paper's equations
# --------------------------------------------------------------------------
lam_s, phi_s = sy.symbols("lam phi", real=True)
_X = sy.cos(phi_s) * sy.cos(lam_s)
_Y = sy.cos(phi_s) * sy.sin(lam_s)
_Z = sy.sin(phi_s)


def _derived_operator(depth, orography, field, dt, alpha):
    """L(field) obtained from the paper's equations, not from the oracle's
    coefficient formulas:
    * linearised pressure gradient (eq. rhslin), terms linear in Phi^{n+1}:
      P = (Phi grad(Phi*+H0) + Phi* grad Phi) / 2;
    * momentum forcings (eqs. RSWE2-3) with pressure gradient, Coriolis and
      relaxation implicit, so Q = (dt/2) R^{n+1} (eq. MPDATA, implicit part),
      solved for (Qx, Qy) symbolically (the 2x2 inversion of eq. Qexpr);
    * trapezoidal continuity (eq. SWE1) with v Phi = (Qx h_y, Qy h_x):
      G Phi/dt + (1/2) div = ... ; multiplied by -2 this is L(Phi) - R = 0.
    """
    a, g, om = RADIUS, GRAVITY, OMEGA
    hx, hy = a * sy.cos(phi_s), a
    G = hx * hy
    f = 2 * om * sy.sin(phi_s)
    d = sy.Rational(1, 2) * dt
    hstar = depth + orography
    px = (field * sy.diff(hstar, lam_s) + depth * sy.diff(field, lam_s)) / 2
    py = (field * sy.diff(hstar, phi_s) + depth * sy.diff(field, phi_s)) / 2
    qx, qy = sy.symbols("qx qy")
    sol = sy.solve([sy.Eq(qx, d * (-(g / hx) * px + f * qy - alpha * qx)),
                    sy.Eq(qy, d * (-(g / hy) * py - f * qx - alpha * qy))], [qx, qy], dict=True)[0]
    div = sy.diff(hy * sol[qx], lam_s) + sy.diff(hx * sol[qy], phi_s)
    expr = -div - 2 * G * field / dt
    return sy.lambdify((lam_s, phi_s), expr, "numpy")


def _sample(expr, nx, ny):
    fn = sy.lambdify((lam_s, phi_s), expr, "numpy")
    g = Grid(nx, ny)
    LA, PH = np.meshgrid(g.lam, g.lat)
    return np.broadcast_to(fn(LA, PH), (ny, nx)).astype(np.float64)


def _weighted_rel_err(num, ref, lat):
    w = np.cos(lat)[:, None]
    return np.sqrt(np.sum(w * (num - ref) ** 2) / np.sum(w * ref ** 2))


def _order_study(depth, oro, field, dt, alpha_expr, absorber, grids):
    lop = _derived_operator(depth, oro, field, dt, alpha_expr)
    errs = []
    for nx, ny in grids:
        g = Grid(nx, ny)
        LA, PH = np.meshgrid(g.lam, g.lat)
        op = EllipticOperator(nx, ny, _sample(depth, nx, ny), dt,
                              orography=_sample(oro, nx, ny), absorber=absorber)
        num = op.apply(_sample(field, nx, ny))
        ref = np.broadcast_to(lop(LA, PH), (ny, nx))
        errs.append(_weighted_rel_err(num, ref, g.lat))
    return errs


GRIDS = [(32, 16), (64, 32), (128, 64), (256, 128)]


def test_operator_matches_paper_equations_second_order():
    depth = 8000 + 500 * (0.3 * _X + 0.5 * _Y * _Z + 0.2 * _Z ** 2 + 0.4 * _X * _Y)
    oro = 600 * (0.5 + 0.3 * _X * _Z + 0.2 * _Y + 0.1 * _Z)
    field = _X ** 2 - 0.5 * _Y + _Z ** 3 + _X * _Z + 0.3 * _Y * _Z
    errs = _order_study(depth, oro, field, 600.0, 0, 0.0, GRIDS)
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[-1] < 1e-3, errs
    assert min(orders[1:]) > 1.8, (errs, orders)


def test_operator_with_absorber_matches_paper_equations():
    # absorber alpha(lat) enters the implicit relaxation of the momentum; the
    # profile has a kink, so only convergence (not a clean order) is asked
    amax = 1.0 / (2.0 * 600.0)
    dist = sy.pi / 2 - sy.Abs(phi_s)
    alpha = amax * sy.Max(0, 1 - dist / (3 * sy.pi / 64))
    depth = 8000 + 400 * (0.5 * _X * _Z + 0.3 * _Y)
    oro = 300 * (1 + _X * _Y)
    field = _Z ** 2 + 0.5 * _X * _Y + _Y
    errs = _order_study(depth, oro, field, 600.0, alpha, amax, GRIDS)
    assert errs[-1] < 5e-3 and errs[-1] < errs[0] / 10, errs


@pytest.mark.parametrize("l,m", [(3, 2), (5, 0), (6, 4)])
def test_closed_form_eigenfunction(l, m):
    # f = 0, no absorber, flat orography, uniform depth: B = 0 and
    # L = kappa cos(lat) Lap_S - 2 a^2 cos(lat)/dt, so L Y_lm is
    # -cos(lat) (kappa l(l+1) + 2 a^2/dt) Y_lm with kappa = dt g H / 4
    H, dt = 8000.0, 600.0
    kappa = dt * GRAVITY * H / 4.0
    errs = []
    for nx, ny in GRIDS:
        g = Grid(nx, ny)
        LA, PH = np.meshgrid(g.lam, g.lat)
        from scipy.special import sph_harm_y
        y = sph_harm_y(l, m, 0.5 * np.pi - PH, LA).real
        op = EllipticOperator(nx, ny, np.full((ny, nx), H), dt, omega=0.0)
        ref = -np.cos(PH) * (kappa * l * (l + 1) + 2 * RADIUS ** 2 / dt) * y
        errs.append(_weighted_rel_err(op.apply(y), ref, g.lat))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders[1:]) > 1.8, (errs, orders)
    assert errs[-1] < 1e-3


# --------------------------------------------------------------------------
# algebraic properties
# --------------------------------------------------------------------------
def _random_op(nx, ny, seed, **kw):
    rng = np.random.default_rng(seed)
    depth = 8000 + 300 * rng.standard_normal((ny, nx))
    oro = 200 * rng.random((ny, nx))
    return EllipticOperator(nx, ny, depth, 600.0, orography=oro, **kw)


def test_adjoint_identity_without_rotation_and_b_terms():
    op = _random_op(32, 16, 1, omega=0.0, b_terms=False, absorber=1e-4)
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal((2, 16, 32))
    lhs, rhs = np.sum(u * op.apply(v)), np.sum(op.apply(u) * v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_rotation_makes_operator_non_symmetric():
    op = _random_op(16, 8, 3, b_terms=False)
    m = op.dense()
    asym = np.linalg.norm(m - m.T) / np.linalg.norm(m)
    assert asym > 1e-6
    op_b = _random_op(16, 8, 3, omega=0.0)          # B terms alone also break symmetry
    m_b = op_b.dense()
    assert np.linalg.norm(m_b - m_b.T) / np.linalg.norm(m_b) > 1e-8


def test_negative_definite():
    op = _random_op(16, 8, 4)
    m = op.dense()
    sym = 0.5 * (m + m.T)
    assert np.max(np.linalg.eigvalsh(sym)) < 0.0


def test_diagonal_matches_dense():
    op = _random_op(16, 8, 5, absorber=1e-3)
    assert np.allclose(op.diagonal().ravel(), np.diag(op.dense()), rtol=1e-13, atol=0)


def test_stencil_is_nine_point_with_across_pole_partners():
    # a unit impulse in the south polar row only reaches its zonal neighbours,
    # the row above, and the points half a circle away in the same row
    nx, ny = 16, 8
    op = _random_op(nx, ny, 6)
    u = np.zeros((ny, nx))
    u[0, 3] = 1.0
    col = op.apply(u)
    reached = set(zip(*np.nonzero(col)))
    allowed = {(j, i % nx) for j in (0, 1) for i in (2, 3, 4)}
    allowed |= {(0, (i + nx // 2) % nx) for i in (2, 3, 4)}
    assert reached <= allowed
    assert (0, (3 + nx // 2 + 1) % nx) in reached or (0, (3 + nx // 2 - 1) % nx) in reached


def test_linear_and_shape_preserving():
    op = _random_op(32, 16, 7)
    rng = np.random.default_rng(8)
    u, v = rng.standard_normal((2, 16, 32))
    assert np.allclose(op.apply(2.0 * u - 3.0 * v), 2.0 * op.apply(u) - 3.0 * op.apply(v), rtol=1e-12, atol=1e-3)
