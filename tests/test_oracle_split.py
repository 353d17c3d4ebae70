"""Pins of the split single-precision residual oracle (paper Section 4.2.1,
eq. L_Operator_SP), CPU only."""
import numpy as np
import pytest

from oracle.operator import EllipticOperator
from oracle.split import split_fields, base_differences, face_differences, residual_split, residual_naive_sp
from workloads import problem


def _state(nx, ny):
    pr = problem(2, nx, ny, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    phi = pr["depth"] + 3.0 * pr["x_true"]          # a depth near Phi*
    base = pr["depth"] - 20.0 * pr["x_true"]        # the base, taken some steps before
    rhs = op.apply(phi + 5.0 * pr["x_true"])        # R of the next state: r_0 = L(phi) - R
    hat, _ = split_fields(base)
    tilde = (phi - hat.astype(np.float64)).astype(np.float32)
    return op, phi, rhs, hat, tilde


def test_split_fields_recover_the_depth():
    pr = problem(2, 64, 32)
    hat, tilde = split_fields(pr["depth"])
    assert hat.dtype == np.float32 and tilde.dtype == np.float32
    err = np.abs(hat.astype(np.float64) + tilde.astype(np.float64) - pr["depth"])
    assert np.max(err / pr["depth"]) < 1e-14       # float64-level, as the paper states
    assert np.max(np.abs(tilde)) <= np.max(np.abs(pr["depth"])) * 2.0 ** -24


@pytest.mark.parametrize("nx,ny", [(64, 32), (256, 128)])
def test_float64_split_formula_is_the_operator(nx, ny):
    # linearity: differences of Phi_hat plus those of Phi_tilde, and the B, C
    # terms on their sum, give L(Phi_hat + Phi_tilde) when nothing is rounded
    op, phi, rhs, hat, tilde = _state(nx, ny)
    dh = face_differences(hat.astype(np.float64), np.float64)
    r = residual_split(op, hat, dh, tilde, rhs, polar=0, dtype=np.float64)
    ref = op.apply(hat.astype(np.float64) + tilde.astype(np.float64)) - rhs
    assert np.max(np.abs(r - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_face_differences_by_hand():
    phi = np.arange(4 * 6, dtype=np.float64).reshape(4, 6) ** 1.5
    d = face_differences(phi, np.float64)
    i, j = 2, 1
    assert d["lon_e"][j, i] == phi[j, i + 1] - phi[j, i]
    assert d["lat_e"][j, i] == phi[j + 1, i] - phi[j - 1, i] + phi[j + 1, i + 1] - phi[j - 1, i + 1]
    assert d["lat_n"][j, i] == phi[j + 1, i] - phi[j, i]
    assert d["lon_n"][j, i] == phi[j, i + 1] - phi[j, i - 1] + phi[j + 1, i + 1] - phi[j + 1, i - 1]
    # row 0: the row beyond the south pole is row 0 shifted by NX/2
    assert d["lat_e"][0, i] == phi[1, i] - phi[0, (i + 3) % 6] + phi[1, i + 1] - phi[0, (i + 4) % 6]


def test_split_reduces_the_float32_error_most_at_the_poles():
    # the property the paper reports for eq. L_Operator_SP: against the float64
    # residual, the split float32 evaluation is far more accurate than the
    # plain float32 one next to the poles (orders of magnitude), and not worse
    # elsewhere
    op, phi, rhs, hat, tilde = _state(512, 256)
    ref = op.apply(phi) - rhs
    rs = residual_split(op, hat, base_differences(hat), tilde, rhs, polar=0)
    rn = residual_naive_sp(op, phi, rhs)

    def rowerr(r):
        return np.sqrt(np.mean((r - ref) ** 2, axis=1) / np.mean(ref ** 2, axis=1))

    es, en = rowerr(rs), rowerr(rn)
    assert np.all(es[[0, -1]] * 100 < en[[0, -1]])
    assert np.linalg.norm(rs - ref) < np.linalg.norm(rn - ref)
    assert np.median(es) < 1e-3


def test_polar_bands_take_the_float64_operator():
    op, phi, rhs, hat, tilde = _state(64, 32)
    r = residual_split(op, hat, base_differences(hat), tilde, rhs, polar=3)
    full = op.apply(hat.astype(np.float64) + tilde.astype(np.float64)) - rhs
    assert np.array_equal(r[:3], full[:3]) and np.array_equal(r[-3:], full[-3:])
    assert not np.array_equal(r[3:-3], full[3:-3])
    assert np.all(r[3:-3] == r[3:-3].astype(np.float32))
