"""Split single-precision residual (paper Section 4.2.1, eq. L_Operator_SP)
through the C-ABI, against the oracle (oracle/split.py).

Float32 rows: the GPU forms its float32 coefficients from Phi* in float32
(scaled by dt/2a^2) where the oracle rounds the float64 ones, and sums in its
own order, so the two agree to a few float32 ulps of the stencil's summands
(including C Phi_SP, much larger than r).  Float64 polar rows: the operator
parity bound."""
import numpy as np
import pytest
import torch

from oracle.operator import EllipticOperator
from oracle.split import split_fields, base_differences, residual_split, residual_naive_sp
from workloads import problem
from test_gpu_parity import stencil_magnitude, dev, host, EPS

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


def _case(nx, ny, oro=False):
    pr = problem(2, nx, ny, dt=600.0)
    orog = 1500.0 * np.random.default_rng(5).random((ny, nx)) if oro else None
    op = EllipticOperator(nx, ny, pr["depth"], 600.0, orography=orog)
    phi = pr["depth"] + 3.0 * pr["x_true"]
    base = pr["depth"] - 20.0 * pr["x_true"]
    rhs = op.apply(phi + 5.0 * pr["x_true"])
    hat, _ = split_fields(base)
    tilde = (phi - hat.astype(np.float64)).astype(np.float32)
    return pr, orog, op, phi, base, rhs, hat, tilde


@pytest.mark.parametrize("nx,ny,polar,oro", [(64, 32, 1, False), (256, 128, 3, False), (512, 256, 3, True),
                                             (512, 256, 0, False), (16, 6, 2, False), (1024, 512, 4, False)])
def test_split_residual_matches_oracle(gpu_lib, nx, ny, polar, oro):
    pr, orog, op, phi, base, rhs, hat, tilde = _case(nx, ny, oro)
    s = gpu_lib.Solver([(nx, ny)], polar_rows=polar)
    s.set_operator(0, pr["depth"], 600.0, orography=orog)
    s.set_split_base(0, dev(base))
    r = host(s.residual_split(0, torch.from_numpy(tilde).cuda(), dev(rhs)))
    ref = residual_split(op, hat, base_differences(hat), tilde, rhs, polar=polar)
    sp = hat.astype(np.float64) + tilde.astype(np.float64)
    mag = stencil_magnitude(op, sp)
    rows32 = np.r_[polar:ny - polar]
    rows64 = np.r_[0:polar, ny - polar:ny] if polar else np.r_[0:0]
    bound32 = 64 * EPS32 * mag[rows32] + EPS32 * np.abs(ref[rows32])
    assert np.all(np.abs(r[rows32] - ref[rows32]) <= bound32), np.max(np.abs(r[rows32] - ref[rows32]) / bound32)
    assert np.all(r[rows32] == r[rows32].astype(np.float32))
    if len(rows64):
        bound64 = 32 * EPS * mag[rows64]
        assert np.all(np.abs(r[rows64] - ref[rows64]) <= bound64)


def test_split_residual_accuracy_at_the_poles(gpu_lib):
    # the paper's property, on the GPU: without float64 bands the split
    # float32 residual is orders of magnitude closer to the float64 one than
    # the plain float32 evaluation next to the poles
    nx, ny = 512, 256
    pr, orog, op, phi, base, rhs, hat, tilde = _case(nx, ny)
    s = gpu_lib.Solver([(nx, ny)], polar_rows=0)
    s.set_operator(0, pr["depth"], 600.0)
    s.set_split_base(0, dev(base))
    r = host(s.residual_split(0, torch.from_numpy(tilde).cuda(), dev(rhs)))
    ref = op.apply(phi) - rhs
    naive = residual_naive_sp(op, phi, rhs)

    def rowerr(x):
        return np.sqrt(np.mean((x - ref) ** 2, axis=1) / np.mean(ref ** 2, axis=1))

    assert np.all(rowerr(r)[[0, -1]] * 100 < rowerr(naive)[[0, -1]])
    assert np.median(rowerr(r)) < 1e-3


def test_split_residual_errors(gpu_lib):
    s = gpu_lib.Solver([(64, 32)])
    pr = problem(1, 64, 32)
    s.set_operator(0, pr["depth"], 600.0)
    t = torch.zeros((32, 64), dtype=torch.float32, device="cuda")
    rhs = dev(np.zeros((32, 64)))
    with pytest.raises(gpu_lib.GcrError):
        s.residual_split(0, t, rhs)              # no base yet
    s.set_split_base(0, dev(pr["depth"]))
    with pytest.raises(gpu_lib.GcrError):
        s.residual_split(0, t, rhs, out=rhs)     # r aliases R
    r = host(s.residual_split(0, t, rhs))
    assert np.all(np.isfinite(r))
