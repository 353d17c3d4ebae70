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

from oracle.gcr import gcr
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


@pytest.mark.parametrize("precision", [4, 5])
def test_single_solve_from_split_r0_vs_oracle(gpu_lib, precision):
    """The split residual as a solve's r_0 (GCR_F_SPLIT_R0, paper Section
    4.2.1): two consecutive warm-started steps of a depth-like unknown share
    one base taken earlier, as the paper keeps the base for many time steps.
    Each step's GPU solve (float32 cycle) is compared with oracle/split.py's
    residual of the same warm start followed by the oracle's GCR from that
    residual: the two evaluate the split float32 residual in different
    orders, so their r_0 differ by float32 ulps of the stencil's largest
    summand (C Phi_SP, about 1e3 times r_0 here), which bounds how far their
    increments x - x_0 can differ (2e-3 of the increment)."""
    nx, ny = 256, 128
    polar = 2                # the default polar rows at NY = 128: the split's float64 bands
    pr = problem(2, nx, ny, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    base = pr["depth"] - 20.0 * pr["x_true"]
    hat, _ = split_fields(base)
    dh = base_differences(hat)
    s = gpu_lib.Solver([(nx, ny)], precision=precision, rtol=1e-5, max_iters=40, flags=gpu_lib.F_SPLIT_R0)
    s.set_operator(0, pr["depth"], 600.0)
    s.set_split_base(0, dev(base))
    x0 = pr["depth"].copy()
    for step in range(2):
        target = pr["depth"] + (3.0 + 2.0 * step) * pr["x_true"]
        rhs = op.apply(target)
        tilde = (x0 - hat.astype(np.float64)).astype(np.float32)
        r0 = residual_split(op, hat, dh, tilde, rhs, polar=polar)
        ores = gcr(op, rhs, x0=x0, r0=r0, rtol=1e-5)
        x = dev(x0)
        rep = s.solve([dev(rhs)], [x])[0]
        xg = host(x)
        assert rep.status == gpu_lib.OK, rep
        assert rep.r0_norm == pytest.approx(np.linalg.norm(r0), rel=1e-3)
        inc_g, inc_o = xg - x0, ores.x - x0
        assert np.linalg.norm(inc_g - inc_o) <= 2e-3 * np.linalg.norm(inc_o), (step, rep)
        # the split start is accurate: against the float64 residual of x_0 the
        # solve reduces the error of the state by orders of magnitude
        true0 = np.linalg.norm(op.apply(x0) - rhs)
        assert np.linalg.norm(op.apply(xg) - rhs) <= 1e-2 * true0
        x0 = xg
    s.close()


def test_split_r0_needs_a_base(gpu_lib):
    pr = problem(2, 64, 32, dt=600.0)
    s = gpu_lib.Solver([(64, 32)], precision=gpu_lib.SINGLE, flags=gpu_lib.F_SPLIT_R0)
    s.set_operator(0, pr["depth"], 600.0)
    x = dev(pr["depth"])
    with pytest.raises(gpu_lib.GcrError) as ei:
        s.solve([dev(np.zeros((32, 64)))], [x])
    assert ei.value.code == gpu_lib.ESTATE
    s.close()
