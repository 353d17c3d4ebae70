"""Parity of the HIP path with the float64 oracle, through the C-ABI.

Operator and preconditioner: element by element, within a bound derived from
float64 rounding of the stencil's summands (operator) or from the row
systems' conditioning (preconditioner).  Full solves: the tolerances of the
solver's contract -- float64 form: true relative residual at the requested
tolerance, the oracle's iteration count +-1, solution within 1e-9 of the
oracle's; mixed forms: relative L2 distance to the oracle's solution <= 1e-5.
"""
import numpy as np
import pytest
import torch

from oracle.operator import EllipticOperator
from oracle.precond import Preconditioner
from oracle.gcr import gcr, CONVERGED
from workloads import problem, batch_problems

from form_emul import stencil_magnitude

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make_solver(lib, sizes, **kw):
    return lib.Solver(sizes, **kw)


OPS = [
    # nx, ny, dt, extras
    (64, 32, 600.0, {}),
    (128, 64, 400.0, dict(absorber=1.0 / (2 * 400.0), orography=True)),
    (256, 128, 600.0, dict(b_terms=False)),
    (512, 256, 600.0, {}),
    (1024, 512, 100.0, dict(orography=True)),
    (8, 2, 600.0, {}),
    (16, 7, 900.0, dict(absorber=1e-3)),
    (1024, 512, 100.0, dict(orography="smooth")),
]


def _build(nx, ny, dt, extras, seed=0):
    pr = problem(2, nx, ny, instance=seed, dt=dt)
    oro = None
    if extras.get("orography") == "smooth":     # degree <= 16 harmonics, 0..3000 m
        from workloads import harmonic_field
        f = harmonic_field(nx, ny, 16, np.random.default_rng(177 + seed), lmin=1)
        oro = 1500.0 * (1.0 + f / np.max(np.abs(f)))
    elif extras.get("orography"):               # white noise, 0..1500 m: a stress case
        rng = np.random.default_rng(77 + seed)
        oro = 1500.0 * rng.random((ny, nx))
    kw = dict(absorber=extras.get("absorber", 0.0), b_terms=extras.get("b_terms", True))
    op = EllipticOperator(nx, ny, pr["depth"], dt, orography=oro, **kw)
    return pr, oro, kw, op


@pytest.mark.parametrize("nx,ny,dt,extras", OPS)
def test_operator_parity(gpu_lib, nx, ny, dt, extras):
    pr, oro, kw, op = _build(nx, ny, dt, extras)
    s = make_solver(gpu_lib, [(nx, ny)])
    s.set_operator(0, pr["depth"], dt, orography=oro, **kw)
    x = np.random.default_rng(5).standard_normal((ny, nx))
    y = host(s.apply_operator(0, dev(x)))
    ref = op.apply(x)
    bound = 32 * EPS * stencil_magnitude(op, x)
    err = np.abs(y - ref)
    assert np.all(err <= bound), (err.max(), (err / bound).max())


@pytest.mark.parametrize("nx,ny,dt,extras", OPS)
def test_operator_parity_device_inputs(gpu_lib, nx, ny, dt, extras):
    # same operator built from device-resident depth/orography
    pr, oro, kw, op = _build(nx, ny, dt, extras, seed=1)
    s = make_solver(gpu_lib, [(nx, ny)])
    s.set_operator(0, dev(pr["depth"]), dt, orography=None if oro is None else dev(oro), **kw)
    x = pr["x_true"]
    y = host(s.apply_operator(0, dev(x)))
    ref = op.apply(x)
    assert np.all(np.abs(y - ref) <= 32 * EPS * stencil_magnitude(op, x))


@pytest.mark.parametrize("nx,ny,dt,extras", OPS)
@pytest.mark.parametrize("option,iters", [(3, 2), (3, 1), (3, 4), (0, 1), (1, 1), (2, 2), (2, 3)])
def test_preconditioner_parity(gpu_lib, nx, ny, dt, extras, option, iters):
    pr, oro, kw, op = _build(nx, ny, dt, extras)
    s = make_solver(gpu_lib, [(nx, ny)], precond=option, richardson_iters=iters)
    s.set_operator(0, pr["depth"], dt, orography=oro, **kw)
    r = np.random.default_rng(9).standard_normal((ny, nx))
    e = host(s.apply_precond(0, dev(r)))
    ref = Preconditioner(op, option, iters)(r)
    tol = preconditioner_bound(op, option, iters, r, ref)
    # the bound is relative to the result, so a zero or a 1%-perturbed output
    # fails: at 90% of the points at least, and everywhere the bound stays
    # below 1e-6 of max |ref| -- except with white-noise orography and two or
    # more Richardson iterations, where the zonal B terms of P^M (grid-scale
    # gradients of H* over cos(lat)) outweigh the meridional terms eta is
    # scaled by, and the worst-case propagation through the iterations next to
    # the poles is far above 1e-6 (its rows are still checked at that bound)
    assert np.mean(0.01 * np.abs(ref) > tol) > 0.9
    if not (extras.get("orography") is True and option == 3 and iters >= 2):
        assert np.max(tol) <= 1e-6 * np.max(np.abs(ref))
    err = np.abs(e - ref)
    assert np.all(err <= tol), (float(np.max(err / np.maximum(tol, 1e-300))), float(np.max(err)))


def preconditioner_bound(op, option, iters, r, ref):
    """Pointwise float64 rounding bound of P^{-1}(r), 64 eps per rounding
    step, relative to the local magnitude of the iterates (rows j-1..j+1).
    Option 3: form_emul.richardson_bound with float64's unit roundoff.
    Option 2: each later iteration evaluates L (sum |L summands| / |diag|)
    and propagates an earlier error by at most 1 + that factor."""
    from form_emul import rows_max3, richardson_bound
    if option == 0:
        return np.zeros_like(ref)
    its = [Preconditioner(op, option, mu)(r) for mu in range(1, iters + 1)] if option in (2, 3) else [ref]
    local = np.max([rows_max3(q) for q in its], axis=0)
    c = 64 * EPS
    if option == 1:   # e = r / diag(L): the diagonal's own rounding, with the latitude conditioning
        a = np.max(stencil_magnitude(op, np.ones_like(ref)) / np.abs(op.diagonal()), axis=1)[:, None]
        return c * a * local
    if option == 2:
        a = np.max(stencil_magnitude(op, np.ones_like(ref)) / np.abs(op.diagonal()), axis=1)[:, None]
        delta = c * local
        for _ in range(1, iters):
            delta = rows_max3(delta) * (1.0 + a) + c * (1.0 + a) * local
        return delta
    return richardson_bound(op, iters, local, EPS)


def _solve_pair(lib, pr, op, nx, ny, rtol, precision=0, **kw):
    rhs = op.apply(pr["x_true"])
    ores = gcr(op, rhs, rtol=rtol, max_iters=kw.get("max_iters", 200))
    s = make_solver(lib, [(nx, ny)], precision=precision, rtol=rtol, record_history=True, **kw)
    s.set_operator(0, pr["depth"], pr["dt"])
    x = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    rep = s.solve([dev(rhs)], [x], record_history=True)[0]
    assert len(rep.history) == rep.iterations + 1
    return ores, rep, host(x), rhs


def test_config1_fp64_parity(gpu_lib):
    # 64x32, dt = 600 s, rtol 1e-10, GCR(3), option 3 with two Richardson iterations
    pr = problem(1, 64, 32, dt=600.0)
    op = EllipticOperator(64, 32, pr["depth"], 600.0)
    ores, rep, x, rhs = _solve_pair(gpu_lib, pr, op, 64, 32, 1e-10)
    assert ores.status == CONVERGED and rep.status == gpu_lib.OK
    assert abs(rep.iterations - ores.iterations) <= 1
    assert rep.rel_res_true <= 1e-10
    true_res = np.linalg.norm(op.apply(x) - rhs) / ores.r0_norm
    assert true_res <= 1e-10
    assert np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x) <= 1e-9
    assert rep.r0_norm == pytest.approx(ores.r0_norm, rel=1e-12)
    n = min(len(rep.history), len(ores.history))
    assert n >= 4
    assert np.allclose(rep.history[:n], ores.history[:n], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("nx,ny", [(256, 128), (512, 256)])
def test_fp64_parity(gpu_lib, nx, ny):
    pr = problem(2, nx, ny, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    ores, rep, x, rhs = _solve_pair(gpu_lib, pr, op, nx, ny, 1e-8)
    assert rep.status == gpu_lib.OK
    assert abs(rep.iterations - ores.iterations) <= 1
    assert rep.rel_res_true <= 1e-8
    assert np.linalg.norm(op.apply(x) - rhs) / ores.r0_norm <= 1e-8
    assert np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x) <= 1e-9


@pytest.mark.parametrize("nx,ny", [(256, 128), (512, 256)])
@pytest.mark.parametrize("precision", [1, 2, 3, 4, 5])
def test_mixed_forms_vs_oracle(gpu_lib, nx, ny, precision):
    pr = problem(2, nx, ny, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    ores, rep, x, rhs = _solve_pair(gpu_lib, pr, op, nx, ny, 1e-8, precision=precision, max_iters=60)
    err = np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x)
    true_res = np.linalg.norm(op.apply(x) - rhs) / ores.r0_norm
    print(f"\nprecision={precision} {nx}x{ny}: status={rep.status} it={rep.iterations} "
          f"restarts={rep.restarts} rec={rep.rel_res_recursive:.3e} true={rep.rel_res_true:.3e} "
          f"(host {true_res:.3e}) err_vs_oracle={err:.3e} oracle_it={ores.iterations}")
    assert rep.rel_res_true == pytest.approx(true_res, rel=1e-6, abs=1e-14)
    if precision in (2, 3):
        # residual replacement: converged on the float64 true residual
        assert rep.status == gpu_lib.OK and true_res <= 1e-8
    if precision in (4, 5):
        # float32 cycle without replacement (5: float64 polar bands): a float32
        # plateau (1e-7 to 1e-6 here), below the float16 one of precision 1
        # (about 3e-5)
        assert rep.status == gpu_lib.OK and true_res <= 1e-5 and err <= 1e-6
    if precision == 3:
        # float32 operator inside the iteration: the float64 iteration count +-1
        assert abs(rep.iterations - ores.iterations) <= 1
    assert err <= 1e-5


def test_zero_rhs_and_exact_guess(gpu_lib):
    pr = problem(1, 64, 32)
    s = make_solver(gpu_lib, [(64, 32)])
    s.set_operator(0, pr["depth"], 600.0)
    x = torch.zeros((32, 64), dtype=torch.float64, device="cuda")
    rep = s.solve([torch.zeros_like(x)], [x])[0]
    assert rep.status == gpu_lib.OK and rep.iterations == 0 and torch.all(x == 0)
    # exact initial guess: r_0 == 0 up to rounding -> at most one cycle
    op = EllipticOperator(64, 32, pr["depth"], 600.0)
    xt = dev(pr["x_true"])
    rhs = s.apply_operator(0, xt)
    x2 = xt.clone()
    rep = s.solve([rhs], [x2])[0]
    assert rep.status in (gpu_lib.OK, gpu_lib.STAGNATED)
    assert torch.allclose(x2, xt, rtol=0, atol=1e-12)


@pytest.mark.parametrize("precision", [0, 3])
def test_warm_start_batch_all_widths(gpu_lib, precision):
    """Nonzero initial guesses in a batch spanning every points-per-lane class
    (nx = 8 .. 1024): the caller's x and rhs are read in place by the first
    residual (pole rows included) and x is written back by the last one.
    Same guess in the oracle: same r_0 and, in float64, the same solution."""
    sizes = [(8, 4), (64, 16), (128, 32), (256, 16), (1024, 8)]
    rtol = 1e-10 if precision == 0 else 1e-8
    s = make_solver(gpu_lib, sizes, precision=precision, rtol=rtol, max_iters=100)
    rng = np.random.default_rng(7)
    ops, rhs, x0, xs = [], [], [], []
    for m, (nx, ny) in enumerate(sizes):
        pr = problem(2, nx, ny, instance=m, dt=600.0)
        op = EllipticOperator(nx, ny, pr["depth"], 600.0)
        s.set_operator(m, pr["depth"], 600.0)
        ops.append(op)
        rhs.append(op.apply(pr["x_true"]))
        g = pr["x_true"] + 0.3 * np.std(pr["x_true"]) * rng.standard_normal((ny, nx))
        x0.append(g)
        xs.append(dev(g))
    rhs_d = [dev(r) for r in rhs]
    reps = s.solve(rhs_d, xs)
    for m, (nx, ny) in enumerate(sizes):
        op = ops[m]
        ores = gcr(op, rhs[m], x0=x0[m], rtol=rtol, max_iters=100)
        x = host(xs[m])
        rep = reps[m]
        assert np.array_equal(host(rhs_d[m]), rhs[m]), "rhs must be read only"
        assert rep.r0_norm == pytest.approx(ores.r0_norm, rel=1e-12), (nx, ny)
        true_res = np.linalg.norm(op.apply(x) - rhs[m]) / ores.r0_norm
        assert rep.rel_res_true == pytest.approx(true_res, rel=1e-6, abs=1e-14), (nx, ny)
        assert rep.status == gpu_lib.OK and true_res <= rtol, (nx, ny, rep)
        err = np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x)
        assert err <= (1e-9 if precision == 0 else 1e-6), (nx, ny, err)
        if precision == 0:
            assert abs(rep.iterations - ores.iterations) <= 1, (nx, ny, rep.iterations, ores.iterations)


@pytest.mark.parametrize("precision", [0, 3])
@pytest.mark.parametrize("oro", [False, True])
def test_residual_1024_point_rows(gpu_lib, precision, oro):
    """Rows of 1024 points take the float64 residual in two halves: the
    first residual (r_0, from the caller's x and rhs in natural order, poles
    included) against the oracle's to 1e-12, the final one (pooled x)
    against the host's recomputation; with orography the kernels read H*."""
    nx, ny, dt = 1024, 12, 100.0
    rtol = 1e-10 if precision == 0 else 1e-8
    pr = problem(2, nx, ny, instance=5, dt=dt)
    h0 = 1500.0 * np.random.default_rng(3).random((ny, nx)) if oro else None
    op = EllipticOperator(nx, ny, pr["depth"], dt, orography=h0)
    rhs = op.apply(pr["x_true"])
    g = pr["x_true"] + 0.3 * np.std(pr["x_true"]) * np.random.default_rng(4).standard_normal((ny, nx))
    s = make_solver(gpu_lib, [(nx, ny)], precision=precision, rtol=rtol, max_iters=100)
    s.set_operator(0, pr["depth"], dt, orography=h0)
    x = dev(g)
    rep = s.solve([dev(rhs)], [x])[0]
    ores = gcr(op, rhs, x0=g, rtol=rtol, max_iters=100)
    assert rep.r0_norm == pytest.approx(ores.r0_norm, rel=1e-12)
    xh = host(x)
    true_res = np.linalg.norm(op.apply(xh) - rhs) / ores.r0_norm
    assert rep.rel_res_true == pytest.approx(true_res, rel=1e-6, abs=1e-14)
    assert rep.status == gpu_lib.OK and true_res <= rtol, rep
    err = np.linalg.norm(xh - ores.x) / np.linalg.norm(ores.x)
    assert err <= (1e-9 if precision == 0 else 1e-6), err


@pytest.mark.parametrize("precision", [0, 3])
def test_largest_grid_solve(gpu_lib, precision):
    """The largest grid the library takes (1024 x 4096, 4.2 M points, polar
    rows 9.6 m wide): too large for the oracle's GCR, so the GPU solution is
    checked through the oracle's operator -- its true residual and r_0 --
    which holds at any size."""
    nx, ny, rtol = 1024, 4096, 1e-8
    pr = problem(2, nx, ny, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    rhs = op.apply(pr["x_true"])
    s = make_solver(gpu_lib, [(nx, ny)], precision=precision, rtol=rtol, max_iters=200)
    s.set_operator(0, pr["depth"], 600.0)
    x = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    rep = s.solve([dev(rhs)], [x])[0]
    print(f"\n{nx}x{ny} precision={precision}: status={rep.status} it={rep.iterations} "
          f"true={rep.rel_res_true:.3e}")
    r0 = np.linalg.norm(rhs)
    assert rep.r0_norm == pytest.approx(r0, rel=1e-12)
    true_res = np.linalg.norm(op.apply(host(x)) - rhs) / r0
    assert rep.status == gpu_lib.OK and true_res <= rtol
    assert rep.rel_res_true == pytest.approx(true_res, rel=1e-6, abs=1e-14)
    err = np.linalg.norm(host(x) - pr["x_true"]) / np.linalg.norm(pr["x_true"])
    assert err <= 1e-5


def test_largest_batch_of_smallest_grids(gpu_lib):
    """4096 members (the largest batch) of 8 x 4 grids, each with its own
    depth field and time step, in one solve; sampled members vs the oracle."""
    nx, ny, B = 8, 4, 4096
    prs = [problem(2, nx, ny, instance=m, dt=300.0 + 900.0 * (m % 7) / 6) for m in range(B)]
    s = make_solver(gpu_lib, [(nx, ny)] * B, rtol=1e-10, max_iters=100)
    depth = [dev(p["depth"]) for p in prs]
    s.set_operators(list(range(B)), depth, [p["dt"] for p in prs])
    ops = {}
    rhs = []
    for m, p in enumerate(prs):
        op = EllipticOperator(nx, ny, p["depth"], p["dt"])
        ops[m] = op
        rhs.append(dev(op.apply(p["x_true"])))
    xs = [torch.zeros((ny, nx), dtype=torch.float64, device="cuda") for _ in range(B)]
    reps = s.solve(rhs, xs)
    assert all(r.status == gpu_lib.OK and r.rel_res_true <= 1e-10 for r in reps)
    for m in (0, 1, 2047, 3000, 4095):
        ores = gcr(ops[m], host(rhs[m]), rtol=1e-10, max_iters=100)
        assert abs(reps[m].iterations - ores.iterations) <= 1, m
        err = np.linalg.norm(host(xs[m]) - ores.x) / np.linalg.norm(ores.x)
        assert err <= 1e-9, (m, err)


@pytest.mark.parametrize("precision", [0, 3, 4])
def test_member_groups_equal_one_stream(gpu_lib, precision):
    """A batch large enough to be split into member groups on two streams
    (64 x 512x256) gives bitwise the solutions and reports of the same solve
    on one stream, on every one of repeated solves."""
    B, nx, ny = 64, 512, 256
    prs = [problem(2, nx, ny, instance=m, dt=600.0) for m in range(B)]
    depth = [dev(p["depth"]) for p in prs]
    dts = [p["dt"] for p in prs]
    f = make_solver(gpu_lib, [(nx, ny)] * B)
    f.set_operators(list(range(B)), depth, dts)
    rhs = [f.apply_operator(m, dev(p["x_true"])).clone() for m, p in enumerate(prs)]
    f.close()
    results = []
    for one in (True, False):
        s = make_solver(gpu_lib, [(nx, ny)] * B, precision=precision, one_stream=one)
        s.set_operators(list(range(B)), depth, dts)
        for rep_i in range(1 if one else 3):
            xs = [torch.zeros((ny, nx), dtype=torch.float64, device="cuda") for _ in range(B)]
            reps = s.solve(rhs, xs)
            results.append(([host(x) for x in xs], [(r.status, r.iterations, r.restarts, r.rel_res_true)
                                                    for r in reps]))
        s.close()
    ref_x, ref_r = results[0]
    assert all(st == gpu_lib.OK for st, _, _, _ in ref_r)
    for xs, rr in results[1:]:
        assert rr == ref_r
        assert all(np.array_equal(a, b) for a, b in zip(xs, ref_x))


@pytest.mark.parametrize("precision", [0, 3])
@pytest.mark.parametrize("k", [1, 2, 5, 8])
def test_gcr_windows_many_cycles(gpu_lib, k, precision):
    """GCR(k) for other windows, on a case that runs many cycles (no
    preconditioner): the oracle's iteration count and solution.  Exercises
    the once-per-cycle solution updates with every window length, including
    k = 1 (every iteration ends a cycle)."""
    pr = problem(1, 64, 32)
    op = EllipticOperator(64, 32, pr["depth"], 600.0)
    rhs = op.apply(pr["x_true"])
    ores = gcr(op, rhs, k=k, rtol=1e-7, precond=0, max_iters=800)
    s = make_solver(gpu_lib, [(64, 32)], k=k, precision=precision, precond=0, rtol=1e-7, max_iters=800)
    s.set_operator(0, pr["depth"], 600.0)
    x = torch.zeros((32, 64), dtype=torch.float64, device="cuda")
    rep = s.solve([dev(rhs)], [x])[0]
    assert rep.status == gpu_lib.OK
    err = np.linalg.norm(host(x) - ores.x) / np.linalg.norm(ores.x)
    if precision == 0:
        assert rep.iterations == ores.iterations and err <= 1e-9, (rep.iterations, ores.iterations, err)
    else:
        assert abs(rep.iterations - ores.iterations) <= 2 and err <= 1e-5, (rep.iterations, ores.iterations, err)
    assert np.linalg.norm(op.apply(host(x)) - rhs) <= 1.05e-7 * np.linalg.norm(rhs)


def test_max_iters_reached(gpu_lib):
    pr = problem(1, 64, 32)
    op = EllipticOperator(64, 32, pr["depth"], 600.0)
    rhs = op.apply(pr["x_true"])
    s = make_solver(gpu_lib, [(64, 32)], precond=0, rtol=0.0, max_iters=7)
    s.set_operator(0, pr["depth"], 600.0)
    x = torch.zeros((32, 64), dtype=torch.float64, device="cuda")
    rep = s.solve([dev(rhs)], [x])[0]
    assert rep.status == gpu_lib.NOT_CONVERGED and rep.iterations == 7
    ores = gcr(op, rhs, rtol=0.0, max_iters=7, precond=0)
    assert np.linalg.norm(host(x) - ores.x) <= 1e-9 * np.linalg.norm(ores.x)


def test_linf_exit_matches_oracle(gpu_lib):
    """Maximum-norm exit on a slowly converging case (no preconditioner,
    float64): the iteration count and solution of the oracle with the same
    exit test, over tolerances that fall between iterations; the Euclidean
    exit stops elsewhere for some of them."""
    pr = problem(1, 64, 32)
    op = EllipticOperator(64, 32, pr["depth"], 600.0)
    rhs = op.apply(pr["x_true"])
    differs = 0
    for eps in (1e-3, 1e-5, 1e-7, 1e-9):
        ores = gcr(op, rhs, rtol=eps, precond=0, max_iters=500, norm="linf")
        s = make_solver(gpu_lib, [(64, 32)], precond=0, rtol=eps, max_iters=500, linf_exit=True)
        s.set_operator(0, pr["depth"], 600.0)
        x = torch.zeros((32, 64), dtype=torch.float64, device="cuda")
        rep = s.solve([dev(rhs)], [x])[0]
        assert rep.status == gpu_lib.OK and rep.iterations == ores.iterations, (eps, rep.iterations, ores.iterations)
        assert np.linalg.norm(host(x) - ores.x) <= 1e-9 * np.linalg.norm(ores.x), eps
        r = op.apply(host(x)) - rhs
        assert np.max(np.abs(r)) <= eps * np.max(np.abs(rhs)) * (1 + 1e-6), eps
        differs += ores.iterations != gcr(op, rhs, rtol=eps, precond=0, max_iters=500).iterations
    assert differs >= 2


@pytest.mark.parametrize("precision", [0, 3])
def test_linf_exit_benchmark_batch(gpu_lib, precision):
    """Benchmark-size members (512x256) with the maximum-norm exit: every
    member's true residual meets the test, and the float64 form takes the
    oracle's iteration count."""
    probs = [problem(2, 512, 256, instance=m, dt=600.0) for m in range(4)]
    s = make_solver(gpu_lib, [(512, 256)] * 4, precision=precision, linf_exit=True, rtol=1e-8)
    ops = [EllipticOperator(512, 256, p["depth"], p["dt"]) for p in probs]
    rhs = [op.apply(p["x_true"]) for op, p in zip(ops, probs)]
    s.set_operators([0, 1, 2, 3], [dev(p["depth"]) for p in probs], [p["dt"] for p in probs])
    x = [torch.zeros((256, 512), dtype=torch.float64, device="cuda") for _ in probs]
    reps = s.solve([dev(r) for r in rhs], x)
    for m, (op, r0) in enumerate(zip(ops, rhs)):
        assert reps[m].status == gpu_lib.OK, (m, reps[m])
        r = op.apply(host(x[m])) - r0
        assert np.max(np.abs(r)) <= 1e-8 * np.max(np.abs(r0)) * 1.05, m
        if precision == 0 and m == 0:
            assert reps[m].iterations == gcr(op, r0, rtol=1e-8, norm="linf").iterations


@pytest.mark.parametrize("option", [0, 1, 2])
def test_other_preconditioners_solve(gpu_lib, option):
    pr = problem(1, 64, 32)
    op = EllipticOperator(64, 32, pr["depth"], 600.0)
    rhs = op.apply(pr["x_true"])
    ores = gcr(op, rhs, rtol=1e-10, precond=option, max_iters=500)
    s = make_solver(gpu_lib, [(64, 32)], precond=option, rtol=1e-10, max_iters=500)
    s.set_operator(0, pr["depth"], 600.0)
    x = torch.zeros((32, 64), dtype=torch.float64, device="cuda")
    rep = s.solve([dev(rhs)], [x])[0]
    assert rep.status == gpu_lib.OK
    assert abs(rep.iterations - ores.iterations) <= max(1, ores.iterations // 20)
    assert np.linalg.norm(host(x) - ores.x) / np.linalg.norm(ores.x) <= 1e-8


@pytest.mark.parametrize("precision", [0, 2, 3])
def test_batch_members_equal_solo_solves(gpu_lib, precision):
    probs = batch_problems(3, 5, grids=((64, 32), (128, 64), (256, 128)))
    sizes = [(p["nx"], p["ny"]) for p in probs]
    ops = [EllipticOperator(p["nx"], p["ny"], p["depth"], p["dt"]) for p in probs]
    rhs = [dev(op.apply(p["x_true"])) for op, p in zip(ops, probs)]
    sb = make_solver(gpu_lib, sizes, precision=precision)
    for m, p in enumerate(probs):
        sb.set_operator(m, p["depth"], p["dt"])
    xb = [torch.zeros((ny, nx), dtype=torch.float64, device="cuda") for nx, ny in sizes]
    reps = sb.solve(rhs, xb)
    for m, p in enumerate(probs):
        s1 = make_solver(gpu_lib, [sizes[m]], precision=precision)
        s1.set_operator(0, p["depth"], p["dt"])
        x1 = torch.zeros_like(xb[m])
        r1 = s1.solve([rhs[m]], [x1])[0]
        assert r1.iterations == reps[m].iterations
        assert torch.equal(x1, xb[m]), m
        ores = gcr(ops[m], host(rhs[m]), rtol=1e-8)
        assert np.linalg.norm(host(x1) - ores.x) / np.linalg.norm(ores.x) <= (1e-9 if precision == 0 else 1e-5)


@pytest.mark.parametrize("precision", [0, 3])
def test_orography_and_flat_members_in_one_class(gpu_lib, precision):
    """Members with and without orography in one row class, then the same
    solver after operators change between the two kinds: every solve must
    match the oracle with each member's own operator (a class that is all
    flat runs the kernels that read Phi* only)."""
    nx, ny, n = 128, 64, 4
    probs = [problem(2, nx, ny, instance=m, dt=400.0) for m in range(n)]
    oros = [1500.0 * np.random.default_rng(90 + m).random((ny, nx)) for m in range(n)]
    s = make_solver(gpu_lib, [(nx, ny)] * n, precision=precision)
    tol = 1e-9 if precision == 0 else 1e-5
    for kinds in ((0, 1, 0, 1), (0, 0, 0, 1), (0, 0, 0, 0), (1, 1, 1, 1)):
        ops = []
        for m, p in enumerate(probs):
            oro = oros[m] if kinds[m] else None
            s.set_operator(m, p["depth"], p["dt"], orography=oro)
            ops.append(EllipticOperator(nx, ny, p["depth"], p["dt"], orography=oro))
        rhs = [dev(op.apply(p["x_true"])) for op, p in zip(ops, probs)]
        x = [torch.zeros((ny, nx), dtype=torch.float64, device="cuda") for _ in range(n)]
        reps = s.solve(rhs, x)
        for m in range(n):
            assert reps[m].status == gpu_lib.OK, (kinds, m, reps[m])
            ores = gcr(ops[m], host(rhs[m]), rtol=1e-8)
            err = np.linalg.norm(host(x[m]) - ores.x) / np.linalg.norm(ores.x)
            assert err <= tol, (kinds, m, err)
            xt = probs[m]["x_true"]
            y = host(s.apply_operator(m, dev(xt)))
            assert np.all(np.abs(y - ops[m].apply(xt)) <= 32 * EPS * stencil_magnitude(ops[m], xt)), (kinds, m)


def test_solve_is_deterministic(gpu_lib):
    pr = problem(2, 256, 128)
    op = EllipticOperator(256, 128, pr["depth"], 600.0)
    rhs = dev(op.apply(pr["x_true"]))
    s = make_solver(gpu_lib, [(256, 128)], precision=2)
    s.set_operator(0, pr["depth"], 600.0)
    outs = []
    for _ in range(2):
        x = torch.zeros((128, 256), dtype=torch.float64, device="cuda")
        s.solve([rhs], [x])
        outs.append(x)
    assert torch.equal(outs[0], outs[1])


def test_batched_assembly_matches_single(gpu_lib):
    probs = batch_problems(3, 4, grids=((64, 32), (128, 64)))
    sizes = [(p["nx"], p["ny"]) for p in probs]
    a = make_solver(gpu_lib, sizes)
    b = make_solver(gpu_lib, sizes)
    depths = [dev(p["depth"]) for p in probs]
    a.set_operators([3, 1, 0, 2], [depths[3], depths[1], depths[0], depths[2]], [probs[m]["dt"] for m in (3, 1, 0, 2)])
    for m, p in enumerate(probs):
        b.set_operator(m, p["depth"], p["dt"])
    for m, p in enumerate(probs):
        x = dev(np.random.default_rng(m).standard_normal((p["ny"], p["nx"])))
        assert torch.equal(a.apply_operator(m, x), b.apply_operator(m, x))


def test_binding_names_bad_fields_and_members(gpu_lib):
    """The binding's one-pass field checks reject a wrong dtype, shape or
    member index and name the entry; valid calls (orography given for some
    members only) still assemble and solve."""
    probs = batch_problems(3, 3, grids=((64, 32),))
    sizes = [(p["nx"], p["ny"]) for p in probs]
    s = make_solver(gpu_lib, sizes)
    depths = [dev(p["depth"]) for p in probs]
    dts = [p["dt"] for p in probs]
    with pytest.raises(ValueError, match=r"depth\[2\]"):
        s.set_operators([0, 1, 2], depths[:2] + [depths[2].float()], dts)
    with pytest.raises(ValueError, match="members must lie"):
        s.set_operators([0, 1, 3], depths, dts)
    with pytest.raises(ValueError, match=r"orography\[1\]"):
        s.set_operators([0, 1, 2], depths, dts, orographies=[None, depths[1].t(), None])
    s.set_operators([0, 1, 2], depths, dts, orographies=[None, torch.zeros_like(depths[1]), None])
    rhs = [s.apply_operator(m, dev(p["x_true"])) for m, p in enumerate(probs)]
    x = [torch.zeros_like(r) for r in rhs]
    with pytest.raises(ValueError, match=r"x\[1\]"):
        s.solve(rhs, [x[0], x[1].t(), x[2]])
    with pytest.raises(ValueError, match=r"rhs\[0\]"):
        s.solve([rhs[0][:, :-1]] + rhs[1:], x)
    reps = s.solve(rhs, x)
    assert [r.status for r in reps] == [0, 0, 0] and all(r.iterations > 0 for r in reps)


# ---------------------------------------------------------------------------
# full sizes, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------
def _sampled_members_check(gpu_lib, probs, precision, sample, err_tol):
    """Batch solve of `probs` (one launch sequence, batched assembly from
    device depth fields, zero initial guesses in one buffer); every member
    must reach the tolerance by its float64 true residual, and the sampled
    members must match the oracle's solution."""
    sizes = [(p["nx"], p["ny"]) for p in probs]
    s = make_solver(gpu_lib, sizes, precision=precision, max_iters=100)
    f = make_solver(gpu_lib, sizes)
    depth = [dev(p["depth"]) for p in probs]
    for m, p in enumerate(probs):
        f.set_operator(m, depth[m], p["dt"])
    rhs = [f.apply_operator(m, dev(p["x_true"])) for m, p in enumerate(probs)]
    s.set_operators(list(range(len(probs))), depth, [p["dt"] for p in probs])
    x = [torch.zeros_like(r) for r in rhs]
    reps = s.solve(rhs, x)
    for m, rp in enumerate(reps):
        assert rp.status == gpu_lib.OK, (m, rp)
        assert rp.rel_res_true <= 1.05e-8, (m, rp)
    for m in sample:
        p = probs[m]
        op = EllipticOperator(p["nx"], p["ny"], p["depth"], p["dt"])
        ores = gcr(op, host(rhs[m]), rtol=1e-8)
        err = np.linalg.norm(host(x[m]) - ores.x) / np.linalg.norm(ores.x)
        assert err <= err_tol, (m, err)
    return reps


@pytest.mark.parametrize("precision,tol", [(3, 1e-5), (0, 1e-9)])
def test_benchmark_batch_sampled_against_oracle(gpu_lib, precision, tol):
    """64 members of 512x256 as in the benchmark; members 0, 21, 42, 63 are
    compared with the oracle point by point."""
    probs = [problem(2, 512, 256, instance=m, dt=600.0) for m in range(64)]
    _sampled_members_check(gpu_lib, probs, precision, (0, 21, 42, 63), tol)


def test_uneven_batch_sampled_against_oracle(gpu_lib):
    """64 members with grids drawn from {128x64, 256x128, 512x256}, their
    own depth range and time step, mixed precision; one member of each grid
    size is compared with the oracle."""
    probs = batch_problems(3, 64)
    sample = []
    for size in ((128, 64), (256, 128), (512, 256)):
        sample.append(next(m for m, p in enumerate(probs) if (p["nx"], p["ny"]) == size))
    _sampled_members_check(gpu_lib, probs, 3, sample, 1e-5)


@pytest.mark.parametrize("precision", [4, 5])
def test_uneven_batch_single_forms(gpu_lib, precision):
    """The single-precision solver cycles (4: float32 throughout; 5: float64
    polar bands) on the uneven 64-member batch, every points-per-lane class
    of its three grid sizes in one launch sequence.  Without residual
    replacement the true residual stops on a float32 plateau (about 2e-5 at
    most on this batch), so every member must converge by its own residual
    with a true residual of at most 1e-4, and one member of each grid size
    must match the oracle's solution to 1e-6."""
    probs = batch_problems(3, 64)
    sizes = [(p["nx"], p["ny"]) for p in probs]
    s = make_solver(gpu_lib, sizes, precision=precision, max_iters=100)
    f = make_solver(gpu_lib, sizes)
    depth = [dev(p["depth"]) for p in probs]
    for m, p in enumerate(probs):
        f.set_operator(m, depth[m], p["dt"])
    rhs = [f.apply_operator(m, dev(p["x_true"])) for m, p in enumerate(probs)]
    s.set_operators(list(range(len(probs))), depth, [p["dt"] for p in probs])
    x = [torch.zeros_like(r) for r in rhs]
    reps = s.solve(rhs, x)
    for m, rp in enumerate(reps):
        assert rp.status == gpu_lib.OK and rp.rel_res_true <= 1e-4, (m, rp)
    for size in ((128, 64), (256, 128), (512, 256)):
        m = next(i for i, p in enumerate(probs) if (p["nx"], p["ny"]) == size)
        p = probs[m]
        op = EllipticOperator(p["nx"], p["ny"], p["depth"], p["dt"])
        ores = gcr(op, host(rhs[m]), rtol=1e-8)
        xm = host(x[m])
        true_res = np.linalg.norm(op.apply(xm) - host(rhs[m])) / ores.r0_norm
        err = np.linalg.norm(xm - ores.x) / np.linalg.norm(ores.x)
        print(f"\nprecision={precision} member {m} {size}: true={true_res:.3e} err_vs_oracle={err:.3e}")
        assert reps[m].rel_res_true == pytest.approx(true_res, rel=1e-6, abs=1e-14)
        assert err <= 1e-6, (m, err)


@pytest.mark.parametrize("precision", [0, 3])
@pytest.mark.parametrize("fault", ["nan", "zero"])
def test_fault_injection_reports_stagnation(gpu_lib, precision, fault):
    """A non-finite preconditioner output, or a zero search direction (<L p,
    L p> = 0), in the first iteration of the second GCR(3) cycle stops every
    member with STAGNATED (paper Section 2.3: breakdown ends the iteration).
    x is the last finite iterate -- bitwise that of the same solve stopped
    by max_iters after k+1 iterations -- and its float64 true residual is
    reported."""
    nx, ny, B, k = 128, 64, 3, 3
    prs = [problem(2, nx, ny, instance=m, dt=600.0) for m in range(B)]
    ops = [EllipticOperator(nx, ny, p["depth"], 600.0) for p in prs]
    rhs = [dev(o.apply(p["x_true"])) for o, p in zip(ops, prs)]
    flag = gpu_lib.F_FAULT_NAN_PC if fault == "nan" else gpu_lib.F_FAULT_ZERO_DIR

    def run(flags, max_iters):
        s = make_solver(gpu_lib, [(nx, ny)] * B, precision=precision, rtol=1e-15, max_iters=max_iters, flags=flags)
        for m, p in enumerate(prs):
            s.set_operator(m, p["depth"], 600.0)
        x = [torch.zeros_like(r) for r in rhs]
        reps = s.solve(rhs, x)
        s.close()
        return reps, [host(v) for v in x]

    rf, xf = run(flag, 50)
    rs, xs = run(0, k + 1)
    for m in range(B):
        assert rf[m].status == gpu_lib.STAGNATED and rf[m].iterations == k + 1, rf[m]
        assert rs[m].status == gpu_lib.NOT_CONVERGED and rs[m].iterations == k + 1, rs[m]
        assert np.all(np.isfinite(xf[m]))
        assert np.array_equal(xf[m], xs[m])
        true = np.linalg.norm(ops[m].apply(xf[m]) - host(rhs[m])) / rf[m].r0_norm
        assert rf[m].rel_res_true == pytest.approx(true, rel=1e-6)
        assert rf[m].rel_res_true < 1e-3


@pytest.mark.parametrize("nx,ny", [(128, 64), (256, 128), (512, 256)])
def test_mixed_plateau_against_emulated_half(gpu_lib, nx, ny, capsys):
    """GCR_MIXED (float16 storage of the operator and preconditioner
    coefficients, float32 arithmetic, no residual replacement) stalls at a
    true residual of the same order as the paper's half-precision solver,
    which the oracle emulates with 10-bit significands and float64's exponent
    range at the paper's rounding points (Sections 3.3, 4.3): both plateau
    far above the tolerance their recursive residuals reach."""
    from oracle.emulated import gcr_half
    pr = problem(2, nx, ny, dt=600.0)
    op = EllipticOperator(nx, ny, pr["depth"], 600.0)
    rhs = op.apply(pr["x_true"])
    polar = max(1, int(np.ceil(np.log2(max(ny // 32, 1)))))
    emu = gcr_half(op, rhs, rtol=1e-8, polar=polar)
    s = make_solver(gpu_lib, [(nx, ny)], precision=gpu_lib.MIXED, rtol=1e-8, max_iters=60)
    s.set_operator(0, pr["depth"], 600.0)
    x = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    rep = s.solve([dev(rhs)], [x])[0]
    true_res = np.linalg.norm(op.apply(host(x)) - rhs) / np.linalg.norm(rhs)
    with capsys.disabled():
        print(f"\n[plateau {nx}x{ny}] GCR_MIXED true residual {true_res:.2e} ({rep.iterations} it.), "
              f"emulated half-precision solver {emu.rel_res_true:.2e} ({emu.iterations} it.)")
    assert rep.rel_res_recursive <= 1e-8 and emu.rel_res_recursive <= 1e-8
    assert true_res > 1e-7 and emu.rel_res_true > 1e-7
    assert 0.05 <= true_res / emu.rel_res_true <= 20


def _graph_case(kind):
    if kind == "uneven":
        prs = batch_problems(3, 12)
    elif kind == "groups":      # large enough for two member groups on two streams
        prs = [problem(2, 512, 256, instance=m, dt=600.0) for m in range(32)]
    else:
        prs = [problem(2, 128, 64, instance=m, dt=600.0) for m in range(4)]
    return prs


@pytest.mark.parametrize("kind", ["uniform", "uneven", "groups"])
@pytest.mark.parametrize("precision", [0, 1, 3])
def test_graph_replay_equals_stream_launches(gpu_lib, kind, precision):
    """GCR_F_GRAPH: the iterations and cycle ends are captured into HIP graphs
    on first use and replayed after.  Three consecutive solves -- a new
    right-hand side each time, eager work and synchronisations in between,
    and in the last one a member switched to orography (which drops the
    captured graphs of its group) -- each bitwise equal to the same solve
    launched kernel by kernel."""
    prs = _graph_case(kind)
    sizes = [(p["nx"], p["ny"]) for p in prs]
    solvers = {g: make_solver(gpu_lib, sizes, precision=precision, rtol=1e-8, max_iters=60, graph=g)
               for g in (False, True)}
    for s in solvers.values():
        for m, p in enumerate(prs):
            s.set_operator(m, p["depth"], p["dt"])
    ops = [EllipticOperator(p["nx"], p["ny"], p["depth"], p["dt"]) for p in prs]
    for rnd in range(3):
        if rnd == 2:
            oro = 300.0 * np.abs(prs[0]["x_true"])
            for s in solvers.values():
                s.set_operator(0, prs[0]["depth"], prs[0]["dt"], orography=oro)
            ops[0] = EllipticOperator(prs[0]["nx"], prs[0]["ny"], prs[0]["depth"], prs[0]["dt"], orography=oro)
        rhs = [dev(o.apply((1.0 + rnd) * p["x_true"])) for o, p in zip(ops, prs)]
        out = {}
        for g, s in solvers.items():
            x = [torch.zeros_like(r) for r in rhs]
            reps = s.solve(rhs, x)
            out[g] = (reps, [host(v) for v in x])
            torch.cuda.synchronize()
            _ = torch.randn(1 << 20, device="cuda").sum().item()     # eager work between solves
        for m in range(len(prs)):
            ra, rb = out[False][0][m], out[True][0][m]
            assert (ra.status, ra.iterations, ra.restarts) == (rb.status, rb.iterations, rb.restarts), (rnd, m)
            assert ra.rel_res_true == rb.rel_res_true
            assert np.array_equal(out[False][1][m], out[True][1][m]), (rnd, m)
            assert ra.status == gpu_lib.OK or precision == 1
    for s in solvers.values():
        s.close()
