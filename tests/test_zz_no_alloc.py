"""The preconditioner entry point that allocates nothing
(gcr_apply_precond_static, for callers that cannot allocate device memory)
against gcr_apply_precond of a float64 solver with the same operator: two
calls in a row, the largest size the static work array takes and then a
smaller one (with orography and another Richardson count), each bitwise the
solver's result (the same kernels on the same inputs)."""
import numpy as np
import pytest
import torch

from workloads import problem

pytestmark = pytest.mark.gpu


def _inputs(nx, ny, dt, orography, seed):
    pr = problem(2, nx, ny, instance=seed, dt=dt)
    rng = np.random.default_rng(500 + seed)
    depth = torch.from_numpy(pr["depth"]).cuda()
    oro = torch.from_numpy(1500.0 * rng.random((ny, nx))).cuda() if orography else None
    r = torch.from_numpy(rng.standard_normal((ny, nx))).cuda()
    return depth, oro, r


def _solver_result(lib, nx, ny, dt, iters, depth, oro, r):
    s = lib.Solver([(nx, ny)], precision=lib.FP64, richardson_iters=iters)
    s.set_operator(0, depth, dt, orography=oro)
    e = s.apply_precond(0, r)
    torch.cuda.synchronize()
    s.close()
    return e


def test_static_preconditioner_equals_the_solver_twice(gpu_lib):
    lib = gpu_lib
    cases = [(512, 256, 600.0, 2, False, 1), (128, 64, 400.0, 3, True, 2)]
    assert cases[0][0] * cases[0][1] == lib.STATIC_MAX_POINTS
    outs = []
    for nx, ny, dt, iters, orography, seed in cases:
        depth, oro, r = _inputs(nx, ny, dt, orography, seed)
        e = lib.apply_precond_static(r, depth, dt, orography=oro, richardson_iters=iters)
        outs.append((e, depth, oro, r, nx, ny, dt, iters))
    torch.cuda.synchronize()
    for e, depth, oro, r, nx, ny, dt, iters in outs:
        ref = _solver_result(lib, nx, ny, dt, iters, depth, oro, r)
        assert torch.all(torch.isfinite(e))
        assert torch.equal(e, ref), float((e - ref).abs().max() / ref.abs().max())


def test_static_preconditioner_rejects_sizes_beyond_its_array(gpu_lib):
    lib = gpu_lib
    depth, _, r = _inputs(1024, 256, 600.0, False, 3)
    with pytest.raises(lib.GcrError) as ei:
        lib.apply_precond_static(r, depth, 600.0)
    assert ei.value.code == lib.EINVAL and "exceeds" in str(ei.value)
