"""Element-wise parity of the precision forms' operator and preconditioner.

gcr_apply_operator_form and gcr_apply_precond_form run the kernels a solve
of the solver's precision form runs (paper Sections 4.2-4.3 say which
quantity is held in which precision).  They are compared point by point with
the rounding model of tests/form_emul.py: the float64 oracle's steps with
exactly the stored quantities rounded as the form stores them.  What is left
between the two is float32 arithmetic, so the bounds are float32 ones:

* operator: 32 u32 times the pointwise sum of |summands| of the stencil (the
  bound of the float64 operator test with float32's unit roundoff), plus the
  float32 formation of the B coefficients from the float32 depth;
* preconditioner: form_emul.richardson_bound with float32's unit roundoff
  (per iteration: the row systems' condition bound, the P^M evaluation, and
  the propagation of earlier errors); where the intermediate is stored as
  float16 a float32 rounding may take a float16 rounding decision the other
  way, so up to 1% of the points may differ by float16 ulps (within the same
  bound with float16's unit roundoff).

Each test also checks on the CPU that its bound bites (a 1% error of the
result would exceed it at most points) and pins the model to the float64
oracle within the float16 / float32 rounding of what it stores.
"""
import numpy as np
import pytest
import torch

from oracle.operator import EllipticOperator
from oracle.precond import Preconditioner
from workloads import problem

import form_emul as fe
from form_emul import U16, U32, stencil_magnitude

pytestmark = pytest.mark.gpu

FORMS = [fe.MIXED, fe.MIXED_FP64DOT, fe.MIXED_HALF_PC, fe.SINGLE, fe.SINGLE_POLAR64]
CASES = [
    # nx, ny, dt, extras
    (64, 32, 600.0, {}),
    (128, 64, 400.0, dict(absorber=1.0 / (2 * 400.0), orography=True)),
    (256, 128, 600.0, dict(b_terms=False)),
    (512, 256, 600.0, {}),
    (16, 7, 900.0, dict(absorber=1e-3)),
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def build(lib, nx, ny, dt, extras, form, **kw):
    pr = problem(2, nx, ny, instance=3, dt=dt)
    oro = None
    if extras.get("orography"):
        oro = 1500.0 * np.random.default_rng(78).random((ny, nx))
    okw = dict(absorber=extras.get("absorber", 0.0), b_terms=extras.get("b_terms", True))
    op = EllipticOperator(nx, ny, pr["depth"], dt, orography=oro, **okw)
    s = lib.Solver([(nx, ny)], precision=form, **kw)
    s.set_operator(0, pr["depth"], dt, orography=oro, **okw)
    return pr, oro, okw, op, s


def model_magnitude(model, x):
    m = stencil_magnitude(model.inner, x)
    if model.outer is not None:
        m = np.maximum(m, stencil_magnitude(model.outer, x))
    return m


@pytest.mark.parametrize("nx,ny,dt,extras", CASES)
@pytest.mark.parametrize("form", FORMS)
def test_operator_form_parity(gpu_lib, nx, ny, dt, extras, form):
    pr, oro, okw, op, s = build(gpu_lib, nx, ny, dt, extras, form)
    x = np.random.default_rng(11).standard_normal((ny, nx))
    y = host(s.apply_operator_form(0, dev(x)))
    model = fe.operator_model(form, op, pr["depth"], oro, **okw)
    ref = fe.emulate_operator(form, model, x)
    xv = fe.f32(x)
    mag = model_magnitude(model, xv)
    on_the_fly = form in (fe.MIXED_HALF_PC, fe.SINGLE, fe.SINGLE_POLAR64)
    if on_the_fly and okw["b_terms"]:
        mag = mag + fe.b_term_magnitude(op, pr["depth"], oro) * fe.neighbourhood_max(xv)
    bound = 32 * U32 * mag
    err = np.abs(y - ref)
    assert np.all(err <= bound), (form, float(np.max(err / bound)))
    # the bound bites: a 1% error would exceed it at most points, zero everywhere
    assert np.mean(0.01 * np.abs(ref) > bound) > 0.5
    assert np.all(np.abs(ref) > bound) or np.mean(np.abs(ref) > bound) > 0.99
    # the model against the float64 oracle: only what the form stores is rounded
    u = U16 if form in (fe.MIXED, fe.MIXED_FP64DOT) else U32
    exact = op.apply(x)
    mag64 = stencil_magnitude(op, np.abs(x))
    if on_the_fly and okw["b_terms"]:
        mag64 = mag64 + fe.b_term_magnitude(op, pr["depth"], oro) * fe.neighbourhood_max(x)
    # float16 coefficients of magnitude below float16's normal range are stored
    # with an absolute error of up to 2^-25 (scaled units)
    assert np.all(np.abs(ref - exact) <= 8 * u * mag64 + 8 * U32 * mag64 + 2.0 ** -25 / fe.scale_of(op)
                  * 24 / min(op.grid.dlam, op.grid.dphi) ** 2 * fe.neighbourhood_max(x))


@pytest.mark.parametrize("nx,ny,dt,extras", CASES)
@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("iters", [2, 3])
def test_precond_form_parity(gpu_lib, nx, ny, dt, extras, form, iters):
    pr, oro, okw, op, s = build(gpu_lib, nx, ny, dt, extras, form, richardson_iters=iters)
    r = np.random.default_rng(12).standard_normal((ny, nx))
    e = host(s.apply_precond_form(0, dev(r)))
    model, kind = fe.precond_model(form, op, pr["depth"], oro, **okw)
    sc = fe.scale_of(op)
    ref = fe.emulate_precond(form, model, kind, r, sc, iters)
    local = np.max([fe.rows_max3(fe.emulate_precond(form, model, kind, r, sc, mu))
                    for mu in range(1, iters + 1)], axis=0)
    tight = fe.richardson_bound(op, iters, local, U32)
    err = np.abs(e - ref)
    if kind == "half":
        over = err > tight
        assert np.mean(over) <= 0.01, (form, float(np.mean(over)), float(np.max(err / tight)))
        flips = fe.richardson_bound(op, iters, local, U16)
        assert np.all(err <= flips), (form, float(np.max(err / flips)))
    else:
        assert np.all(err <= tight), (form, float(np.max(err / tight)))
    # the bound bites: a 1% error would exceed it at most points
    assert np.mean(0.01 * np.abs(ref) > tight) > 0.5
    # the model against the float64 oracle: within the rounding of what it stores
    u = U16 if kind == "half" else U32
    exact = Preconditioner(op, 3, iters)(r)
    assert np.all(np.abs(ref - exact) <= fe.richardson_bound(op, iters, local, u))


@pytest.mark.parametrize("nx,ny,dt,extras", CASES[:4])
def test_fp64_form_is_the_float64_entry_point(gpu_lib, nx, ny, dt, extras):
    pr, oro, okw, op, s = build(gpu_lib, nx, ny, dt, extras, gpu_lib.FP64)
    x = dev(np.random.default_rng(13).standard_normal((ny, nx)))
    assert torch.equal(s.apply_operator_form(0, x), s.apply_operator(0, x))
    assert torch.equal(s.apply_precond_form(0, x), s.apply_precond(0, x))
