"""The semi-implicit step around the solve (gcr_si_step: paper Sections
2.1-2.2, eqs. SWE1-SWE3, RSWE2-RSWE3, MPDATA, rhslin, Qexpr, Elliptic, vadv)
through the C-ABI, against the oracle's step (oracle/si_step.py) with a
direct float64 solve.

The GPU step computes the explicit part in float64 in its own order and
solves to rtol 1e-12 (float64 form), so its new state differs from the
oracle's by rounding amplified through MPDATA's ratios and the solve: a few
hundred ulps of the fields.  Bounds: 1e-11 of max|Phi| for Phi, 1e-10 of
max|Q_x| for the momenta.  The same bounds are far below what a planted
mistake in the oracle (a dropped metric term) changes.  A reduced-precision
form is checked against the bound its rtol allows."""
import numpy as np
import pytest
import torch

from oracle import si_step as si
from oracle.gcr import gcr
from test_oracle_si_step import _rand_state, _orography, TOL_PHI, TOL_Q

pytestmark = pytest.mark.gpu



def direct(op, rhs, x0):
    return np.linalg.solve(op.dense(), rhs.ravel()).reshape(rhs.shape)


def iterative(op, rhs, x0):
    return gcr(op, rhs, x0, rtol=1e-13, max_iters=500).x


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def _member(nx, ny, seed, oro=True, qbar=True):
    s = _rand_state(nx, ny, seed)
    so = _rand_state(nx, ny, seed + 1)
    h0 = _orography(nx, ny, seed) if oro else np.zeros((ny, nx))
    rng = np.random.default_rng(seed + 2)
    qb = (rng.normal(size=(ny, nx)) * 1e4, rng.normal(size=(ny, nx)) * 1e4) if qbar else \
        (np.zeros((ny, nx)), np.zeros((ny, nx)))
    return s, so, h0, qb, oro, qbar


def _gpu_step(lib, sizes, members, dts, absorber, precision=None, rtol=1e-12):
    kw = dict(rtol=rtol, max_iters=500)
    if precision is not None:
        kw["precision"] = precision
    solver = lib.Solver(sizes, **kw)
    states = [tuple(dev(f) for f in (m[0].phi, m[0].qx, m[0].qy)) for m in members]
    olds = [tuple(dev(f) for f in (m[1].phi, m[1].qx, m[1].qy)) for m in members]
    news = [tuple(torch.empty_like(f) for f in st) for st in states]
    oros = [dev(m[2]) if m[4] else None for m in members]
    qbars = [(dev(m[3][0]), dev(m[3][1])) if m[5] else None for m in members]
    reps = solver.si_step(states, olds, news, dts, orographies=oros, qbars=qbars, absorber=absorber)
    return [tuple(host(f) for f in nw) for nw in news], reps, solver


def _check(got, ref, tol_phi=TOL_PHI, tol_q=TOL_Q):
    phi, qx, qy = got
    sphi = np.abs(ref.phi).max()
    sq = np.abs(ref.qx).max()
    assert np.abs(phi - ref.phi).max() <= tol_phi * sphi, np.abs(phi - ref.phi).max() / sphi
    assert np.abs(qx - ref.qx).max() <= tol_q * sq, np.abs(qx - ref.qx).max() / sq
    assert np.abs(qy - ref.qy).max() <= tol_q * sq, np.abs(qy - ref.qy).max() / sq


@pytest.mark.parametrize("nx,ny,oro,qbar", [(64, 32, True, True), (32, 20, False, False), (16, 6, True, False)])
def test_si_step_matches_oracle(gpu_lib, nx, ny, oro, qbar):
    m = _member(nx, ny, 30 + nx, oro, qbar)
    p = si.Params(dt=900.0, absorber=1e-4)
    (got,), reps, _ = _gpu_step(gpu_lib, [(nx, ny)], [m], [p.dt], p.absorber)
    assert reps[0].status == 0
    ref, _ = si.si_step(nx, ny, m[0], m[1], m[2], m[3], p, direct)
    _check(got, ref)
    assert np.abs(ref.phi - m[0].phi).max() > 1e-4 * np.abs(ref.phi).max()   # the step did something


def test_si_step_batch_of_sizes(gpu_lib):
    sizes = [(64, 32), (32, 20), (128, 64), (8, 4)]
    members = [_member(nx, ny, 50 + 7 * i, oro=i % 2 == 0, qbar=i < 2) for i, (nx, ny) in enumerate(sizes)]
    dts = [900.0, 600.0, 450.0, 1200.0]
    absorber = 2e-4
    got, reps, _ = _gpu_step(gpu_lib, sizes, members, dts, absorber)
    for i, ((nx, ny), m) in enumerate(zip(sizes, members)):
        assert reps[i].status == 0
        solve = direct if nx * ny <= 2048 else iterative
        ref, _ = si.si_step(nx, ny, m[0], m[1], m[2], m[3], si.Params(dt=dts[i], absorber=absorber), solve)
        _check(got[i], ref)


def test_si_step_three_steps(gpu_lib):
    # the step fed its own output: (n-1, n) -> (n, n+1)
    nx, ny = 64, 32
    s, so, h0, qb, _, _ = _member(nx, ny, 70)
    p = si.Params(dt=900.0, absorber=1e-4)
    solver = gpu_lib.Solver([(nx, ny)], rtol=1e-12, max_iters=500)
    g_old = tuple(dev(f) for f in (so.phi, so.qx, so.qy))
    g_cur = tuple(dev(f) for f in (s.phi, s.qx, s.qy))
    h0d, qbd = dev(h0), (dev(qb[0]), dev(qb[1]))
    r_old, r_cur = so, s
    for _ in range(3):
        g_new = tuple(torch.empty_like(f) for f in g_cur)
        solver.si_step([g_cur], [g_old], [g_new], [p.dt], orographies=[h0d], qbars=[qbd], absorber=p.absorber)
        r_new, _ = si.si_step(nx, ny, r_cur, r_old, h0, qb, p, direct)
        g_old, g_cur = g_cur, g_new
        r_old, r_cur = r_cur, r_new
    _check(tuple(host(f) for f in g_cur), r_cur, 1e-10, 1e-9)


def test_si_step_mass_conserved_on_gpu(gpu_lib):
    nx, ny = 128, 64
    m = _member(nx, ny, 80)
    (got,), reps, _ = _gpu_step(gpu_lib, [(nx, ny)], [m], [900.0], 1e-4)
    lat = -0.5 * np.pi + (np.arange(ny) + 0.5) * np.pi / ny
    G = np.cos(lat)[:, None]
    m0, m1 = (G * m[0].phi).sum(), (G * got[0]).sum()
    # the solve's residual (rtol 1e-12 of ||r_0||) bounds the drift
    assert abs(m1 - m0) <= 1e-11 * m0


def test_si_step_reduced_precision_form(gpu_lib):
    # the headline form (half-precision preconditioner, float64 residual
    # replacement) at rtol 1e-8: Phi within what that residual allows
    nx, ny = 64, 32
    m = _member(nx, ny, 90)
    p = si.Params(dt=900.0, absorber=1e-4)
    (got,), reps, _ = _gpu_step(gpu_lib, [(nx, ny)], [m], [p.dt], p.absorber,
                                precision=gpu_lib.MIXED_HALF_PC, rtol=1e-8)
    assert reps[0].status == 0 and reps[0].rel_res_true <= 1e-8 * 1.5
    ref, _ = si.si_step(nx, ny, m[0], m[1], m[2], m[3], p, direct)
    dphi = np.abs(ref.phi - m[0].phi).max()
    assert np.abs(got[0] - ref.phi).max() <= 1e-6 * dphi


def test_si_step_rejects_aliasing(gpu_lib):
    nx, ny = 16, 8
    m = _member(nx, ny, 95)
    solver = gpu_lib.Solver([(nx, ny)])
    st = tuple(dev(f) for f in (m[0].phi, m[0].qx, m[0].qy))
    with pytest.raises(gpu_lib.GcrError):
        solver.si_step([st], [st], [st], [900.0])
    new = tuple(torch.empty_like(f) for f in st)
    with pytest.raises(gpu_lib.GcrError):
        solver.si_step([st], [st], [new], [-1.0])


def test_si_step_full_size_batch_sampled(gpu_lib):
    # the model-step workload at full size (64 members of 512x256 over
    # synthetic mountains, dt 200 s, absorbers 1/(200 dt)), in one batch as
    # the bench runs it; members 0 and 63 against the oracle's step
    from workloads import model_state
    nx, ny, count, dt = 512, 256, 64, 200.0
    absorber = 1.0 / (200.0 * dt)
    states = [model_state(nx, ny, m) for m in range(count)]
    cur = [tuple(dev(st[k]) for k in ("phi", "qx", "qy")) for st in states]
    oro = [dev(st["orography"]) for st in states]
    new = [tuple(torch.empty_like(f) for f in c) for c in cur]
    solver = gpu_lib.Solver([(nx, ny)] * count, rtol=1e-12, max_iters=500)
    reps = solver.si_step(cur, cur, new, [dt] * count, orographies=oro, absorber=absorber)
    assert all(r.status == 0 for r in reps)
    z = np.zeros((ny, nx))
    p = si.Params(dt=dt, absorber=absorber)
    for m in (0, count - 1):
        st = states[m]
        s0 = si.State(st["phi"], st["qx"], st["qy"])
        ref, _ = si.si_step(nx, ny, s0, s0, st["orography"], (z, z), p, iterative)
        _check(tuple(host(f) for f in new[m]), ref)


def test_si_step_binding_names_bad_fields(gpu_lib):
    """The one-pass field checks of si_step fall back to the per-field check,
    which names the failing entry; a valid call still steps."""
    nx, ny = 16, 8
    m = _member(nx, ny, 96)
    solver = gpu_lib.Solver([(nx, ny)] * 2, max_iters=500)
    st = [tuple(dev(f) for f in (m[0].phi, m[0].qx, m[0].qy)) for _ in range(2)]
    old = [tuple(dev(f) for f in (m[1].phi, m[1].qx, m[1].qy)) for _ in range(2)]
    new = [tuple(torch.empty_like(f) for f in s) for s in st]
    oro = [dev(m[2]), dev(m[2])]
    with pytest.raises(ValueError, match=r"new\[1\]"):
        solver.si_step(st, old, [new[0], (new[1][0], new[1][1].float(), new[1][2])], [900.0, 900.0])
    with pytest.raises(ValueError, match=r"old\[0\] must be \(phi, qx, qy\)"):
        solver.si_step(st, [old[0][:2], old[1]], new, [900.0, 900.0])
    with pytest.raises(ValueError, match=r"orography\[1\]"):
        solver.si_step(st, old, new, [900.0, 900.0], orographies=[None, st[0][0].t()])
    reps = solver.si_step(st, old, new, [900.0, 900.0], orographies=oro)
    assert [r.status for r in reps] == [0, 0]
    assert torch.equal(new[0][0], new[1][0])
