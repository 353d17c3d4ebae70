"""The learned preconditioner's network and its use inside GCR, on the GPU,
against the float64 network of oracle/cnn.py.

Forward and gradients, exactly: integer inputs and sparse integer weights
keep every intermediate value an integer below 256 and every sum below
2^24, so neither bf16 storage nor float32 accumulation rounds anything and
the kernels must reproduce the float64 oracle bit for bit (the test checks
on the CPU that its data has this property).

Forward and gradients, general values: the oracle evaluated with bfloat16
rounding at the points where the kernels round (tests/cnn_emul.py); what
remains is float32 versus float64 accumulation, ~1e-7 relative.  Where that
difference moves a hidden activation across a bf16 rounding boundary the two
round it to neighbouring bf16 values (probability ~1e-7 / 2^-8 per
rounding), which moves the outputs within its receptive field by ~1e-3 of
the output scale.  So: the median point agrees to 1e-5 of the scale, none
differs by more than 1e-2 of it, the relative L2 distance is below 3e-3 --
far below any indexing mistake (a wrong tap, pole shift or transposition
changes outputs by O(1)).

The learned correction inside the solver is checked against its definition,
e = e_2 + T^{-1}(s sigma N(features)), with e_2, T and the features from the
float64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import cnn
from oracle.operator import EllipticOperator
from oracle.precond import Preconditioner, row_matrix, row_systems
from workloads import problem

import cnn_emul as E

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def random_params(c_in, seed, last_scale=1.0, bias_scale=0.1):
    rng = np.random.default_rng(seed)
    params = cnn.init_params(c_in, rng)
    w, b = params[-1]
    params[-1] = (rng.standard_normal(w.shape) * np.sqrt(2.0 / (9 * cnn.WIDTH)) * last_scale, b)
    return [(w, rng.standard_normal(b.shape) * bias_scale) for w, b in params]


GRIDS = [(64, 16, 2), (128, 9, 1), (256, 6, 3)]
# several 16-row bands per column strip with a ragged last band, and 16 strips per row
BAND_GRIDS = [(128, 37, 2), (1024, 20, 1)]


def assert_bf16_close(got, ref, what=""):
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    assert err.max() <= 1e-2 * scale, (what, err.max(), scale)
    assert np.median(err) <= 1e-5 * scale, (what, np.median(err), scale)
    assert np.linalg.norm(got - ref) <= 3e-3 * np.linalg.norm(ref), (what, np.linalg.norm(got - ref),
                                                                       np.linalg.norm(ref))


def _exact(a):
    return np.array_equal(E.bf16(a), a) and np.abs(a).max() < 256


def exact_case(nx, ny, batch, seed, c_in=3):
    """Integer data on which the network computes without rounding: the
    first seed from `seed` on whose activations and back-propagated
    gradients are all bf16-exact."""
    shapes = [(cnn.WIDTH, c_in)] + [(cnn.WIDTH, cnn.WIDTH)] * 3 + [(1, cnn.WIDTH)]
    dens = [0.2, 0.03, 0.03, 0.03, 0.2]
    idx = cnn.neighbour_index(ny, nx)
    for sd in range(seed, seed + 50):
        rng = np.random.default_rng(sd)
        params = []
        for (co, ci), d in zip(shapes, dens):
            w = rng.integers(-1, 2, (co, ci, 3, 3)) * (rng.random((co, ci, 3, 3)) < d)
            params.append((w.astype(np.float64), rng.integers(-1, 2, co).astype(np.float64)))
        x = rng.integers(-1, 2, (batch, c_in, ny, nx)).astype(np.float64)
        dy = rng.integers(-1, 2, (batch, ny, nx)).astype(np.float64)
        ok = True
        ys, grads = [], [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
        for b in range(batch):
            acts = cnn.forward(params, x[b])
            ok = ok and all(_exact(a) for a in acts[1:])
            ys.append(acts[-1][0])
            d = dy[b][None]
            for n in range(len(params) - 1, -1, -1):
                dx, dw, db = cnn.conv3x3_backward(acts[n], params[n][0], d, idx)
                grads[n] = (grads[n][0] + dw, grads[n][1] + db)
                d = dx * (acts[n] > 0.0)
                ok = ok and (n == 0 or _exact(d))
        if ok:
            return params, x, dy, np.array(ys), grads
    raise AssertionError("no rounding-free test data found")


@pytest.mark.parametrize("nx,ny,batch", GRIDS + BAND_GRIDS)
def test_forward_exact(gpu_lib, nx, ny, batch):
    params, x, _, yref, _ = exact_case(nx, ny, batch, seed=nx + ny)
    net = gpu_lib.Network(nx, ny, batch, 3)
    net.set_params(E.flatten(params))
    y = host(net.forward(dev(x, torch.float32)))
    assert np.array_equal(y, yref), np.abs(y - yref).max()
    net.close()


@pytest.mark.parametrize("c_in", [8, 9, 32])
def test_input_channel_counts_exact(gpu_lib, c_in):
    """Inputs of up to 8 channels are stored 8 per pixel, more as 32: both
    layouts, forward and every gradient, bit-exact on rounding-free data."""
    nx, ny, batch = 64, 8, 2
    params, x, dy, yref, gref = exact_case(nx, ny, batch, seed=100 + c_in, c_in=c_in)
    net = gpu_lib.Network(nx, ny, batch, c_in)
    net.set_params(E.flatten(params))
    y = host(net.forward(dev(x, torch.float32)))
    assert np.array_equal(y, yref), np.abs(y - yref).max()
    g = E.unflatten(net.gradients(dev(x, torch.float32), dev(dy, torch.float32)), c_in)
    for n, ((gw, gb), (rw, rb)) in enumerate(zip(g, gref)):
        assert np.array_equal(gw, rw), (n, np.abs(gw - rw).max())
        assert np.array_equal(gb, rb), (n, gb, rb)
    net.close()


@pytest.mark.parametrize("nx,ny,batch", GRIDS)
def test_gradient_exact(gpu_lib, nx, ny, batch):
    params, x, dy, _, gref = exact_case(nx, ny, batch, seed=3 * nx + ny)
    net = gpu_lib.Network(nx, ny, batch, 3)
    net.set_params(E.flatten(params))
    g = E.unflatten(net.gradients(dev(x, torch.float32), dev(dy, torch.float32)), 3)
    for n, ((gw, gb), (rw, rb)) in enumerate(zip(g, gref)):
        assert np.array_equal(gw, rw), (n, np.abs(gw - rw).max(), np.argwhere(gw != rw)[:5])
        assert np.array_equal(gb, rb), (n, gb, rb)
    net.close()


@pytest.mark.parametrize("nx,ny,batch", GRIDS + BAND_GRIDS)
def test_forward_parity(gpu_lib, nx, ny, batch):
    c_in = 3
    params = random_params(c_in, 10 + nx)
    flat = E.flatten(params)
    pw = E.unflatten(flat, c_in)            # the float32 parameters the GPU sees
    rng = np.random.default_rng(nx + ny)
    x = rng.standard_normal((batch, c_in, ny, nx))
    net = gpu_lib.Network(nx, ny, batch, c_in)
    net.set_params(flat)
    y = host(net.forward(dev(x, torch.float32)))
    for b in range(batch):
        ref = E.forward(pw, x[b].astype(np.float32).astype(np.float64))[-1][0]
        assert_bf16_close(y[b], ref, b)
    net.close()


def test_forward_pole_rows_sensitive(gpu_lib):
    """A point next to a pole feeds the output half a circle away, across the
    pole; a network that pads with zeros instead would not see it."""
    nx, ny, c_in = 64, 8, 3
    params = random_params(c_in, 5)
    flat = E.flatten(params)
    net = gpu_lib.Network(nx, ny, 1, c_in)
    net.set_params(flat)
    x = np.zeros((1, c_in, ny, nx))
    y0 = host(net.forward(dev(x, torch.float32)))
    x[0, :, 0, 3] = 1.0
    y1 = host(net.forward(dev(x, torch.float32)))
    ref = E.forward(E.unflatten(flat, c_in), x[0])[-1][0] - E.forward(E.unflatten(flat, c_in), 0 * x[0])[-1][0]
    diff = y1[0] - y0[0]
    assert np.abs(diff[0, 3 + nx // 2]) > 0 or np.abs(ref[0, 3 + nx // 2]) == 0
    assert_bf16_close(diff, ref)
    net.close()


@pytest.mark.parametrize("nx,ny,batch", GRIDS + BAND_GRIDS[:1])
def test_gradient_parity(gpu_lib, nx, ny, batch):
    c_in = 3
    params = random_params(c_in, 20 + nx)
    flat = E.flatten(params)
    pw = E.unflatten(flat, c_in)
    rng = np.random.default_rng(7 * nx + ny)
    x = rng.standard_normal((batch, c_in, ny, nx)).astype(np.float32)
    dy = rng.standard_normal((batch, ny, nx)).astype(np.float32)
    net = gpu_lib.Network(nx, ny, batch, c_in)
    net.set_params(flat)
    g = net.gradients(dev(x, torch.float32), dev(dy, torch.float32))
    ref = [(np.zeros_like(w), np.zeros_like(b)) for w, b in pw]
    for b in range(batch):
        acts = E.forward(pw, x[b].astype(np.float64))
        gb = E.backward(pw, acts, dy[b].astype(np.float64))
        ref = [(rw + dw, rb + db) for (rw, rb), (dw, db) in zip(ref, gb)]
    got = E.unflatten(g, c_in)
    for n, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        # flips of back-propagated values add up over the pixel sums
        assert np.linalg.norm(gw - rw) <= 1e-2 * np.linalg.norm(rw), (n, "w")
        assert np.linalg.norm(gb - rb) <= 1e-2 * np.linalg.norm(rb), (n, "b")
    net.close()


def test_train_step_is_adam_on_mse(gpu_lib):
    nx, ny, batch, c_in = 64, 8, 2, 3
    params = random_params(c_in, 3)
    flat = E.flatten(params)
    rng = np.random.default_rng(4)
    x = dev(rng.standard_normal((batch, c_in, ny, nx)), torch.float32)
    t = dev(rng.standard_normal((batch, ny, nx)), torch.float32)
    net = gpu_lib.Network(nx, ny, batch, c_in)
    net.set_params(flat)
    y = net.forward(x)
    torch.cuda.synchronize()
    diff = (y - t).double()
    loss_ref = float((diff * diff).mean())
    dy = (2.0 * (y - t) / y.numel()).float().contiguous()
    g = net.gradients(x, dy)
    lr = 1e-3
    loss = net.train_step(x, t, lr)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    p1 = net.get_params().astype(np.float64)
    exp, _, _ = cnn.adam_step(flat.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr)
    assert np.abs(p1 - exp).max() <= 1e-6
    net.close()


def test_training_reduces_loss(gpu_lib):
    """Fit a fixed smooth target: the loss must fall by a large factor."""
    nx, ny, batch, c_in = 64, 16, 4, 3
    rng = np.random.default_rng(11)
    x = rng.standard_normal((batch, c_in, ny, nx))
    # a target the network can represent: a local linear filter of the input
    tgt = 0.5 * x[:, 0] - 0.25 * np.roll(x[:, 1], 1, axis=2) + 0.1 * x[:, 2]
    net = gpu_lib.Network(nx, ny, batch, c_in)
    net.set_params(E.flatten(cnn.init_params(c_in, np.random.default_rng(2))))
    xd, td = dev(x, torch.float32), dev(tgt, torch.float32)
    losses = [net.train_step(xd, td, 3e-3) for _ in range(300)]
    assert losses[-1] < 0.05 * losses[0], (losses[0], losses[-1])
    net.close()


# ---------------------------------------------------------------------------
# inside the solver
# ---------------------------------------------------------------------------
def _member(nx, ny, seed=0, dt=600.0):
    pr = problem(2, nx, ny, instance=seed, dt=dt)
    op = EllipticOperator(nx, ny, pr["depth"], dt)
    return pr, op


def _setup(lib, sizes, prs, precision, precond, **kw):
    s = lib.Solver(sizes, precision=precision, precond=precond, **kw)
    for m, pr in enumerate(prs):
        s.set_operator(m, dev(pr["depth"]), pr["dt"])
    return s


def test_features_match_oracle(gpu_lib):
    nx, ny = 128, 64
    pr, op = _member(nx, ny, seed=3)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((ny, nx)) * 10.0
    rhs = op.apply(pr["x_true"])
    s = _setup(gpu_lib, [(nx, ny)], [pr], gpu_lib.FP64, gpu_lib.PC_SEMI_IMPLICIT)
    feat, target, sigma = s.learned_features(0, dev(x), dev(rhs), hi_iters=8)
    feat, target = host(feat), host(target)
    r = op.apply(x) - rhs
    sig = np.sqrt(np.mean(r * r))
    assert abs(sigma - sig) <= 1e-12 * sig
    sc = pr["dt"] / (2.0 * 6.371e6 ** 2)
    e2 = Preconditioner(op, 3, 2)(r)
    e8 = Preconditioner(op, 3, 8)(r)
    ref = [r / sig, e2 / (sc * sig), np.broadcast_to(np.cos(op.grid.lat)[:, None], (ny, nx))]
    for c in range(3):
        scale = np.abs(ref[c]).max()
        assert np.abs(feat[c] - ref[c]).max() <= 1e-6 * scale, c
    lo, di, up = row_systems(op)
    d = e8 - e2
    tref = (lo * np.roll(d, 1, axis=1) + di * d + up * np.roll(d, -1, axis=1)) / (sc * sig)
    # T amplifies the float64 rounding of e8 and e2 by its row sums
    amp = (np.abs(lo) + np.abs(di) + np.abs(up)) * np.abs(e8) / (sc * sig)
    assert np.abs(target - tref).max() <= 1e-6 * np.abs(tref).max() + 1e-11 * amp.max()
    s.close()


def test_learned_precond_definition(gpu_lib):
    """Stand-alone P^{-1} with the network = e_2 + T^{-1}(s sigma N(features))."""
    nx, ny = 128, 32
    pr, op = _member(nx, ny, seed=1)
    params = E.flatten(random_params(3, 31))
    s = _setup(gpu_lib, [(nx, ny)], [pr], gpu_lib.FP64, gpu_lib.PC_LEARNED)
    s.set_learned(params)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((ny, nx))
    zero = np.zeros((ny, nx))
    feat, _, sigma = s.learned_features(0, dev(x), dev(zero))
    r = dev(op.apply(x))
    e = host(s.apply_precond(0, r))
    net = gpu_lib.Network(nx, ny, 1, 3)
    net.set_params(params)
    yn = host(net.forward(feat[None].contiguous()))[0]
    sc = pr["dt"] / (2.0 * 6.371e6 ** 2)
    e2 = Preconditioner(op, 3, 2)(op.apply(x))
    lo, di, up = row_systems(op)
    z = np.stack([np.linalg.solve(row_matrix(lo[j], di[j], up[j]), sc * sigma * yn[j]) for j in range(ny)])
    exp = e2 + z
    corr = np.abs(z).max()
    # e_2 from the GPU differs from the oracle's by its float64 rounding only
    assert np.abs(e - exp).max() <= 1e-9 * np.abs(e2).max() + 1e-9 * corr
    assert corr > 1e-3 * np.abs(e2).max()       # the correction is really applied
    net.close()
    s.close()


@pytest.mark.parametrize("precision", [0, 3])
def test_zero_network_is_plain(gpu_lib, precision):
    """N = 0 leaves P^{-1} unchanged: the solve is bitwise the plain one."""
    nx, ny, B = 128, 64, 3
    prs = [problem(2, nx, ny, instance=m, dt=600.0) for m in range(B)]
    rhs = [dev(EllipticOperator(nx, ny, p["depth"], 600.0).apply(p["x_true"])) for p in prs]
    plain = _setup(gpu_lib, [(nx, ny)] * B, prs, precision, gpu_lib.PC_SEMI_IMPLICIT)
    lrn = _setup(gpu_lib, [(nx, ny)] * B, prs, precision, gpu_lib.PC_LEARNED)
    lrn.set_learned(np.zeros(gpu_lib.cnn_param_count(3), dtype=np.float32))
    x0 = [torch.zeros_like(r) for r in rhs]
    x1 = [torch.zeros_like(r) for r in rhs]
    r0 = plain.solve(rhs, x0)
    r1 = lrn.solve(rhs, x1)
    for m in range(B):
        assert r0[m].iterations == r1[m].iterations
        assert r1[m].status == gpu_lib.OK and r1[m].fallback_used == 0
        assert torch.equal(x0[m], x1[m])
    plain.close()
    lrn.close()


def test_learned_solve_and_fallback(gpu_lib):
    """Random networks: GCR converges whatever directions it is given (it
    minimises over them), with or without dropping the network; a fallback
    ratio no cycle can meet drops it at the end of the first cycle, and the
    solve finishes with the plain preconditioner, reporting FALLBACK_USED."""
    nx, ny, B = 128, 64, 2
    prs = [problem(2, nx, ny, instance=m, dt=600.0) for m in range(B)]
    ops = [EllipticOperator(nx, ny, p["depth"], 600.0) for p in prs]
    rhs = [dev(o.apply(p["x_true"])) for o, p in zip(ops, prs)]
    bad = E.flatten(random_params(3, 77, last_scale=3.0))
    mild = E.flatten(random_params(3, 78, last_scale=0.01, bias_scale=0.0))
    # the default setting: the plain preconditioner's residual history on the
    # same problems as the reference a learned solve must keep up with
    from paper_2103_16120_amd.learned import reference_history
    plain = _setup(gpu_lib, [(nx, ny)] * B, prs, gpu_lib.FP64, gpu_lib.PC_SEMI_IMPLICIT, max_iters=200,
                   record_history=True)
    ref = reference_history(plain.solve(rhs, [torch.zeros_like(r) for r in rhs], record_history=True))
    plain.close()
    assert len(ref) >= 5
    for params, ratio, use_ref, expect_fb in ((bad, 1e-9, False, True), (bad, 0.5, True, True),
                                              (bad, 0.5, False, None), (mild, 0.9, False, None)):
        s = _setup(gpu_lib, [(nx, ny)] * B, prs, gpu_lib.FP64, gpu_lib.PC_LEARNED, max_iters=200)
        s.set_learned(params, fallback_ratio=ratio)
        if use_ref:
            s.set_learned_reference(ref)
        x = [torch.zeros_like(r) for r in rhs]
        reps = s.solve(rhs, x)
        for m in range(B):
            rp = reps[m]
            assert rp.rel_res_true <= 1.1e-8, (ratio, m, rp)
            if expect_fb:
                assert rp.fallback_used == 1 and rp.status == gpu_lib.FALLBACK_USED, rp
            else:
                assert rp.status in (gpu_lib.OK, gpu_lib.FALLBACK_USED), rp
                assert rp.fallback_used == (rp.status == gpu_lib.FALLBACK_USED)
            xo = host(x[m])
            assert np.abs(xo - prs[m]["x_true"]).max() <= 1e-5 * np.abs(prs[m]["x_true"]).max()
        s.close()


def test_learned_errors(gpu_lib):
    nx, ny = 64, 16
    pr, _ = _member(nx, ny)
    s = _setup(gpu_lib, [(nx, ny)], [pr], gpu_lib.FP64, gpu_lib.PC_LEARNED)
    x = dev(np.zeros((ny, nx)))
    with pytest.raises(gpu_lib.GcrError) as ei:
        s.solve([x], [torch.zeros_like(x)])
    assert ei.value.code == gpu_lib.ESTATE
    with pytest.raises(gpu_lib.GcrError):
        s.set_learned(np.zeros(10, dtype=np.float32))
    with pytest.raises(gpu_lib.GcrError):
        s.set_learned(np.zeros(gpu_lib.cnn_param_count(3), dtype=np.float32), fallback_ratio=0.0)
    s.close()
    with pytest.raises(gpu_lib.GcrError):
        gpu_lib.Solver([(64, 16), (128, 16)], precond=gpu_lib.PC_LEARNED)
    with pytest.raises(gpu_lib.GcrError):
        gpu_lib.Network(48, 16, 1)


def test_trained_network_gain(gpu_lib, capsys):
    """What the shipped, trained network gains over the plain preconditioner
    on held-out problems of the benchmark family (parity unpinned: the gain is
    measured and reported, not pinned).  Both must reach the tolerance by their
    float64 true residual and agree on the solution."""
    from paper_2103_16120_amd.learned import load_weights, DEFAULT_WEIGHTS
    params, head = load_weights(DEFAULT_WEIGHTS)
    nx, ny, B = 512, 256, 8
    prs = [problem(2, nx, ny, instance=m, dt=600.0) for m in range(B)]
    f = gpu_lib.Solver([(nx, ny)] * B, precision=gpu_lib.FP64)
    depth = [dev(p["depth"]) for p in prs]
    for m, p in enumerate(prs):
        f.set_operator(m, depth[m], p["dt"])
    rhs = [f.apply_operator(m, dev(p["x_true"])) for m, p in enumerate(prs)]
    from paper_2103_16120_amd.learned import reference_history
    out = {}
    ref = None
    for name, pc in (("plain", gpu_lib.PC_SEMI_IMPLICIT), ("learned", gpu_lib.PC_LEARNED)):
        s = gpu_lib.Solver([(nx, ny)] * B, precision=gpu_lib.MIXED_HALF_PC, precond=pc, record_history=True)
        if pc == gpu_lib.PC_LEARNED:
            s.set_learned(params)
            assert len(ref) >= 5
            s.set_learned_reference(ref)
        for m, p in enumerate(prs):
            s.set_operator(m, depth[m], p["dt"])
        x = [torch.zeros_like(r) for r in rhs]
        reps = s.solve(rhs, x, record_history=True)
        for rp in reps:
            assert rp.status in (gpu_lib.OK, gpu_lib.FALLBACK_USED) and rp.rel_res_true <= 1.05e-8, rp
        if ref is None:
            ref = reference_history(reps)
        out[name] = (reps, [host(v) for v in x])
        s.close()
    for a, b in zip(out["plain"][1], out["learned"][1]):
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)
    # no iteration count regresses: a member keeps the network only while it
    # is at least as far as the plain preconditioner's history, and the one
    # that drops it has lost at most the iteration that showed the regression
    for rp, rl in zip(out["plain"][0], out["learned"][0]):
        assert rl.iterations <= rp.iterations + (1 if rl.fallback_used else 0), (rp, rl)
        assert rl.fallback_used or rl.iterations <= rp.iterations
    it_p = np.mean([r.iterations for r in out["plain"][0]])
    it_l = np.mean([r.iterations for r in out["learned"][0]])
    fb = sum(r.fallback_used for r in out["learned"][0])
    with capsys.disabled():
        print(f"\n[trained network] mean GCR iterations: plain {it_p:.2f}, learned {it_l:.2f}, "
              f"{fb} of {B} members fell back (training loss {head.get('loss_last'):.3g} "
              f"of target mean square {head.get('target_mean_square'):.3g})")
