"""Training and storage of the learned preconditioner's network.

Data: for seeded depth problems of the benchmark family, the residuals r_n
of plain GCR(3) after n = 0..n_max iterations (float64 solves on the GPU),
turned into network inputs and targets by gcr_learned_features:
    input  = (r / sigma, e_lo / (s sigma), cos(lat)),
    target = T(e_hi - e_lo) / (s sigma),
where e_lo / e_hi are the semi-implicit Richardson preconditioner with 2 and
`hi_iters` iterations and T its row operator (the solver adds
T^{-1}(s sigma N) to e_lo).  A network that reproduces the target turns the
2-iteration preconditioner into the stronger one at the cost of one network
evaluation.  Training: Adam on the mean squared error, all on the GPU
(cnn_train_step).

Weights file: 8-byte little-endian header length, a JSON header (format,
channels, parameter count, training summary), then the float32 parameters in
the order of cnn_param_count.

    python -m paper_2103_16120_amd.learned --out weights.bin
"""
from __future__ import annotations

import argparse
import json
import os
import struct
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "learned_512x256.bin")
MAGIC = "mpgcr-learned-v1"


def save_weights(path, params, header):
    params = np.ascontiguousarray(params, dtype=np.float32).ravel()
    head = dict(header, format=MAGIC, count=int(params.size))
    blob = json.dumps(head, sort_keys=True).encode()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "wb") as f:
        f.write(struct.pack("<Q", len(blob)))
        f.write(blob)
        f.write(params.astype("<f4").tobytes())


def load_weights(path):
    """Returns (params float32 array, header dict)."""
    with open(path, "rb") as f:
        n = struct.unpack("<Q", f.read(8))[0]
        if n > 1 << 20:
            raise ValueError(f"{path}: header too long")
        head = json.loads(f.read(n).decode())
        if head.get("format") != MAGIC:
            raise ValueError(f"{path}: not a learned-preconditioner weights file")
        params = np.frombuffer(f.read(), dtype="<f4").astype(np.float32)
    if params.size != head["count"]:
        raise ValueError(f"{path}: {params.size} parameters, header says {head['count']}")
    return params, head


def reference_history(reports):
    """Reference residual history for the learned fallback
    (gcr_set_learned_reference): entry i is the geometric mean over the
    members of the plain solve's relative residual after iteration i, for the
    iterations every member reached (reports: lib.Report with history)."""
    hs = [r.history for r in reports if r.history]
    if not hs:
        return []
    n = min(len(h) for h in hs)
    h = np.array([h[:n] for h in hs], dtype=np.float64)
    with np.errstate(divide="ignore"):
        ref = np.exp(np.mean(np.log(np.maximum(h, 1e-300)), axis=0))
    return list(ref)


def family_problems(family, nx, ny, first_instance, count):
    """Seeded problems of a workload family: "bench" -- the benchmark's
    (depth 8000 m + 500 m degree <= 8 harmonics, dt 600 s); "batch" -- the
    uneven batch's style at one grid (depth 4000-10000 m, dt uniform in
    [300, 1200] s), with seeds of its own."""
    from workloads import problem
    if family == "bench":
        return [problem(2, nx, ny, instance=first_instance + m, dt=600.0) for m in range(count)]
    out = []
    for m in range(count):
        rng = np.random.default_rng(41_000 + first_instance + m)
        out.append(problem(4, nx, ny, instance=first_instance + m, dt=float(rng.uniform(300.0, 1200.0)),
                           depth_mean=7000.0, depth_amp=3000.0))
    return out


def initial_guesses(p, starts):
    """x_0 of the residual sequences of one problem: zero, then x_true plus
    seeded smooth perturbations of decreasing size and growing degree (warm
    starts of a time-stepping run)."""
    from workloads import harmonic_field
    nx, ny = p["nx"], p["ny"]
    out = [np.zeros((ny, nx))]
    for k in range(1, starts):
        rng = np.random.default_rng(p["seed"] * 7 + k)
        amp = 10.0 ** (-k)
        out.append(p["x_true"] + harmonic_field(nx, ny, 8 + 8 * k, rng, lmin=1, amplitude=amp))
    return out


def make_dataset(lib, torch, nx, ny, problems, first_instance, n_max, hi_iters, group=16, log=print,
                 family="bench", starts=1):
    """Features [S, 3, ny, nx] and targets [S, ny, nx] (float32 CUDA tensors):
    for each problem and each of `starts` initial guesses, the residuals after
    0..n_max plain float64 GCR(3) iterations."""
    feats, targets = [], []
    for g0 in range(0, problems, group):
        cnt = min(group, problems - g0)
        prs = family_problems(family, nx, ny, first_instance + g0, cnt)
        depth = [torch.from_numpy(p["depth"]).cuda() for p in prs]
        fs = lib.Solver([(nx, ny)] * cnt, precision=lib.FP64, precond=lib.PC_SEMI_IMPLICIT)
        for m, p in enumerate(prs):
            fs.set_operator(m, depth[m], p["dt"])
        rhs = [fs.apply_operator(m, torch.from_numpy(p["x_true"]).cuda()) for m, p in enumerate(prs)]
        guesses = [initial_guesses(p, starts) for p in prs]
        for st in range(starts):
            for n in range(0, n_max + 1):
                x = [torch.from_numpy(guesses[m][st]).cuda() for m in range(cnt)]
                if n > 0:
                    s = lib.Solver([(nx, ny)] * cnt, precision=lib.FP64, precond=lib.PC_SEMI_IMPLICIT,
                                   min_iters=n, max_iters=n, rtol=0.0)
                    for m, p in enumerate(prs):
                        s.set_operator(m, depth[m], p["dt"])
                    s.solve(rhs, x)
                    s.close()
                for m in range(cnt):
                    f, t, sig = fs.learned_features(m, x[m], rhs[m], hi_iters=hi_iters)
                    if sig > 0:
                        feats.append(f)
                        targets.append(t)
        fs.close()
        log(f"data: {g0 + cnt}/{problems} problems, {len(feats)} samples")
    return torch.stack(feats), torch.stack(targets)


def init_params(c_in, seed, width=32, layers=5):
    """He-normal weights, zero biases, a zero last layer (the network starts
    as no correction); flat float32 in the cnn_param_count order."""
    rng = np.random.default_rng(seed)
    out = []
    for n in range(layers):
        ci = c_in if n == 0 else width
        co = 1 if n == layers - 1 else width
        w = rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci))
        if n == layers - 1:
            w[:] = 0.0
        out += [w, np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


def train(lib, torch, feats, targets, steps, batch, lr, seed=0, log=print, params0=None, lr_final=None):
    """Adam on random mini-batches of the dataset, learning rate decaying
    from lr to lr_final along a cosine; returns (params, losses)."""
    nx, ny = feats.shape[3], feats.shape[2]
    net = lib.Network(nx, ny, batch, lib.LEARNED_CHANNELS)
    net.set_params(init_params(lib.LEARNED_CHANNELS, seed) if params0 is None else params0)
    rng = np.random.default_rng(seed)
    S = feats.shape[0]
    losses = []
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.from_numpy(rng.choice(S, size=min(batch, S), replace=False)).cuda()
        xb = feats.index_select(0, idx).contiguous()
        tb = targets.index_select(0, idx).contiguous()
        rate = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * it / steps))
        losses.append(net.train_step(xb, tb, rate))
        if (it + 1) % max(1, steps // 10) == 0:
            log(f"step {it + 1}/{steps}: loss {np.mean(losses[-50:]):.4e} ({time.perf_counter() - t0:.1f} s)")
    params = net.get_params()
    net.close()
    return params, losses


def evaluate(lib, torch, params, nx, ny, count, precision, fallback_ratio=0.5, first_instance=0, family="bench"):
    """Iterations and solve time of plain vs learned on `count` held-out
    problems; the learned solve falls back against the plain solve's
    residual history."""
    prs = family_problems(family, nx, ny, first_instance, count)
    depth = [torch.from_numpy(p["depth"]).cuda() for p in prs]
    f = lib.Solver([(nx, ny)] * count, precision=lib.FP64)
    for m, p in enumerate(prs):
        f.set_operator(m, depth[m], p["dt"])
    rhs = [f.apply_operator(m, torch.from_numpy(p["x_true"]).cuda()) for m, p in enumerate(prs)]
    f.close()
    out = {}
    ref = None
    for name, pc in (("plain", lib.PC_SEMI_IMPLICIT), ("learned", lib.PC_LEARNED)):
        s = lib.Solver([(nx, ny)] * count, precision=precision, precond=pc, max_iters=100, record_history=True)
        if pc == lib.PC_LEARNED:
            s.set_learned(params, fallback_ratio)
            s.set_learned_reference(ref)
        s.set_operators(list(range(count)), depth, [p["dt"] for p in prs])
        x = [torch.zeros_like(r) for r in rhs]
        warm = s.solve(rhs, x, record_history=True)      # warm-up
        if ref is None:
            ref = reference_history(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for xx in x:
            xx.zero_()
        reps = s.solve(rhs, x)
        dt = time.perf_counter() - t0
        its = [r.iterations for r in reps]
        out[name] = dict(iters=its, iters_mean=float(np.mean(its)), iters_min=int(min(its)), iters_max=int(max(its)),
                         fallbacks=int(sum(r.fallback_used for r in reps)),
                         rel_res_true_max=float(max(r.rel_res_true for r in reps)),
                         ms=round(1e3 * dt, 3))
        s.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--problems", type=int, default=64)
    ap.add_argument("--first-instance", type=int, default=1000)
    ap.add_argument("--n-max", type=int, default=5, help="residuals after 0..n_max GCR iterations")
    ap.add_argument("--hi-iters", type=int, default=4, help="Richardson iterations of the target")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval", type=int, default=32, help="held-out problems for the comparison")
    ap.add_argument("--family", default="bench", choices=("bench", "batch"), help="training problems")
    ap.add_argument("--starts", type=int, default=1, help="initial guesses per problem")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2103_16120_amd import lib

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    feats, targets = make_dataset(lib, torch, args.nx, args.ny, args.problems, args.first_instance, args.n_max,
                                  args.hi_iters, log=log, family=args.family, starts=args.starts)
    log(f"dataset {tuple(feats.shape)} in {time.perf_counter() - t0:.1f} s; target rms "
        f"{float(targets.double().pow(2).mean().sqrt()):.3e}")
    params, losses = train(lib, torch, feats, targets, args.steps, args.batch, args.lr, args.seed, log=log,
                           lr_final=args.lr_final)
    base = float(targets.double().pow(2).mean())
    summary = dict(nx=args.nx, ny=args.ny, problems=args.problems, family=args.family, starts=args.starts,
                   samples=int(feats.shape[0]), n_max=args.n_max, hi_iters=args.hi_iters,
                   steps=args.steps, batch=args.batch, lr=args.lr, lr_final=args.lr_final, seed=args.seed,
                   loss_first=float(np.mean(losses[:20])), loss_last=float(np.mean(losses[-50:])),
                   target_mean_square=base, channels=lib.LEARNED_CHANNELS)
    del feats, targets
    ev = {}
    for prec_name, prec in (("fp64", lib.FP64), ("mixed_half_pc", lib.MIXED_HALF_PC)):
        # held out: the benchmark's members (instances 0.., disjoint from any
        # training seed) and further problems of the training family
        ev[prec_name] = evaluate(lib, torch, params, args.nx, args.ny, args.eval, prec)
        ev[prec_name + "_family"] = evaluate(lib, torch, params, args.nx, args.ny, args.eval, prec,
                                             first_instance=args.first_instance + args.problems,
                                             family=args.family)
        log(f"{prec_name}: {json.dumps(ev[prec_name])}")
        log(f"{prec_name} ({args.family} family): {json.dumps(ev[prec_name + '_family'])}")
    summary["evaluation"] = ev
    save_weights(args.out, params, summary)
    log(json.dumps(summary))


if __name__ == "__main__":
    main()
