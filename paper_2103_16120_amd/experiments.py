"""Measurements of the batched and time-sequence workloads (one JSON line each).

    python -m paper_2103_16120_amd.experiments single     # one solve (64x32 at 1e-10, 256x128 at 1e-8)
    python -m paper_2103_16120_amd.experiments batch      # 64 members of uneven grids
    python -m paper_2103_16120_amd.experiments sequence   # 200 warm-started solves at 1024x512
    python -m paper_2103_16120_amd.experiments precond    # preconditioner options 0-3, Richardson count
    python -m paper_2103_16120_amd.experiments polar      # float32 polar-band width in the mixed forms
    python -m paper_2103_16120_amd.experiments exitnorm   # Euclidean vs maximum-norm exit test
    python -m paper_2103_16120_amd.experiments split      # split single-precision residual kernel
    python -m paper_2103_16120_amd.experiments model      # the semi-implicit step around the solve

single: one member of the configuration family (depth 8000 m + 500 m x
degree<=8 harmonics, dt 600 s, R = L(degree<=12 field)), 64x32 solved to 1e-10
and 256x128 to 1e-8, in every precision form; a step is assembly + solve of
the one member, repeated.  Each form's error is its solution's relative L2
distance to the float64 solution.

batch: 64 independent solves, grids drawn from {128x64, 256x128, 512x256},
depth 4000-10000 m, dt in [300, 1200] s, solved in one batch in every
precision form; a step is the batched assembly plus the solve.  Each form's
error is its solution's relative L2 distance to the float64 solution (the
float64 solution itself is checked against the CPU oracle by the GPU tests).

sequence: depth of a zonal jet in gradient-wind balance plus advected
degree-16 perturbations, dt = 100 s; step n solves L_n(x) = L_n(Phi*_{n+1})
warm-started from the previous solution.  Plain float64, the mixed
half-precision-preconditioner form, and the mixed form with the learned
preconditioner; total wall time (assembly + solve) and the iteration
histogram.

precond: the benchmark batch (64 x 512x256, dt 600 s, rtol 1e-8) with each
preconditioner of paper Section 2.3 -- option 0 (none), 1 (diagonal of L),
2 (diagonally preconditioned explicit Richardson on L), 3 (semi-implicit
Richardson, eq. P_Operator) -- and 1 to 4 Richardson iterations for options
2 and 3; float64 form, and option 3 in the mixed half-precision-
preconditioner form.  Iterations relative to option 0 and the time per step.

polar: the benchmark batch in the three mixed forms with 0 to 8 rows per pole
kept in float32 (float16 elsewhere): iterations, the float64 true residual
and the distance to the float64 solution.

exitnorm: the benchmark batch in every precision form with the Euclidean exit
test (eq. exitcondition) and with the maximum-norm test the paper also tried:
iterations, time per step and both norms of the final true residual relative
to the initial one.

split: the split single-precision residual (Section 4.2.1, eq.
L_Operator_SP) of one member per call, 512x256, 1024x512 and 1024x4096 (the
largest grid, which alone fills the GPU), three float64 rows per pole: per-call kernel time of the split residual and of the float64
operator (per-kernel HIP events), and the split kernel's algorithmic bandwidth
(Phi_tilde 4, Phi_hat 4, four stored differences 16, Phi* 8, R 8, r 8 bytes per
point, pooled fields).

model: the semi-implicit time step of the shallow-water model around the solve
(gcr_si_step), for 64 members of 512x256 over synthetic mountains (zonal jet
u = 40 cos(lat) m/s with its balanced free surface, orography up to 2000 m of
degree <= 8, depth perturbations of 100 m up to degree 16; dt 200 s and polar
absorbers 1/(200 dt), the paper's settings for this grid).  A step is the
explicit part (forcings, MPDATA of Phi and Q, the implicit inversion), the
operator assembly from Phi*, the solve (rtol 1e-8) and the momentum recovery
for the whole batch; the timed steps repeat one step from the same state, so
every step does the same work.  Reported: time per step, its explicit-part
share (per-kernel HIP events in a separate pass), the explicit kernels'
algorithmic bandwidth (504 bytes per point: 63 float64 reads and writes),
solver iterations, and a five-step trajectory (iterations, mass drift,
largest velocity).
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _lib():
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    from paper_2103_16120_amd import lib
    return torch, lib


def single(args):
    torch, lib = _lib()
    from workloads import problem
    out = {"workload": "one solve per step: 64x32 (rtol 1e-10) and 256x128 (rtol 1e-8), dt 600 s", "cases": {}}
    for cfg, nx, ny, rtol in ((1, 64, 32, 1e-10), (2, 256, 128, 1e-8)):
        pr = problem(cfg, nx, ny, dt=600.0)
        depth = torch.from_numpy(pr["depth"]).cuda()
        f = lib.Solver([(nx, ny)], precision=lib.FP64)
        f.set_operator(0, depth, pr["dt"])
        rhs = f.apply_operator(0, torch.from_numpy(pr["x_true"]).cuda()).clone()
        f.close()
        case, ref = {}, None
        forms = [("fp64", lib.FP64), ("mixed_half_pc", lib.MIXED_HALF_PC),
                 ("mixed_fp64dot", lib.MIXED_FP64DOT), ("mixed", lib.MIXED)]
        if rtol >= 1e-8:   # the float32 cycles stop on a plateau above 1e-10
            forms += [("single", lib.SINGLE), ("single_polar64", lib.SINGLE_POLAR64)]
        for name, prec in forms:
            s = lib.Solver([(nx, ny)], precision=prec, rtol=rtol, max_iters=100)
            x = torch.zeros_like(rhs)

            def step():
                s.set_operator(0, depth, pr["dt"])
                x.zero_()
                return s.solve([rhs], [x])[0]

            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                rep = step()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            sol = x.cpu().numpy()
            if ref is None:
                ref = sol
            case[name] = {"solves_per_s": round(1.0 / dt, 1), "ms_per_solve": round(1e3 * dt, 3),
                          "iterations": rep.iterations, "status": rep.status, "rel_res_true": rep.rel_res_true,
                          "rel_l2_vs_fp64": float(np.linalg.norm(sol - ref) / np.linalg.norm(ref))}
            s.close()
            print(f"# {nx}x{ny} {name}: {json.dumps(case[name])}", flush=True)
        out["cases"][f"{nx}x{ny}"] = case
    print(json.dumps(out), flush=True)


def batch(args):
    torch, lib = _lib()
    from workloads import batch_problems
    probs = batch_problems(3, args.count)
    sizes = [(p["nx"], p["ny"]) for p in probs]
    depth = [torch.from_numpy(p["depth"]).cuda() for p in probs]
    dts = [p["dt"] for p in probs]
    f = lib.Solver(sizes, precision=lib.FP64)
    f.set_operators(list(range(len(probs))), depth, dts)
    rhs = [f.apply_operator(m, torch.from_numpy(p["x_true"]).cuda()) for m, p in enumerate(probs)]
    f.close()
    pts = sum(nx * ny for nx, ny in sizes)
    out = {"workload": f"{len(probs)} members, grids {dict(collections.Counter(f'{a}x{b}' for a, b in sizes))}, "
                       f"dt {min(dts):.0f}-{max(dts):.0f} s, rtol {args.rtol:g}",
           "points": pts, "forms": {}}
    ref = None
    for name, prec in (("fp64", lib.FP64), ("mixed_half_pc", lib.MIXED_HALF_PC),
                       ("mixed_fp64dot", lib.MIXED_FP64DOT), ("mixed", lib.MIXED), ("single", lib.SINGLE),
                       ("single_polar64", lib.SINGLE_POLAR64)):
        s = lib.Solver(sizes, precision=prec, rtol=args.rtol, max_iters=100, one_stream=args.one_stream,
                       graph=args.graph)
        # one buffer for all solutions (members of several sizes): the zero
        # initial guess is one fill
        offs = np.cumsum([0] + [nx * ny for nx, ny in sizes])
        X = torch.zeros(int(offs[-1]), dtype=torch.float64, device="cuda")
        xs = [X[offs[m]:offs[m + 1]].view(ny, nx) for m, (nx, ny) in enumerate(sizes)]

        def step():
            s.set_operators(list(range(len(probs))), depth, dts)
            X.zero_()
            return s.solve(rhs, xs)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            reps = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        sol = [x.cpu().numpy() for x in xs]
        if ref is None:
            ref = sol
        err = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(sol, ref)]
        its = [r.iterations for r in reps]
        out["forms"][name] = {"solves_per_s": round(len(probs) / dt, 1), "ms_per_step": round(1e3 * dt, 3),
                              "iters_mean": float(np.mean(its)), "iters_min": int(min(its)),
                              "iters_max": int(max(its)), "statuses": sorted(set(r.status for r in reps)),
                              "rel_res_true_max": float(max(r.rel_res_true for r in reps)),
                              "rel_l2_vs_fp64_max": max(err)}
        s.close()
        print(f"# {name}: {json.dumps(out['forms'][name])}", flush=True)
    print(json.dumps(out), flush=True)


def _bench_batch(torch, lib, count):
    from workloads import problem
    probs = [problem(2, 512, 256, instance=m, dt=600.0) for m in range(count)]
    depth = [torch.from_numpy(p["depth"]).cuda() for p in probs]
    f = lib.Solver([(512, 256)] * count, precision=lib.FP64)
    f.set_operators(list(range(count)), depth, [p["dt"] for p in probs])
    rhs = [f.apply_operator(m, torch.from_numpy(p["x_true"]).cuda()) for m, p in enumerate(probs)]
    torch.cuda.synchronize()
    f.close()
    return probs, depth, rhs


def _time_solver(torch, s, probs, depth, rhs, steps, warmup):
    # one buffer for all solutions: the zero initial guess is one fill
    X = torch.zeros((len(rhs),) + tuple(rhs[0].shape), dtype=rhs[0].dtype, device=rhs[0].device)
    xs = [X[m] for m in range(len(rhs))]

    def step():
        s.set_operators(list(range(len(probs))), depth, [p["dt"] for p in probs])
        X.zero_()
        return s.solve(rhs, xs)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        reps = step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, reps, xs


def precond(args):
    torch, lib = _lib()
    probs, depth, rhs = _bench_batch(torch, lib, args.count)
    out = {"workload": f"{args.count} x 512x256, dt 600 s, rtol {args.rtol:g}, GCR(3), max {args.max_iters} iterations",
           "cases": []}
    cases = [("fp64", lib.FP64, 0, 1), ("fp64", lib.FP64, 1, 1)]
    cases += [("fp64", lib.FP64, 2, r) for r in (1, 2, 3, 4)]
    cases += [("fp64", lib.FP64, 3, r) for r in (1, 2, 3, 4)]
    cases += [("mixed_half_pc", lib.MIXED_HALF_PC, 3, r) for r in (1, 2, 3, 4)]
    base = None
    for form, prec, opt, ri in cases:
        s = lib.Solver([(512, 256)] * args.count, precision=prec, precond=opt, richardson_iters=ri,
                       rtol=args.rtol, max_iters=args.max_iters)
        dt, reps, _ = _time_solver(torch, s, probs, depth, rhs, args.steps, args.warmup)
        s.close()
        its = [r.iterations for r in reps]
        if base is None:
            base = float(np.mean(its))
        rec = {"form": form, "option": opt, "richardson_iters": ri if opt >= 2 else None,
               "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
               "iters_vs_option0": round(float(np.mean(its)) / base - 1.0, 3),
               "statuses": sorted(set(r.status for r in reps)),
               "rel_res_true_max": float(max(r.rel_res_true for r in reps)),
               "ms_per_step": round(1e3 * dt, 3), "solves_per_s": round(len(probs) / dt, 1)}
        out["cases"].append(rec)
        print(f"# {json.dumps(rec)}", flush=True)
    print(json.dumps(out), flush=True)


def polar(args):
    torch, lib = _lib()
    probs, depth, rhs = _bench_batch(torch, lib, args.count)
    s = lib.Solver([(512, 256)] * args.count, precision=lib.FP64, rtol=args.rtol)
    _, _, ref = _time_solver(torch, s, probs, depth, rhs, 1, 0)
    s.close()
    ref = [x.cpu().numpy() for x in ref]
    out = {"workload": f"{args.count} x 512x256, dt 600 s, rtol {args.rtol:g}, GCR(3), semi-implicit Richardson x2",
           "cases": []}
    for form, prec in (("mixed", lib.MIXED), ("mixed_fp64dot", lib.MIXED_FP64DOT),
                       ("mixed_half_pc", lib.MIXED_HALF_PC)):
        for rows in (0, 1, 2, 3, 4, 8):
            s = lib.Solver([(512, 256)] * args.count, precision=prec, polar_rows=rows, rtol=args.rtol,
                           max_iters=args.max_iters)
            dt, reps, xs = _time_solver(torch, s, probs, depth, rhs, args.steps, args.warmup)
            s.close()
            err = [float(np.linalg.norm(x.cpu().numpy() - r) / np.linalg.norm(r)) for x, r in zip(xs, ref)]
            its = [r.iterations for r in reps]
            rec = {"form": form, "polar_rows": rows, "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
                   "statuses": sorted(set(r.status for r in reps)),
                   "rel_res_true_max": float(max(r.rel_res_true for r in reps)), "rel_l2_vs_fp64_max": max(err),
                   "ms_per_step": round(1e3 * dt, 3)}
            out["cases"].append(rec)
            print(f"# {json.dumps(rec)}", flush=True)
    print(json.dumps(out), flush=True)


def exitnorm(args):
    torch, lib = _lib()
    probs, depth, rhs = _bench_batch(torch, lib, args.count)
    f = lib.Solver([(512, 256)] * args.count, precision=lib.FP64)
    f.set_operators(list(range(args.count)), depth, [p["dt"] for p in probs])
    out = {"workload": f"{args.count} x 512x256, dt 600 s, rtol {args.rtol:g}, GCR(3), semi-implicit Richardson x2",
           "cases": []}
    for form, prec in (("fp64", lib.FP64), ("mixed_half_pc", lib.MIXED_HALF_PC),
                       ("mixed_fp64dot", lib.MIXED_FP64DOT), ("mixed", lib.MIXED)):
        for norm in ("l2", "linf"):
            s = lib.Solver([(512, 256)] * args.count, precision=prec, rtol=args.rtol, max_iters=args.max_iters,
                           linf_exit=norm == "linf")
            dt, reps, xs = _time_solver(torch, s, probs, depth, rhs, args.steps, args.warmup)
            s.close()
            l2, linf = [], []
            for m, x in enumerate(xs):
                r = (f.apply_operator(m, x) - rhs[m]).double()
                l2.append(float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(rhs[m])))
                linf.append(float(r.abs().max() / rhs[m].abs().max()))
            its = [r.iterations for r in reps]
            rec = {"form": form, "exit_norm": norm, "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
                   "statuses": sorted(set(r.status for r in reps)), "true_rel_l2_max": max(l2),
                   "true_rel_linf_max": max(linf), "ms_per_step": round(1e3 * dt, 3)}
            out["cases"].append(rec)
            print(f"# {json.dumps(rec)}", flush=True)
    f.close()
    print(json.dumps(out), flush=True)


def split(args):
    torch, lib = _lib()
    from workloads import problem
    out = {"workload": "split single-precision residual of one member per call, polar rows 3", "cases": {}}
    for nx, ny in ((512, 256), (1024, 512), (1024, 4096)):
        pr = problem(2, nx, ny, dt=600.0)
        s = lib.Solver([(nx, ny)], polar_rows=3)
        depth = torch.from_numpy(pr["depth"]).cuda()
        s.set_operator(0, depth, 600.0)
        base = depth - 20.0 * torch.from_numpy(pr["x_true"]).cuda()
        s.set_split_base(0, base)
        phi = depth + 3.0 * torch.from_numpy(pr["x_true"]).cuda()
        tilde = (phi - base.float().double()).float().contiguous()
        rhs = s.apply_operator(0, phi + 5.0 * torch.from_numpy(pr["x_true"]).cuda()).clone()
        r = torch.empty_like(rhs)
        y = torch.empty_like(rhs)
        for _ in range(args.warmup):
            s.residual_split(0, tilde, rhs, out=r)
            s.apply_operator(0, phi, out=y)
        torch.cuda.synchronize()
        s.set_kernel_timing(True)
        for _ in range(args.calls):
            s.residual_split(0, tilde, rhs, out=r)
            s.apply_operator(0, phi, out=y)
        kt = s.kernel_times()
        s.set_kernel_timing(False)
        n_res, ms_res = kt["residual"]
        n_op, ms_op = kt["apply_L"]
        us_res, us_op = 1e3 * ms_res / n_res, 1e3 * ms_op / n_op
        pts = nx * ny
        rel = ((r - (y - rhs)).abs().max() / (y - rhs).abs().max()).item()
        out["cases"][f"{nx}x{ny}"] = {"split_us": round(us_res, 2), "float64_operator_us": round(us_op, 2),
                                       "split_GBps": round(48.0 * pts / (us_res * 1e-6) / 1e9, 1),
                                       "split_frac_of_8TBps": round(48.0 * pts / (us_res * 1e-6) / 8e12, 4),
                                       "max_rel_diff_vs_float64": rel}
        s.close()
        print(f"# {nx}x{ny}: {json.dumps(out['cases'][f'{nx}x{ny}'])}", flush=True)
    print(json.dumps(out), flush=True)


def sequence(args):
    torch, lib = _lib()
    from workloads import jet_sequence_depth
    nx, ny, dt, n = args.nx, args.ny, args.dt, args.steps
    t0 = time.perf_counter()
    depth = [torch.from_numpy(jet_sequence_depth(nx, ny, k, dt)).cuda() for k in range(n + 1)]
    f = lib.Solver([(nx, ny)], precision=lib.FP64)
    rhs = []
    for k in range(n):
        f.set_operators([0], [depth[k]], [dt])
        rhs.append(f.apply_operator(0, depth[k + 1]).clone())
    torch.cuda.synchronize()
    f.close()
    print(f"# inputs ready in {time.perf_counter() - t0:.1f} s", flush=True)
    out = {"workload": f"{n} consecutive {nx}x{ny} solves, dt {dt:g} s, warm start, rtol {args.rtol:g}",
           "legs": {}}
    legs = [("plain_fp64", lib.FP64, lib.PC_SEMI_IMPLICIT), ("plain_mixed_half_pc", lib.MIXED_HALF_PC,
                                                              lib.PC_SEMI_IMPLICIT)]
    params = None
    if not args.no_learned:
        from paper_2103_16120_amd.learned import load_weights, DEFAULT_WEIGHTS
        params, _ = load_weights(DEFAULT_WEIGHTS)
        legs.append(("learned_mixed_half_pc", lib.MIXED_HALF_PC, lib.PC_LEARNED))
    sols = {}
    for name, prec, pc in legs:
        s = lib.Solver([(nx, ny)], precision=prec, precond=pc, rtol=args.rtol, max_iters=200)
        if pc == lib.PC_LEARNED:
            s.set_learned(params, 0.5)
        x = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
        # one untimed solve warms the kernels up; the sequence then starts from zero
        s.set_operators([0], [depth[0]], [dt])
        s.solve([rhs[0]], [x])
        x.zero_()
        torch.cuda.synchronize()
        its, stats, fb = [], [], 0
        t0 = time.perf_counter()
        for k in range(n):
            s.set_operators([0], [depth[k]], [dt])
            rep = s.solve([rhs[k]], [x])[0]
            its.append(rep.iterations)
            stats.append(rep.status)
            fb += rep.fallback_used
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sols[name] = x.cpu().numpy()
        out["legs"][name] = {"wall_s": round(wall, 4), "ms_per_solve": round(1e3 * wall / n, 3),
                             "iters_total": int(sum(its)),
                             "iters_histogram": dict(sorted(collections.Counter(its).items())),
                             "statuses": dict(collections.Counter(stats)), "fallbacks": fb}
        s.close()
        print(f"# {name}: {json.dumps(out['legs'][name])}", flush=True)
    ref = sols["plain_fp64"]
    for name, v in sols.items():
        out["legs"][name]["final_rel_l2_vs_fp64"] = float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
    print(json.dumps(out), flush=True)


def si_bytes_per_point(orography=True, qbar=False):
    """Algorithmic bytes per point of the step's explicit kernels: the float64
    fields each reads and writes once (forcings and Courant numbers 10,
    donor cell 8, antidiffusive velocities 11, corrective pass with the
    implicit inversion 19, right-hand side 6, recovery 6), plus H0 in three
    of them and the two relaxation targets in two."""
    return 8 * (60 + (3 if orography else 0) + (4 if qbar else 0))


def model(args):
    torch, lib = _lib()
    from workloads import model_state
    nx, ny, count, dt = args.nx, args.ny, args.count, args.dt
    absorber = 1.0 / (200.0 * dt)
    t0 = time.perf_counter()
    states = [model_state(nx, ny, m) for m in range(count)]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cur = [tuple(dev(st[k]) for k in ("phi", "qx", "qy")) for st in states]
    oro = [dev(st["orography"]) for st in states]
    new = [tuple(torch.empty_like(f) for f in c) for c in cur]
    lat = -0.5 * np.pi + (np.arange(ny) + 0.5) * np.pi / ny
    wcos = torch.from_numpy(np.cos(lat)[:, None].repeat(nx, 1)).cuda()
    print(f"# inputs ready in {time.perf_counter() - t0:.1f} s", flush=True)
    out = {"workload": f"{count} members of {nx}x{ny} over synthetic mountains, dt {dt:g} s, absorber 1/(200 dt), "
                       f"rtol {args.rtol:g}", "points": count * nx * ny, "forms": {}}
    for name, prec in (("fp64", lib.FP64), ("mixed_half_pc", lib.MIXED_HALF_PC)):
        s = lib.Solver([(nx, ny)] * count, precision=prec, rtol=args.rtol, max_iters=200)
        step = lambda: s.si_step(cur, cur, new, [dt] * count, orographies=oro, absorber=absorber)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            reps = step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1) / args.steps
        its = [r.iterations for r in reps]
        s.set_kernel_timing(True)
        step()
        kt = s.kernel_times()
        s.set_kernel_timing(False)
        n_si, ms_si = kt["si_step"]
        ms_solver = sum(v[1] for k, v in kt.items() if k != "si_step")
        rec = {"ms_per_step": round(ms, 3), "steps_per_s": round(1e3 / ms, 2),
               "member_steps_per_s": round(count * 1e3 / ms, 1),
               "iters_mean": float(np.mean(its)), "iters_max": int(max(its)),
               "statuses": sorted(set(r.status for r in reps)),
               "explicit_kernels": {"launches": n_si, "ms": round(ms_si, 4),
                                    "gb_per_s": round(count * nx * ny * si_bytes_per_point() / (ms_si * 1e-3) / 1e9, 1)},
               "solver_kernels_ms": round(ms_solver, 4)}
        # a short trajectory from the initial states
        a = [tuple(f.clone() for f in c) for c in cur]
        b = [tuple(f.clone() for f in c) for c in cur]
        c_ = [tuple(torch.empty_like(f) for f in x) for x in cur]
        m0 = sum(float((wcos * x[0]).sum()) for x in a)
        traj = []
        for n in range(args.trajectory):
            reps = s.si_step(b, a, c_, [dt] * count, orographies=oro, absorber=absorber)
            a, b, c_ = b, c_, a
            m1 = sum(float((wcos * x[0]).sum()) for x in b)
            vmax = max(float((x[2] / x[0]).abs().max()) for x in b)
            umax = max(float((x[1] / x[0]).abs().max()) for x in b)
            traj.append({"step": n + 1, "iters_mean": float(np.mean([r.iterations for r in reps])),
                         "mass_drift": m1 / m0 - 1.0, "u_max": round(umax, 3), "v_max": round(vmax, 4)})
        rec["trajectory"] = traj
        out["forms"][name] = rec
        s.close()
        print(f"# {name}: {json.dumps(rec)}", flush=True)
    print(json.dumps(out), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("single")
    g.add_argument("--steps", type=int, default=200)
    g.add_argument("--warmup", type=int, default=10)
    b = sub.add_parser("batch")
    b.add_argument("--count", type=int, default=64)
    b.add_argument("--steps", type=int, default=5)
    b.add_argument("--warmup", type=int, default=1)
    b.add_argument("--rtol", type=float, default=1e-8)
    b.add_argument("--one-stream", action="store_true", help="whole batch on one stream (no member groups)")
    b.add_argument("--graph", action="store_true", help="replay iterations and cycle ends from HIP graphs")
    q = sub.add_parser("sequence")
    q.add_argument("--nx", type=int, default=1024)
    q.add_argument("--ny", type=int, default=512)
    q.add_argument("--dt", type=float, default=100.0)
    q.add_argument("--steps", type=int, default=200)
    q.add_argument("--rtol", type=float, default=1e-8)
    q.add_argument("--no-learned", action="store_true")
    c = sub.add_parser("precond")
    c.add_argument("--count", type=int, default=64)
    c.add_argument("--steps", type=int, default=2)
    c.add_argument("--warmup", type=int, default=1)
    c.add_argument("--rtol", type=float, default=1e-8)
    c.add_argument("--max-iters", type=int, default=2000)
    o = sub.add_parser("polar")
    o.add_argument("--count", type=int, default=64)
    o.add_argument("--steps", type=int, default=10)
    o.add_argument("--warmup", type=int, default=3)
    o.add_argument("--rtol", type=float, default=1e-8)
    o.add_argument("--max-iters", type=int, default=200)
    e = sub.add_parser("exitnorm")
    e.add_argument("--count", type=int, default=64)
    e.add_argument("--steps", type=int, default=10)
    e.add_argument("--warmup", type=int, default=3)
    e.add_argument("--rtol", type=float, default=1e-8)
    e.add_argument("--max-iters", type=int, default=200)
    sp = sub.add_parser("split")
    sp.add_argument("--calls", type=int, default=50)
    sp.add_argument("--warmup", type=int, default=5)
    md = sub.add_parser("model")
    md.add_argument("--nx", type=int, default=512)
    md.add_argument("--ny", type=int, default=256)
    md.add_argument("--count", type=int, default=64)
    md.add_argument("--dt", type=float, default=200.0)
    md.add_argument("--steps", type=int, default=10)
    md.add_argument("--warmup", type=int, default=2)
    md.add_argument("--trajectory", type=int, default=5)
    md.add_argument("--rtol", type=float, default=1e-8)
    args = ap.parse_args(argv)
    {"model": model, "single": single, "batch": batch, "sequence": sequence, "precond": precond, "polar": polar,
     "exitnorm": exitnorm, "split": split}[args.cmd](args)


if __name__ == "__main__":
    main()
