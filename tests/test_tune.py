"""The autotuner: workload key and table lookup (no GPU), and a solver built
with tuned=True (GPU)."""
import json

import pytest

from paper_2103_16120_amd.tune import tune_key, tuned_options


def test_key_ignores_member_order():
    a = [(512, 256), (128, 64), (512, 256)]
    b = [(128, 64), (512, 256), (512, 256)]
    assert tune_key(a, 3) == tune_key(b, 3)
    assert tune_key(a, 3) != tune_key(a, 0)
    assert tune_key(a, 3) != tune_key(a + [(128, 64)], 3)


def test_lookup_defaults_and_stored_choice(tmp_path):
    path = tmp_path / "tuned.json"
    sizes = [(512, 256)] * 4
    assert tuned_options(sizes, 3, str(path)) == {"one_stream": False, "graph": False}
    path.write_text(json.dumps({tune_key(sizes, 3): {"one_stream": True, "graph": False}}))
    assert tuned_options(sizes, 3, str(path)) == {"one_stream": True, "graph": False}
    assert tuned_options(sizes, 0, str(path)) == {"one_stream": False, "graph": False}
    path.write_text("not json")
    assert tuned_options(sizes, 3, str(path)) == {"one_stream": False, "graph": False}


@pytest.mark.gpu
def test_tuned_solver_takes_stored_choice(gpu_lib, tmp_path, monkeypatch):
    """Solver(tuned=True) applies the stored launch options for its workload,
    and the solve is bitwise the same as under the defaults."""
    import numpy as np
    import torch
    from paper_2103_16120_amd import tune
    from workloads import problem

    prs = [problem(2, 512, 256, instance=m, dt=600.0) for m in range(32)]
    sizes = [(p["nx"], p["ny"]) for p in prs]
    prec = gpu_lib.MIXED_HALF_PC
    table = tmp_path / "tuned.json"
    table.write_text(json.dumps({tune_key(sizes, prec): {"one_stream": True, "graph": True}}))
    monkeypatch.setattr(tune, "TUNED_FILE", str(table))
    depth = [torch.from_numpy(p["depth"]).cuda() for p in prs]
    dts = [p["dt"] for p in prs]
    out = {}
    for tuned in (False, True):
        s = gpu_lib.Solver(sizes, precision=prec, rtol=1e-8, tuned=tuned)
        want = (gpu_lib.F_ONE_STREAM | gpu_lib.F_GRAPH) if tuned else 0
        assert s.params.flags & (gpu_lib.F_ONE_STREAM | gpu_lib.F_GRAPH) == want
        s.set_operators(list(range(len(prs))), depth, dts)
        rhs = [s.apply_operator(m, torch.from_numpy(p["x_true"]).cuda()) for m, p in enumerate(prs)]
        sols = []
        for _ in range(2):                      # the second solve replays the captured graphs
            xs = [torch.zeros_like(r) for r in rhs]
            reps = s.solve(rhs, xs)
            torch.cuda.synchronize()
            sols.append(([r.iterations for r in reps], [x.cpu().numpy() for x in xs]))
        out[tuned] = sols
        s.close()
    for a, b in zip(out[False], out[True]):
        assert a[0] == b[0]
        assert all(np.array_equal(u, v) for u, v in zip(a[1], b[1]))
