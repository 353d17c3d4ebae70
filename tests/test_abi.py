"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects invalid arguments before touching a device."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b((?:gcr|cnn)_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2103_16120_amd import lib as L
    return L


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["gcr_create", "gcr_set_operator", "gcr_solve", "gcr_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    cdll = lib._lib
    missing = [n for n in sorted(_declared()) if not hasattr(cdll, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(lib):
    assert _declared() <= set(lib._SIGNATURES)


def test_version_and_status_strings(lib):
    assert "gfx950" in lib.version()
    assert "converged" in lib.status_string(lib.OK)
    assert "invalid" in lib.status_string(lib.EINVAL)


def _params(lib, nx=(64,), ny=(32,), **kw):
    p = lib.GcrParams()
    assert lib._lib.gcr_default_params(C.byref(p)) == lib.OK
    b = len(nx)
    p.batch = b
    p._nxa = (C.c_int32 * b)(*nx)
    p._nya = (C.c_int32 * b)(*ny)
    p.nx, p.ny = p._nxa, p._nya
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_defaults(lib):
    p = lib.GcrParams()
    lib._lib.gcr_default_params(C.byref(p))
    assert (p.k, p.precision, p.precond, p.richardson_iters, p.max_iters) == (3, lib.FP64, lib.PC_SEMI_IMPLICIT, 2, 200)
    assert p.rtol == 1e-8 and p.min_iters == -1 and p.polar_rows == -1
    assert lib._lib.gcr_default_params(None) == lib.EINVAL


@pytest.mark.parametrize("bad", [
    dict(nx=(63,)), dict(nx=(2048,)), dict(nx=(4,)), dict(ny=(1,)), dict(k=0), dict(k=9),
    dict(precision=7), dict(precond=9), dict(richardson_iters=0), dict(max_iters=0),
    dict(rtol=-1.0), dict(rtol=float("nan")), dict(min_iters=500), dict(polar_rows=-2),
])
def test_create_rejects_invalid_params(lib, bad):
    kw = dict(bad)
    nx = kw.pop("nx", (64,))
    ny = kw.pop("ny", (32,))
    p = _params(lib, nx, ny, **kw)
    h = C.c_void_p(123)
    assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL
    assert h.value is None
    assert len(lib._lib.gcr_last_error(None)) > 0


def test_create_null_and_batch_limits(lib):
    h = C.c_void_p()
    assert lib._lib.gcr_create(None, C.byref(h)) == lib.EINVAL
    p = _params(lib)
    p.batch = 0
    assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL
    p = _params(lib)
    p.nx = None
    assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL


def test_destroy_null_is_noop(lib):
    assert lib._lib.gcr_destroy(None) == lib.OK


def test_entry_points_reject_null_solver(lib):
    assert lib._lib.gcr_set_operator(None, 0, None) == lib.EINVAL
    assert lib._lib.gcr_solve(None, None, None, None) == lib.EINVAL
    assert lib._lib.gcr_apply_operator(None, 0, None, None) == lib.EINVAL
    assert lib._lib.gcr_apply_precond(None, 0, None, None) == lib.EINVAL
    assert lib._lib.gcr_si_step(None, None, None) == lib.EINVAL


def test_create_without_gpu_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = _params(lib)
    h = C.c_void_p()
    rc = lib._lib.gcr_create(C.byref(p), C.byref(h))
    assert rc == lib.EHIP and h.value is None


def test_network_entry_points_without_gpu(lib):
    # parameter count: 3 -> 32 -> 32 -> 32 -> 32 -> 1 with 3x3 kernels and biases
    assert lib._lib.cnn_param_count(3) == (32 * 3 * 9 + 32) + 3 * (32 * 32 * 9 + 32) + (32 * 9 + 1)
    assert lib._lib.cnn_param_count(0) == -1 and lib._lib.cnn_param_count(33) == -1
    assert lib._lib.cnn_destroy(None) == lib.OK
    h = C.c_void_p()
    for nx, ny, b, c in ((48, 16, 1, 3), (2048, 16, 1, 3), (64, 1, 1, 3), (64, 16, 0, 3), (64, 16, 1, 0)):
        assert lib._lib.cnn_create(nx, ny, b, c, None, C.byref(h)) == lib.EINVAL
        assert h.value is None
        assert lib._lib.cnn_last_error(None)
    assert lib._lib.cnn_set_params(None, None, 0) == lib.EINVAL
    assert lib._lib.cnn_get_params(None, None, 0) == lib.EINVAL
    assert lib._lib.cnn_forward(None, 1, None, None) == lib.EINVAL
    assert lib._lib.cnn_gradients(None, 1, None, None, None) == lib.EINVAL
    assert lib._lib.cnn_train_step(None, 1, None, None, 1e-3, None) == lib.EINVAL
    assert lib._lib.gcr_set_learned(None, None, 0, 0.5) == lib.EINVAL
    assert lib._lib.gcr_learned_features(None, 0, None, None, 0, None, None, None) == lib.EINVAL


def test_learned_create_needs_one_size(lib):
    p = _params(lib)
    nx = (C.c_int32 * 2)(64, 128)
    ny = (C.c_int32 * 2)(16, 16)
    p.batch, p.nx, p.ny = 2, nx, ny
    p.precond = lib.PC_LEARNED
    h = C.c_void_p()
    assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL
    assert b"one size" in lib._lib.gcr_last_error(None)


def test_create_rejects_unknown_flags(lib):
    p = _params(lib, flags=0x80)
    h = C.c_void_p()
    assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL
    assert b"flags" in lib._lib.gcr_last_error(None)


def test_fault_injection_flags_validated_before_the_device(lib):
    """The two fault-injection flags are known (a GPU-less create fails on
    the device, not on the flags), and they exclude each other."""
    import torch
    h = C.c_void_p()
    p = _params(lib, flags=lib.F_FAULT_NAN_PC | lib.F_FAULT_ZERO_DIR)
    assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL
    assert b"fault" in lib._lib.gcr_last_error(None)
    if torch.cuda.is_available():
        return
    for f in (lib.F_FAULT_NAN_PC, lib.F_FAULT_ZERO_DIR, lib.F_FAULT_NAN_PC | lib.F_RECORD_HISTORY):
        p = _params(lib, flags=f)
        assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EHIP
        assert h.value is None


def test_header_flag_values_match_the_binding(lib):
    text = open(os.path.join(ROOT, "include", "mpgcr.h")).read()
    vals = {m.group(1): int(m.group(2), 16) for m in re.finditer(r"#define GCR_F_(\w+)\s+0x([0-9a-fA-F]+)u", text)}
    for name, v in vals.items():
        assert getattr(lib, "F_" + name) == v, name
    assert set(vals) >= {"RECORD_HISTORY", "ONE_STREAM", "LINF_EXIT", "FAULT_NAN_PC", "FAULT_ZERO_DIR", "SPLIT_R0", "GRAPH"}


def test_split_r0_flag_needs_a_single_precision_cycle(lib):
    h = C.c_void_p()
    for prec in (lib.FP64, lib.MIXED_HALF_PC, lib.MIXED):
        p = _params(lib, flags=lib.F_SPLIT_R0, precision=prec)
        assert lib._lib.gcr_create(C.byref(p), C.byref(h)) == lib.EINVAL
        assert b"SPLIT_R0" in lib._lib.gcr_last_error(None)


def test_learned_reference_rejects_null_solver(lib):
    assert lib._lib.gcr_set_learned_reference(None, None, 0) == lib.EINVAL


def test_static_preconditioner_validates_before_the_device(lib):
    """gcr_apply_precond_static rejects sizes beyond its static work array and
    bad arguments with GCR_EINVAL and a message, without touching a device."""
    op = lib.GcrOperator(dt=600.0, g=lib.GRAVITY, omega=lib.OMEGA, radius=lib.RADIUS, absorber=0.0,
                         depth=C.c_void_p(64), orography=None, b_terms=1, mem_is_device=1)
    f = lib._lib.gcr_apply_precond_static
    one, two = C.c_void_p(128), C.c_void_p(256)
    assert f(512, 512, C.addressof(op), 2, one, two, None) == lib.EINVAL
    assert b"exceeds" in lib._lib.gcr_last_error(None)
    assert f(48, 16, C.addressof(op), 2, one, two, None) == lib.EINVAL
    assert f(64, 1, C.addressof(op), 2, one, two, None) == lib.EINVAL
    assert f(64, 32, C.addressof(op), 0, one, two, None) == lib.EINVAL
    assert f(64, 32, None, 2, one, two, None) == lib.EINVAL
    assert f(64, 32, C.addressof(op), 2, one, one, None) == lib.EINVAL
    op.mem_is_device = 0
    assert f(64, 32, C.addressof(op), 2, one, two, None) == lib.EINVAL
    assert lib.STATIC_MAX_POINTS == 131072
    text = open(os.path.join(ROOT, "include", "mpgcr.h")).read()
    assert "#define GCR_STATIC_MAX_POINTS 131072" in text


def test_si_member_layout_matches_the_header(lib):
    # twelve field pointers, then dt, g, omega, radius, absorber
    assert C.sizeof(lib.GcrSiMember) == 12 * 8 + 5 * 8
    assert lib.GcrSiMember.dt.offset == 96 and lib.GcrSiMember.absorber.offset == 128



def test_batch_tables_match_the_c_structs(lib):
    """The numpy views the binding fills and reads have the C structs' layout:
    a table filled column by column equals the one built field by field, and
    the report view reads back what was written through ctypes."""
    import numpy as np
    n = 5
    dts, ptrs = [600.0, 300.5, 100.0, 50.0, 1.0], [4096 + 64 * i for i in range(n)]
    oro = [None, 77824, None, 5120, None]
    ref = (lib.GcrOperator * n)()
    for t in range(n):
        ref[t] = lib.GcrOperator(dt=dts[t], g=9.8, omega=7.292e-5, radius=6.371e6, absorber=0.25, depth=ptrs[t],
                                 orography=oro[t], b_terms=1, mem_is_device=1)
    ops = np.zeros(n, dtype=lib._OP_DTYPE)
    ops["dt"] = dts
    ops["g"], ops["omega"], ops["radius"], ops["absorber"] = 9.8, 7.292e-5, 6.371e6, 0.25
    ops["depth"] = ptrs
    ops["orography"] = [0 if o is None else o for o in oro]
    ops["b_terms"], ops["mem_is_device"] = 1, 1
    assert lib._OP_DTYPE.itemsize == C.sizeof(lib.GcrOperator)
    assert ops.tobytes() == bytes(ref)
    reps = (lib.GcrReport * 3)()
    for m in range(3):
        r = reps[m]
        r.status, r.iterations, r.restarts, r.fallback_used = m - 1, 5 + m, m, m % 2
        r.r0_norm, r.rel_res_recursive, r.rel_res_true, r.history_len = 1.5 * m, 1e-9 * m, 2e-9 * m, 7
    tab = np.frombuffer(reps, dtype=lib._REP_DTYPE)
    got = list(zip(*[tab[f].tolist() for f in lib._REP_FIELDS]))
    assert got == [(r.status, r.iterations, r.restarts, r.fallback_used, r.r0_norm, r.rel_res_recursive,
                    r.rel_res_true) for r in reps]


def test_field_list_checks_name_the_failing_entry(lib):
    import torch
    shapes = [torch.Size((4, 8))] * 3
    with pytest.raises(ValueError, match="3 fields expected"):
        lib._check_fields([torch.zeros(4, 8, dtype=torch.float64)] * 2, shapes, "rhs")
    with pytest.raises(TypeError, match=r"rhs\[0\] must be a CUDA tensor"):
        lib._check_fields([torch.zeros(4, 8, dtype=torch.float64)] * 3, shapes, "rhs")
    with pytest.raises(TypeError, match=r"x\[0\] must be a CUDA tensor"):
        lib._check_fields([None, None, None], shapes, "x")


def test_si_member_table_matches_the_c_struct(lib):
    import numpy as np
    fields = [f for f, _ in lib.GcrSiMember._fields_]
    ref = (lib.GcrSiMember * 2)()
    tab = np.zeros(2, dtype=lib._SI_DTYPE)
    for m in range(2):
        for i, f in enumerate(fields):
            v = float(i + 0.5 + 100 * m) if f in ("dt", "g", "omega", "radius", "absorber") else 256 * (i + 1) + m
            setattr(ref[m], f, v)
            tab[f][m] = v
    assert lib._SI_DTYPE.itemsize == C.sizeof(lib.GcrSiMember)
    assert tab.tobytes() == bytes(ref)
