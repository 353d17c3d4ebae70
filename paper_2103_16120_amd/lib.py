"""ctypes binding of the mpgcr C-ABI (include/mpgcr.h).

Argument marshalling only: every step of the solve runs in the HIP library.
torch supplies device memory and the stream; fields are float64 CUDA tensors
of shape (ny, nx), contiguous.  When the library has not been built this
module raises at import time instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

from .build import lib_path

# status codes / enums (mirroring include/mpgcr.h)
OK, NOT_CONVERGED, STAGNATED, FALLBACK_USED = 0, 1, 2, 3
EINVAL, ENOMEM, EHIP, ESTATE = -1, -2, -3, -4
FP64, MIXED, MIXED_FP64DOT, MIXED_HALF_PC, SINGLE, SINGLE_POLAR64 = 0, 1, 2, 3, 4, 5
PC_NONE, PC_DIAG, PC_RICHARDSON, PC_SEMI_IMPLICIT, PC_LEARNED = 0, 1, 2, 3, 4
F_RECORD_HISTORY = 0x1
F_ONE_STREAM = 0x2
F_LINF_EXIT = 0x4
F_FAULT_NAN_PC = 0x8
F_FAULT_ZERO_DIR = 0x10
F_SPLIT_R0 = 0x20
F_GRAPH = 0x40

RADIUS = 6.371e6
GRAVITY = 9.80616
OMEGA = 7.292e-5


class GcrParams(C.Structure):
    _fields_ = [
        ("batch", C.c_int32), ("nx", C.POINTER(C.c_int32)), ("ny", C.POINTER(C.c_int32)),
        ("k", C.c_int32), ("precision", C.c_int32), ("precond", C.c_int32),
        ("richardson_iters", C.c_int32), ("polar_rows", C.c_int32), ("min_iters", C.c_int32),
        ("max_iters", C.c_int32), ("rtol", C.c_double), ("stream", C.c_void_p), ("flags", C.c_uint32),
    ]


class GcrOperator(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("g", C.c_double), ("omega", C.c_double), ("radius", C.c_double),
        ("absorber", C.c_double), ("depth", C.c_void_p), ("orography", C.c_void_p),
        ("b_terms", C.c_int32), ("mem_is_device", C.c_int32),
    ]


class GcrReport(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
        ("fallback_used", C.c_int32), ("r0_norm", C.c_double), ("rel_res_recursive", C.c_double),
        ("rel_res_true", C.c_double), ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
        ("history_len", C.c_int32),
    ]


class GcrSiMember(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("phi", "qx", "qy", "phi_old", "qx_old", "qy_old", "orography", "qbar_x",
                                          "qbar_y", "phi_new", "qx_new", "qy_new")] + [
        (n, C.c_double) for n in ("dt", "g", "omega", "radius", "absorber")]


# every symbol the header declares, with its ctypes signature
_SIGNATURES = {
    "gcr_default_params": (C.c_int, [C.POINTER(GcrParams)]),
    "gcr_create": (C.c_int, [C.POINTER(GcrParams), C.POINTER(C.c_void_p)]),
    "gcr_set_operator": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(GcrOperator)]),
    "gcr_set_operators": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(GcrOperator)]),
    "gcr_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(GcrReport)]),
    "gcr_apply_operator": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "gcr_set_split_base": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "gcr_residual_split": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gcr_apply_precond": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "gcr_apply_operator_form": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "gcr_apply_precond_form": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "gcr_destroy": (C.c_int, [C.c_void_p]),
    "gcr_si_step": (C.c_int, [C.c_void_p, C.POINTER(GcrSiMember), C.POINTER(GcrReport)]),
    "gcr_apply_precond_static": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "gcr_status_string": (C.c_char_p, [C.c_int]),
    "gcr_last_error": (C.c_char_p, [C.c_void_p]),
    "gcr_version": (C.c_char_p, []),
    "gcr_set_kernel_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "gcr_kernel_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "gcr_kernel_name": (C.c_char_p, [C.c_int32]),
    "gcr_set_learned": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double]),
    "gcr_set_learned_reference": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32]),
    "gcr_learned_features": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.POINTER(C.c_double)]),
    "cnn_param_count": (C.c_int64, [C.c_int]),
    "cnn_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "cnn_set_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "cnn_get_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "cnn_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "cnn_gradients": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cnn_train_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_float,
                                 C.POINTER(C.c_double)]),
    "cnn_destroy": (C.c_int, [C.c_void_p]),
    "cnn_last_error": (C.c_char_p, [C.c_void_p]),
}

K_ASSEMBLE, K_RESIDUAL, K_SWEEP1, K_SWEEP2, K_APPLY_L, K_ORTH, K_CONTROL, K_COPY, K_LEARNED, K_SOLUTION, \
    K_SI_STEP = range(11)
K_COUNT = 11
LEARNED_CHANNELS = 3


def _load():
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"mpgcr HIP library not built ({path}); run python -m paper_2103_16120_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class GcrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.gcr_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def version() -> str:
    return _lib.gcr_version().decode()


def status_string(code: int) -> str:
    return _lib.gcr_status_string(code).decode()


@dataclass
class Report:
    status: int
    iterations: int
    restarts: int
    fallback_used: int
    r0_norm: float
    rel_res_recursive: float
    rel_res_true: float
    history: list


def _check_field(t: torch.Tensor, ny: int, nx: int, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (ny, nx):
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape ({ny}, {nx})")


_F64 = torch.float64


def _check_fields(ts, shapes, name: str):
    """_check_field over a list (shapes: torch.Size (ny, nx) per entry): one
    pass of cheap attribute tests; the per-entry check only names a failure."""
    if len(ts) != len(shapes):
        raise ValueError(f"{name}: {len(shapes)} fields expected, got {len(ts)}")
    for t, shp in zip(ts, shapes):
        if not (isinstance(t, torch.Tensor) and t.dtype is _F64 and t.is_cuda and t.shape == shp
                and t.is_contiguous()):
            for m, (u, sh) in enumerate(zip(ts, shapes)):
                _check_field(u, sh[0], sh[1], f"{name}[{m}]")
            raise ValueError(f"{name}: contiguous float64 CUDA tensors of the members' shapes expected")


# numpy views of the operator and report tables (one row per member), so a
# batch is filled and read column by column instead of field by field
_OP_DTYPE = np.dtype(GcrOperator)
_SI_DTYPE = np.dtype(GcrSiMember)
_REP_FIELDS = ("status", "iterations", "restarts", "fallback_used", "r0_norm", "rel_res_recursive", "rel_res_true")
_REP_DTYPE = np.dtype({"names": list(_REP_FIELDS), "formats": ["<i4"] * 4 + ["<f8"] * 3,
                       "offsets": [getattr(GcrReport, f).offset for f in _REP_FIELDS],
                       "itemsize": C.sizeof(GcrReport)})


class Solver:
    """A batch of independent GCR(k) depth solves sharing one configuration."""

    def __init__(self, sizes, k=3, precision=FP64, precond=PC_SEMI_IMPLICIT, richardson_iters=2,
                 polar_rows=-1, min_iters=-1, max_iters=200, rtol=1e-8, stream=None, flags=0, one_stream=False,
                 linf_exit=False, record_history=False, graph=False, tuned=False):
        """tuned: take one_stream / graph from the autotuner's table for this
        workload (paper_2103_16120_amd.tune), overriding the arguments."""
        self.sizes = [(int(nx), int(ny)) for nx, ny in sizes]
        self._shapes = [torch.Size((ny, nx)) for nx, ny in self.sizes]
        if tuned:
            from .tune import tuned_options
            opt = tuned_options(self.sizes, precision)
            one_stream, graph = opt["one_stream"], opt["graph"]
        b = len(self.sizes)
        self._nx = (C.c_int32 * b)(*[s[0] for s in self.sizes])
        self._ny = (C.c_int32 * b)(*[s[1] for s in self.sizes])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        p = GcrParams()
        _lib.gcr_default_params(C.byref(p))
        p.batch, p.nx, p.ny = b, self._nx, self._ny
        p.k, p.precision, p.precond = k, precision, precond
        p.richardson_iters, p.polar_rows = richardson_iters, polar_rows
        p.min_iters, p.max_iters, p.rtol = min_iters, max_iters, rtol
        p.stream = C.c_void_p(stream.cuda_stream)
        p.flags = (flags | (F_ONE_STREAM if one_stream else 0) | (F_LINF_EXIT if linf_exit else 0)
                   | (F_RECORD_HISTORY if record_history else 0) | (F_GRAPH if graph else 0))
        self.params = p
        h = C.c_void_p()
        rc = _lib.gcr_create(C.byref(p), C.byref(h))
        if rc < 0:
            raise GcrError(rc, _lib.gcr_last_error(None).decode())
        self._h = h
        self.max_iters = max_iters

    def _err(self, rc):
        return GcrError(rc, _lib.gcr_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.gcr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_operator(self, member, depth, dt, orography=None, absorber=0.0, g=GRAVITY, omega=OMEGA,
                     radius=RADIUS, b_terms=True):
        """depth / orography: float64 CUDA tensors (ny, nx) or numpy arrays."""
        nx, ny = self.sizes[member]
        keep = []

        def ptr(a):
            if a is None:
                return None, None
            if isinstance(a, torch.Tensor):
                _check_field(a, ny, nx, "field")
                return a.data_ptr(), 1
            import numpy as np
            arr = np.ascontiguousarray(a, dtype=np.float64)
            if arr.shape != (ny, nx):
                raise ValueError(f"field must have shape ({ny}, {nx})")
            keep.append(arr)
            return arr.ctypes.data, 0

        dptr, dev = ptr(depth)
        optr, odev = ptr(orography)
        if optr is not None and odev != dev:
            raise ValueError("depth and orography must both be on the host or both on the device")
        op = GcrOperator(dt=dt, g=g, omega=omega, radius=radius, absorber=absorber, depth=dptr,
                         orography=optr, b_terms=1 if b_terms else 0, mem_is_device=dev)
        rc = _lib.gcr_set_operator(self._h, member, C.byref(op))
        if rc < 0:
            raise self._err(rc)

    def set_operators(self, members, depths, dts, orographies=None, absorber=0.0, g=GRAVITY, omega=OMEGA,
                      radius=RADIUS, b_terms=True):
        """Assemble several members in one launch.  depths / orographies:
        float64 CUDA tensors (ny, nx), kept alive by the caller until the
        stream has run the assembly (the next solve synchronises)."""
        n = len(members)
        if len(depths) != n or len(dts) != n:
            raise ValueError("one depth and one dt per member")
        mem = np.array(members, dtype=np.int32)
        if mem.ndim != 1 or (n and (mem.min() < 0 or mem.max() >= len(self.sizes))):
            raise ValueError(f"members must lie in 0..{len(self.sizes) - 1}")
        shapes = [self._shapes[m] for m in mem.tolist()]
        _check_fields(depths, shapes, "depth")
        ops = np.zeros(n, dtype=_OP_DTYPE)
        ops["dt"] = dts
        ops["g"], ops["omega"], ops["radius"], ops["absorber"] = g, omega, radius, absorber
        ops["depth"] = [t.data_ptr() for t in depths]
        if orographies is not None:
            if len(orographies) != n:
                raise ValueError("one orography (or None) per member")
            for t, o in enumerate(orographies):
                if o is not None:
                    _check_field(o, shapes[t][0], shapes[t][1], f"orography[{t}]")
            ops["orography"] = [0 if o is None else o.data_ptr() for o in orographies]
        ops["b_terms"] = 1 if b_terms else 0
        ops["mem_is_device"] = 1
        rc = _lib.gcr_set_operators(self._h, n, mem.ctypes.data_as(C.POINTER(C.c_int32)),
                                    ops.ctypes.data_as(C.POINTER(GcrOperator)))
        if rc < 0:
            raise self._err(rc)

    def solve(self, rhs, x, record_history=False):
        """rhs, x: lists (one per member) of float64 CUDA tensors; x is updated
        in place.  Returns a list of Report."""
        b = len(self.sizes)
        if len(rhs) != b or len(x) != b:
            raise ValueError("one rhs and one x per member")
        if record_history and not (self.params.flags & F_RECORD_HISTORY):
            raise ValueError("record_history needs a solver created with record_history=True")
        _check_fields(rhs, self._shapes, "rhs")
        _check_fields(x, self._shapes, "x")
        rp = (C.c_void_p * b)(*[t.data_ptr() for t in rhs])
        xp = (C.c_void_p * b)(*[t.data_ptr() for t in x])
        reps = (GcrReport * b)()
        bufs = []
        if record_history:
            for m in range(b):
                buf = (C.c_double * (self.max_iters + 1))()
                bufs.append(buf)
                reps[m].history = C.cast(buf, C.POINTER(C.c_double))
                reps[m].history_cap = self.max_iters + 1
        rc = _lib.gcr_solve(self._h, rp, xp, reps)
        if rc < 0:
            raise self._err(rc)
        tab = np.frombuffer(reps, dtype=_REP_DTYPE)
        cols = [tab[f].tolist() for f in _REP_FIELDS]
        if record_history:
            hists = [list(bufs[m][:reps[m].history_len]) for m in range(b)]
        else:
            hists = [[] for _ in range(b)]
        return [Report(*row, h) for row, h in zip(zip(*cols), hists)]

    def si_step(self, states, olds, news, dts, orographies=None, qbars=None, absorber=0.0, g=GRAVITY,
                omega=OMEGA, radius=RADIUS):
        """One semi-implicit time step of every member (gcr_si_step).
        states / olds / news: lists (one per member) of (phi, qx, qy) float64
        CUDA tensors at n, n-1 and n+1 (news written); orographies: list of
        tensors or None; qbars: list of (qbar_x, qbar_y) or None.  Replaces
        every member's operator.  Returns the solve's list of Report."""
        b = len(self.sizes)
        if len(states) != b or len(olds) != b or len(news) != b:
            raise ValueError("one state, old state and new state per member")
        dts = list(dts) if hasattr(dts, "__len__") else [float(dts)] * b
        if not self._si_fields_ok(states, olds, news, orographies, qbars):
            self._si_fields_check(states, olds, news, orographies, qbars)
            raise ValueError("si_step: contiguous float64 CUDA tensors of the members' shapes expected")
        tab = np.zeros(b, dtype=_SI_DTYPE)
        for group, cols in ((states, ("phi", "qx", "qy")), (olds, ("phi_old", "qx_old", "qy_old")),
                            (news, ("phi_new", "qx_new", "qy_new"))):
            for i, col in enumerate(cols):
                tab[col] = [f[i].data_ptr() for f in group]
        if orographies is not None:
            tab["orography"] = [0 if o is None else o.data_ptr() for o in orographies]
        if qbars is not None:
            tab["qbar_x"] = [0 if q is None else q[0].data_ptr() for q in qbars]
            tab["qbar_y"] = [0 if q is None else q[1].data_ptr() for q in qbars]
        tab["dt"] = [float(d) for d in dts]
        tab["g"], tab["omega"], tab["radius"], tab["absorber"] = float(g), float(omega), float(radius), float(absorber)
        reps = (GcrReport * b)()
        rc = _lib.gcr_si_step(self._h, tab.ctypes.data_as(C.POINTER(GcrSiMember)), reps)
        if rc < 0:
            raise self._err(rc)
        rows = zip(*[np.frombuffer(reps, dtype=_REP_DTYPE)[f].tolist() for f in _REP_FIELDS])
        return [Report(*row, []) for row in rows]

    def _si_fields_ok(self, states, olds, news, orographies, qbars):
        """One pass of cheap attribute tests over every field of si_step."""
        if (orographies is not None and len(orographies) != len(self.sizes)) or \
                (qbars is not None and len(qbars) != len(self.sizes)):
            return False
        for m, shp in enumerate(self._shapes):
            ts = list(states[m]) + list(olds[m]) + list(news[m])
            if len(ts) != 9 or len(states[m]) != 3 or len(olds[m]) != 3:
                return False
            if orographies is not None and orographies[m] is not None:
                ts.append(orographies[m])
            if qbars is not None and qbars[m] is not None:
                if len(qbars[m]) != 2:
                    return False
                ts.extend(qbars[m])
            for t in ts:
                if not (isinstance(t, torch.Tensor) and t.dtype is _F64 and t.is_cuda and t.shape == shp
                        and t.is_contiguous()):
                    return False
        return True

    def _si_fields_check(self, states, olds, news, orographies, qbars):
        """The per-field checks of si_step, raising with the failing entry's name."""
        if orographies is not None and len(orographies) != len(self.sizes):
            raise ValueError("one orography (or None) per member")
        if qbars is not None and len(qbars) != len(self.sizes):
            raise ValueError("one (qbar_x, qbar_y) (or None) per member")
        for m, (nx, ny) in enumerate(self.sizes):
            trip = [("state", states[m]), ("old", olds[m]), ("new", news[m])]
            for what, fields in trip:
                if len(fields) != 3:
                    raise ValueError(f"{what}[{m}] must be (phi, qx, qy)")
                for t in fields:
                    _check_field(t, ny, nx, f"{what}[{m}]")
            oro = orographies[m] if orographies is not None else None
            if oro is not None:
                _check_field(oro, ny, nx, f"orography[{m}]")
            qb = qbars[m] if qbars is not None else None
            if qb is not None:
                if len(qb) != 2:
                    raise ValueError(f"qbar[{m}] must be (qbar_x, qbar_y)")
                for t in qb:
                    _check_field(t, ny, nx, f"qbar[{m}]")

    def set_kernel_timing(self, enable=True):
        rc = _lib.gcr_set_kernel_timing(self._h, 1 if enable else 0)
        if rc < 0:
            raise self._err(rc)

    def kernel_times(self):
        """{kernel name: (launches, total milliseconds)} since timing was enabled."""
        out = {}
        for k in range(K_COUNT):
            n = C.c_int64()
            ms = C.c_double()
            rc = _lib.gcr_kernel_time(self._h, k, C.byref(n), C.byref(ms))
            if rc < 0:
                raise self._err(rc)
            out[_lib.gcr_kernel_name(k).decode()] = (n.value, ms.value)
        return out

    def set_split_base(self, member, phi0):
        """Split residual base: Phi_hat = fl32(phi0) and its stored differences."""
        nx, ny = self.sizes[member]
        _check_field(phi0, ny, nx, "phi0")
        rc = _lib.gcr_set_split_base(self._h, member, phi0.data_ptr())
        if rc < 0:
            raise self._err(rc)

    def residual_split(self, member, phi_tilde, rhs, out=None):
        """r = L_SP(Phi_hat + phi_tilde) - rhs (phi_tilde float32, rhs float64)."""
        nx, ny = self.sizes[member]
        if phi_tilde.dtype != torch.float32 or not phi_tilde.is_cuda or not phi_tilde.is_contiguous() \
                or tuple(phi_tilde.shape) != (ny, nx):
            raise ValueError(f"phi_tilde must be a contiguous float32 CUDA tensor of shape {(ny, nx)}")
        _check_field(rhs, ny, nx, "rhs")
        r = torch.empty_like(rhs) if out is None else out
        rc = _lib.gcr_residual_split(self._h, member, phi_tilde.data_ptr(), rhs.data_ptr(), r.data_ptr())
        if rc < 0:
            raise self._err(rc)
        return r

    def apply_operator(self, member, x, out=None):
        nx, ny = self.sizes[member]
        _check_field(x, ny, nx, "x")
        y = torch.empty_like(x) if out is None else out
        rc = _lib.gcr_apply_operator(self._h, member, x.data_ptr(), y.data_ptr())
        if rc < 0:
            raise self._err(rc)
        return y

    def set_learned(self, params, fallback_ratio=0.5):
        """params: float32 numpy array of cnn_param_count(3) network parameters."""
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32).ravel()
        rc = _lib.gcr_set_learned(self._h, arr.ctypes.data, arr.size, float(fallback_ratio))
        if rc < 0:
            raise self._err(rc)

    def set_learned_reference(self, rel_res):
        """Reference relative residuals after iterations 1..n of the plain
        preconditioner (rel_res[0] is ignored; an empty list removes it)."""
        import numpy as np
        arr = np.ascontiguousarray(rel_res, dtype=np.float64).ravel()
        n = max(0, arr.size - 1)
        ptr = arr.ctypes.data_as(C.POINTER(C.c_double)) if arr.size else None
        rc = _lib.gcr_set_learned_reference(self._h, ptr, n)
        if rc < 0:
            raise self._err(rc)

    def learned_features(self, member, x, rhs, hi_iters=0, feat=None, target=None):
        """Features (3, ny, nx) and, with hi_iters > 0, the target (ny, nx)
        of the residual L(x) - rhs, float32 CUDA tensors; returns
        (feat, target or None, sigma)."""
        nx, ny = self.sizes[member]
        _check_field(x, ny, nx, "x")
        _check_field(rhs, ny, nx, "rhs")
        if feat is None:
            feat = torch.empty((LEARNED_CHANNELS, ny, nx), dtype=torch.float32, device=x.device)
        _check_f32(feat, (LEARNED_CHANNELS, ny, nx), "feat")
        if hi_iters > 0:
            if target is None:
                target = torch.empty((ny, nx), dtype=torch.float32, device=x.device)
            _check_f32(target, (ny, nx), "target")
        else:
            target = None
        sig = C.c_double()
        rc = _lib.gcr_learned_features(self._h, member, x.data_ptr(), rhs.data_ptr(), int(hi_iters),
                                       feat.data_ptr(), None if target is None else target.data_ptr(),
                                       C.byref(sig))
        if rc < 0:
            raise self._err(rc)
        return feat, target, sig.value

    def apply_precond(self, member, r, out=None):
        nx, ny = self.sizes[member]
        _check_field(r, ny, nx, "r")
        e = torch.empty_like(r) if out is None else out
        rc = _lib.gcr_apply_precond(self._h, member, r.data_ptr(), e.data_ptr())
        if rc < 0:
            raise self._err(rc)
        return e

    def apply_operator_form(self, member, x, out=None):
        """L(x) with the operator the solve of this precision form applies."""
        nx, ny = self.sizes[member]
        _check_field(x, ny, nx, "x")
        y = torch.empty_like(x) if out is None else out
        rc = _lib.gcr_apply_operator_form(self._h, member, x.data_ptr(), y.data_ptr())
        if rc < 0:
            raise self._err(rc)
        return y

    def apply_precond_form(self, member, r, out=None):
        """P^{-1}(r) with the preconditioner the solve of this precision form applies."""
        nx, ny = self.sizes[member]
        _check_field(r, ny, nx, "r")
        e = torch.empty_like(r) if out is None else out
        rc = _lib.gcr_apply_precond_form(self._h, member, r.data_ptr(), e.data_ptr())
        if rc < 0:
            raise self._err(rc)
        return e


STATIC_MAX_POINTS = 131072


def apply_precond_static(r, depth, dt, orography=None, richardson_iters=2, absorber=0.0, g=GRAVITY,
                         omega=OMEGA, radius=RADIUS, b_terms=True, out=None, stream=None):
    """e = P^{-1}(r) of one member without a solver and without any device
    allocation by the library (gcr_apply_precond_static): r, depth,
    orography, out are float64 CUDA tensors (ny, nx); nx * ny <=
    STATIC_MAX_POINTS."""
    ny, nx = r.shape
    _check_field(r, ny, nx, "r")
    _check_field(depth, ny, nx, "depth")
    if orography is not None:
        _check_field(orography, ny, nx, "orography")
    e = torch.empty_like(r) if out is None else out
    _check_field(e, ny, nx, "out")
    if stream is None:
        stream = torch.cuda.current_stream()
    op = GcrOperator(dt=float(dt), g=g, omega=omega, radius=radius, absorber=absorber, depth=depth.data_ptr(),
                     orography=None if orography is None else orography.data_ptr(), b_terms=1 if b_terms else 0,
                     mem_is_device=1)
    rc = _lib.gcr_apply_precond_static(nx, ny, C.addressof(op), int(richardson_iters), r.data_ptr(),
                                       e.data_ptr(), C.c_void_p(stream.cuda_stream))
    if rc < 0:
        raise GcrError(rc, _lib.gcr_last_error(None).decode())
    return e


def _check_f32(t, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float32 tensor of shape {tuple(shape)}")


def cnn_param_count(c_in=LEARNED_CHANNELS) -> int:
    return int(_lib.cnn_param_count(int(c_in)))


class Network:
    """The learned preconditioner's convolution network on the GPU (forward,
    gradients, Adam training); tensors are float32 CUDA tensors."""

    def __init__(self, nx, ny, max_batch, c_in=LEARNED_CHANNELS, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.nx, self.ny, self.max_batch, self.c_in = int(nx), int(ny), int(max_batch), int(c_in)
        h = C.c_void_p()
        rc = _lib.cnn_create(self.nx, self.ny, self.max_batch, self.c_in, C.c_void_p(stream.cuda_stream),
                             C.byref(h))
        if rc < 0:
            raise GcrError(rc, _lib.cnn_last_error(None).decode())
        self._h = h
        self.nparams = cnn_param_count(self.c_in)

    def _err(self, rc):
        return GcrError(rc, _lib.cnn_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32).ravel()
        rc = _lib.cnn_set_params(self._h, arr.ctypes.data, arr.size)
        if rc < 0:
            raise self._err(rc)

    def get_params(self):
        import numpy as np
        arr = np.empty(self.nparams, dtype=np.float32)
        rc = _lib.cnn_get_params(self._h, arr.ctypes.data, arr.size)
        if rc < 0:
            raise self._err(rc)
        return arr

    def _batch(self, inp):
        _check_f32(inp, (inp.shape[0], self.c_in, self.ny, self.nx), "input")
        return int(inp.shape[0])

    def forward(self, inp, out=None):
        b = self._batch(inp)
        if out is None:
            out = torch.empty((b, self.ny, self.nx), dtype=torch.float32, device=inp.device)
        _check_f32(out, (b, self.ny, self.nx), "out")
        rc = _lib.cnn_forward(self._h, b, inp.data_ptr(), out.data_ptr())
        if rc < 0:
            raise self._err(rc)
        return out

    def gradients(self, inp, dy):
        import numpy as np
        b = self._batch(inp)
        _check_f32(dy, (b, self.ny, self.nx), "dy")
        g = np.empty(self.nparams, dtype=np.float32)
        rc = _lib.cnn_gradients(self._h, b, inp.data_ptr(), dy.data_ptr(), g.ctypes.data)
        if rc < 0:
            raise self._err(rc)
        return g

    def train_step(self, inp, target, lr=1e-3):
        b = self._batch(inp)
        _check_f32(target, (b, self.ny, self.nx), "target")
        loss = C.c_double()
        rc = _lib.cnn_train_step(self._h, b, inp.data_ptr(), target.data_ptr(), float(lr), C.byref(loss))
        if rc < 0:
            raise self._err(rc)
        return loss.value
