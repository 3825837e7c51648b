"""ctypes binding of libcgs.so (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libcgs.so")

FP64, FP32, BF16 = 0, 1, 2
DTYPE_F64, DTYPE_F32 = 0, 1            # CGS_DTYPE_*
MEM_HOST_COPY, MEM_DEVICE_BORROW = 0, 1  # CGS_MEM_*
RUNNING, SOLVED, MAX_ITERS, INFEASIBLE, UNBOUNDED, NUMERICAL = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {RUNNING: "running", SOLVED: "solved", MAX_ITERS: "max_iters",
                INFEASIBLE: "infeasible", UNBOUNDED: "unbounded", NUMERICAL: "numerical"}
ERRORS = {-1: "EINVAL", -2: "EDIM", -3: "ECONE", -4: "ENOMEM", -5: "EHIP", -6: "EBUSY",
          -7: "ESTATE", -8: "ENOTFOUND"}


class CgsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Settings(C.Structure):
    _fields_ = [
        ("eps", C.c_double), ("alpha", C.c_double), ("max_iters", C.c_int32),
        ("check_every", C.c_int32), ("precision", C.c_int32), ("cg_max_iters", C.c_int32),
        ("cg_tol", C.c_double), ("cg_rate", C.c_double), ("cg_floor", C.c_double),
        ("setup_tol", C.c_double), ("setup_max_iters", C.c_int32), ("use_graph", C.c_int32),
        ("bf16_phase1_digits", C.c_int32), ("cg_adaptive", C.c_int32),
        ("fused_max", C.c_int32), ("conv_mfma", C.c_int32), ("normalize", C.c_int32),
        ("fused_lone_max", C.c_int32), ("vec_tile", C.c_int32), ("intervals_per_sync", C.c_int32),
    ]

    @classmethod
    def make(cls, **kw) -> "Settings":
        s = cls()
        lib().cgs_settings_default(C.byref(s))
        for k, v in kw.items():
            if not hasattr(s, k):
                raise KeyError(k)
            setattr(s, k, v)
        return s


class Info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iters", C.c_int32), ("cg_iters", C.c_int64),
        ("pobj", C.c_double), ("dobj", C.c_double), ("res_pri", C.c_double),
        ("res_dual", C.c_double), ("gap", C.c_double), ("tau", C.c_double),
        ("kappa", C.c_double), ("setup_s", C.c_double), ("solve_s", C.c_double),
        ("cert_precision", C.c_int32), ("reserved_", C.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


_LIB = None
_P = C.c_void_p
_I64 = C.c_int64
_D = C.c_double
_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)

_SIGS = {
    "cgs_last_error": (C.c_char_p, []),
    "cgs_version": (C.c_char_p, []),
    "cgs_op_create": (C.c_int, [_I64, _I64, C.POINTER(_P)]),
    "cgs_op_add_identity": (C.c_int, [_P, _I64, _I64, _I64, _D]),
    "cgs_op_add_conv": (C.c_int, [_P, _I64, _I64, _DP, _I64, _I64, _D]),
    "cgs_op_add_dense": (C.c_int, [_P, _I64, _I64, _I64, _I64, _DP, _I64, _D]),
    "cgs_op_add_dense_ex": (C.c_int, [_P, _I64, _I64, _I64, _I64, _P, _I64, C.c_int32, C.c_int32, _D]),
    "cgs_op_info": (C.c_int, [_P, _I64P, _I64P, _I64P]),
    "cgs_op_equilibrate": (C.c_int, [_P, C.c_int64, _I64P, C.c_int64, C.c_int32, _DP, _DP, _DP, _DP,
                                     _DP]),
    "cgs_op_destroy": (None, [_P]),
    "cgs_settings_default": (None, [C.POINTER(Settings)]),
    "cgs_workspace_bytes": (C.c_int, [_P, _I64, _I64P, _I64, C.POINTER(Settings), _I64,
                                      C.POINTER(C.c_size_t)]),
    "cgs_solver_create": (C.c_int, [_P, _I64, _I64P, _I64, C.POINTER(Settings), _I64, _P,
                                    C.c_size_t, _P, C.POINTER(_P)]),
    "cgs_solver_set_data": (C.c_int, [_P, _I64, _DP, _DP]),
    "cgs_solver_reset": (C.c_int, [_P, _I64]),
    "cgs_solve": (C.c_int, [_P, C.POINTER(Info)]),
    "cgs_solver_iterate": (C.c_int, [_P, C.c_int32]),
    "cgs_solver_rounds": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "cgs_solver_get_solution": (C.c_int, [_P, _I64, _DP, _DP, _DP]),
    "cgs_solver_get_state": (C.c_int, [_P, _I64, _DP, _DP, _DP, _DP]),
    "cgs_solver_set_state": (C.c_int, [_P, _I64, _DP, _DP, _DP, _DP]),
    "cgs_solver_residuals": (C.c_int, [_P, C.POINTER(Info)]),
    "cgs_solver_apply": (C.c_int, [_P, C.c_int32, _DP, _DP]),
    "cgs_solver_normal_solve": (C.c_int, [_P, _DP, _DP, _DP, _D, C.c_int32,
                                          C.POINTER(C.c_int32)]),
    "cgs_solver_kernel_time": (C.c_int, [_P, C.c_int32, C.c_int32, _DP]),
    "cgs_solver_autotune": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "cgs_solver_destroy": (None, [_P]),
    "cgs_solve_noalloc": (C.c_int, [_P, _I64, _I64P, _I64, C.POINTER(Settings), _DP, _DP, _P, _DP, _DP,
                                    _DP, C.POINTER(Info)]),
    "cgs_server_request_bytes": (C.c_int, [_P, _I64, _I64P, _I64, C.c_int32,
                                           C.POINTER(C.c_size_t)]),
    "cgs_server_create": (C.c_int, [_I64, C.POINTER(Settings), _P, C.c_size_t, _P,
                                    C.POINTER(_P)]),
    "cgs_server_submit": (C.c_int, [_P, _P, _I64, _I64P, _I64, _DP, _DP, _I64P]),
    "cgs_server_step": (C.c_int, [_P, C.c_int32, _I64P]),
    "cgs_server_poll": (C.c_int, [_P, _I64, C.POINTER(C.c_int32)]),
    "cgs_server_finished": (C.c_int, [_P, _I64P, C.c_int64, _I64P]),
    "cgs_server_fetch": (C.c_int, [_P, _I64, _DP, _DP, _DP, C.POINTER(Info)]),
    "cgs_server_cancel": (C.c_int, [_P, _I64]),
    "cgs_server_usage": (C.c_int, [_P, _I64P, C.POINTER(C.c_size_t)]),
    "cgs_server_destroy": (None, [_P]),
}


def lib() -> C.CDLL:
    """Load libcgs.so (raises when it has not been built: there is no fallback)."""
    global _LIB
    if _LIB is None:
        # PyTorch brings its own HIP runtime (same soname, libamdhip64.so.7).  It
        # must be the one loaded, before libcgs.so, so that the process holds a
        # single HIP/HSA runtime shared by torch's allocator and this library.
        import torch  # noqa: F401
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing; build it with "
                              "`python -m paper_1609_03488_amd.build_lib`")
        L = C.CDLL(library_path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(rc: int) -> None:
    if rc != 0:
        raise CgsError(rc, lib().cgs_last_error().decode())


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a, n: Optional[int] = None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.shape != (n,):
        raise ValueError(f"expected {n} entries, got shape {a.shape}")
    return a


def _q(q: Sequence[int]) -> Tuple[np.ndarray, int]:
    arr = np.ascontiguousarray(np.asarray(list(q), dtype=np.int64))
    return arr, int(arr.shape[0])


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Operator:
    """Structured operator (sum of placed identity / convolution / dense blocks)."""

    def __init__(self, m: int, n: int):
        h = _P()
        _check(lib().cgs_op_create(int(m), int(n), C.byref(h)))
        self._h = h
        self.m, self.n = int(m), int(n)
        self.kinds: List[str] = []
        self._borrowed: list = []   # device tensors the operator reads in place

    def add_identity(self, row0: int, col0: int, length: int, scale: float = 1.0) -> "Operator":
        _check(lib().cgs_op_add_identity(self._h, row0, col0, length, float(scale)))
        self.kinds.append("identity")
        return self

    def add_conv(self, row0: int, col0: int, taps, n_in: int, scale: float = 1.0) -> "Operator":
        t = _f64(taps)
        _check(lib().cgs_op_add_conv(self._h, row0, col0, _dp(t), t.shape[0], n_in, float(scale)))
        self.kinds.append("conv")
        return self

    def add_dense(self, row0: int, col0: int, a, scale: float = 1.0) -> "Operator":
        """Dense block.  ``a``: a 2-D array (FP64 or FP32 numpy data is copied),
        or a 2-D torch tensor: on the GPU (FP32 or FP64, unit column stride) it
        is borrowed -- read in place on the device, never copied to the host --
        and this operator keeps a reference to it; the caller must not change
        it while solvers are being created from the operator."""
        try:
            import torch
            is_tensor = isinstance(a, torch.Tensor)
        except ImportError:   # pragma: no cover
            is_tensor = False
        if is_tensor and a.is_cuda:
            if a.dim() != 2 or a.dtype not in (torch.float32, torch.float64) or a.stride(1) != 1:
                raise ValueError("a borrowed dense block must be a 2-D FP32/FP64 tensor with unit column stride")
            dt = DTYPE_F32 if a.dtype == torch.float32 else DTYPE_F64
            _check(lib().cgs_op_add_dense_ex(self._h, row0, col0, a.shape[0], a.shape[1], a.data_ptr(),
                                             a.stride(0), dt, MEM_DEVICE_BORROW, float(scale)))
            self._borrowed.append(a)
            self.kinds.append("dense")
            return self
        if is_tensor:
            a = a.numpy()
        a = np.asarray(a)
        if a.ndim != 2:
            raise ValueError("dense block must be 2-D")
        if a.dtype == np.float32:
            a = np.ascontiguousarray(a)
            _check(lib().cgs_op_add_dense_ex(self._h, row0, col0, a.shape[0], a.shape[1], a.ctypes.data,
                                             a.shape[1], DTYPE_F32, MEM_HOST_COPY, float(scale)))
        else:
            a = np.ascontiguousarray(a, dtype=np.float64)
            _check(lib().cgs_op_add_dense(self._h, row0, col0, a.shape[0], a.shape[1], _dp(a),
                                          a.shape[1], float(scale)))
        self.kinds.append("dense")
        return self

    def equilibrate(self, l: int, q: Sequence[int], b=None, c=None, level: int = 2):
        """Row / column scalings (D, E) a solver with normalize = level uses for
        this operator and cone, and (sigma_b, sigma_c) when b and c are given."""
        qa = np.asarray(list(q), dtype=np.int64)
        d, e = np.empty(self.m), np.empty(self.n)
        sig = np.empty(2)
        bb = None if b is None else _f64(b, self.m)
        cc = None if c is None else _f64(c, self.n)
        _check(lib().cgs_op_equilibrate(self._h, int(l), qa.ctypes.data_as(_I64P), len(qa), int(level),
                                        None if bb is None else _dp(bb),
                                        None if cc is None else _dp(cc), _dp(d), _dp(e), _dp(sig)))
        return d, e, ((float(sig[0]), float(sig[1])) if bb is not None else None)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _LIB is not None:
            _LIB.cgs_op_destroy(h)
            self._h = None


def _workspace(nbytes: int, device):
    import torch
    buf = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off


class Solver:
    """One problem, or a batch of problems sharing the operator and cone."""

    def __init__(self, op: Operator, l: int, q: Sequence[int], settings: Optional[Settings] = None,
                 batch: int = 1, stream=None, device: str = "cuda"):
        self.op = op
        self.settings = settings if settings is not None else Settings.make()
        self.l = int(l)
        self.q, nq = _q(q)
        self.batch = int(batch)
        nb = C.c_size_t()
        _check(lib().cgs_workspace_bytes(op._h, self.l, self.q.ctypes.data_as(_I64P), nq,
                                         C.byref(self.settings), self.batch, C.byref(nb)))
        self.workspace_bytes = int(nb.value)
        self._buf, ptr = _workspace(self.workspace_bytes, device)
        self._stream = stream
        h = _P()
        _check(lib().cgs_solver_create(op._h, self.l, self.q.ctypes.data_as(_I64P), nq,
                                       C.byref(self.settings), self.batch, ptr,
                                       self.workspace_bytes, _stream_handle(stream), C.byref(h)))
        self._h = h
        self.n, self.m = op.n, op.m

    def set_data(self, inst: int, b, c) -> None:
        b = _f64(b, self.m)
        c = _f64(c, self.n)
        _check(lib().cgs_solver_set_data(self._h, inst, _dp(b), _dp(c)))

    def reset(self, inst: int = -1) -> None:
        """Restart from u = v = (0, 0, 1) keeping b and c on the device."""
        _check(lib().cgs_solver_reset(self._h, int(inst)))

    def kernel_time(self, kernel: int, reps: int = 20) -> float:
        """Mean device milliseconds per launch (HIP events); kernel ids as in cgs.h."""
        ms = C.c_double()
        _check(lib().cgs_solver_kernel_time(self._h, int(kernel), int(reps), C.byref(ms)))
        return float(ms.value)

    def autotune(self, reps: int = 10) -> dict:
        """Pick the fastest convolution engine, GEMM split and vector tile for
        this solver (timed on whole ADMM steps when every instance has data;
        the instances restart afterwards)."""
        ch = (C.c_int32 * 4)()
        _check(lib().cgs_solver_autotune(self._h, int(reps), ch))
        return {"conv_mfma": int(ch[0]), "gemm_target_wgs": int(ch[1]), "vec_tile": int(ch[2])}

    def solve(self) -> List[dict]:
        infos = (Info * self.batch)()
        _check(lib().cgs_solve(self._h, infos))
        return [i.as_dict() for i in infos]

    def iterate(self, iters: int) -> None:
        _check(lib().cgs_solver_iterate(self._h, int(iters)))

    def rounds(self):
        """(check intervals run, intervals run again with more CG launches)."""
        r, rr = C.c_int64(), C.c_int64()
        _check(lib().cgs_solver_rounds(self._h, C.byref(r), C.byref(rr)))
        return int(r.value), int(rr.value)

    def solution(self, inst: int = 0):
        x, y, s = np.empty(self.n), np.empty(self.m), np.empty(self.m)
        _check(lib().cgs_solver_get_solution(self._h, inst, _dp(x), _dp(y), _dp(s)))
        return x, y, s

    def state(self, inst: int = 0):
        """Raw embedding state (u_x, u_y, tau, v_s, kappa) of the problem the
        iteration runs on (the equilibrated one unless normalize = 0)."""
        ux, uy, vs, sc = np.empty(self.n), np.empty(self.m), np.empty(self.m), np.empty(2)
        _check(lib().cgs_solver_get_state(self._h, inst, _dp(ux), _dp(uy), _dp(vs), _dp(sc)))
        return ux, uy, float(sc[0]), vs, float(sc[1])

    def set_state(self, inst: int, ux, uy, tau: float, vs, kappa: float) -> None:
        ux, uy, vs = _f64(ux, self.n), _f64(uy, self.m), _f64(vs, self.m)
        sc = np.array([tau, kappa], dtype=np.float64)
        _check(lib().cgs_solver_set_state(self._h, inst, _dp(ux), _dp(uy), _dp(vs), _dp(sc)))

    def residuals(self) -> List[dict]:
        infos = (Info * self.batch)()
        _check(lib().cgs_solver_residuals(self._h, infos))
        return [i.as_dict() for i in infos]

    def apply(self, v, transpose: bool = False) -> np.ndarray:
        """A v (or A^T v) on the device, A as the iteration sees it (D A E when
        normalize = 2)."""
        v = _f64(v, self.m if transpose else self.n)
        out = np.empty(self.n if transpose else self.m)
        _check(lib().cgs_solver_apply(self._h, 1 if transpose else 0, _dp(v), _dp(out)))
        return out

    def normal_solve(self, rhs, z0=None, tol: float = 1e-8, max_iters: int = 1000):
        rhs = _f64(rhs, self.n)
        z0 = None if z0 is None else _f64(z0, self.n)
        z = np.empty(self.n)
        it = C.c_int32()
        _check(lib().cgs_solver_normal_solve(self._h, _dp(rhs), _dp(z0), _dp(z), float(tol),
                                             int(max_iters), C.byref(it)))
        return z, int(it.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().cgs_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 32 << 20   # CGS_NOALLOC_SCRATCH_BYTES of cgs.h


def solve_noalloc(op: Operator, l: int, q: Sequence[int], b, c, settings: Optional[Settings] = None,
                  stream=None):
    """One solve through cgs_solve_noalloc (no memory allocated by the library:
    its workspace is the library's fixed device array).  Returns x, y, s, info."""
    st = settings if settings is not None else Settings.make()
    qa, nq = _q(q)
    b = _f64(b, op.m)
    c = _f64(c, op.n)
    x, y, s = np.empty(op.n), np.empty(op.m), np.empty(op.m)
    info = Info()
    _check(lib().cgs_solve_noalloc(op._h, int(l), qa.ctypes.data_as(_I64P), nq, C.byref(st), _dp(b), _dp(c),
                                   _stream_handle(stream), _dp(x), _dp(y), _dp(s), C.byref(info)))
    return x, y, s, info.as_dict()


class Server:
    """Continuous batching of independent problems (ticketed requests)."""

    def __init__(self, workspace_bytes: int, max_slots: int, settings: Optional[Settings] = None,
                 stream=None, device: str = "cuda"):
        self.settings = settings if settings is not None else Settings.make()
        self.workspace_bytes = int(workspace_bytes)
        self._buf, ptr = _workspace(self.workspace_bytes, device)
        h = _P()
        _check(lib().cgs_server_create(int(max_slots), C.byref(self.settings), ptr,
                                       self.workspace_bytes, _stream_handle(stream), C.byref(h)))
        self._h = h
        self._shapes = {}

    @staticmethod
    def request_bytes(op: Operator, l: int, q: Sequence[int], precision: int = FP32) -> int:
        qa, nq = _q(q)
        nb = C.c_size_t()
        _check(lib().cgs_server_request_bytes(op._h, int(l), qa.ctypes.data_as(_I64P), nq,
                                              int(precision), C.byref(nb)))
        return int(nb.value)

    def submit(self, op: Operator, l: int, q: Sequence[int], b, c) -> Optional[int]:
        """Ticket, or None when no slot / memory is free (CGS_EBUSY)."""
        qa, nq = _q(q)
        b = _f64(b, op.m)
        c = _f64(c, op.n)
        t = C.c_int64()
        rc = lib().cgs_server_submit(self._h, op._h, int(l), qa.ctypes.data_as(_I64P), nq,
                                     _dp(b), _dp(c), C.byref(t))
        if rc == -6:
            return None
        _check(rc)
        self._shapes[int(t.value)] = (op.n, op.m)
        return int(t.value)

    def step(self, steps: int) -> int:
        n = C.c_int64()
        _check(lib().cgs_server_step(self._h, int(steps), C.byref(n)))
        return int(n.value)

    def poll(self, ticket: int) -> int:
        s = C.c_int32()
        _check(lib().cgs_server_poll(self._h, int(ticket), C.byref(s)))
        return int(s.value)

    def finished(self) -> List[int]:
        """Tickets that have finished and await fetch (admission order)."""
        n = C.c_int64()
        _check(lib().cgs_server_finished(self._h, None, 0, C.byref(n)))
        if n.value == 0:
            return []
        buf = (C.c_int64 * n.value)()
        _check(lib().cgs_server_finished(self._h, buf, n.value, C.byref(n)))
        return list(buf)

    def fetch(self, ticket: int):
        n, m = self._shapes.pop(int(ticket))
        x, y, s = np.empty(n), np.empty(m), np.empty(m)
        info = Info()
        _check(lib().cgs_server_fetch(self._h, int(ticket), _dp(x), _dp(y), _dp(s),
                                      C.byref(info)))
        return x, y, s, info.as_dict()

    def cancel(self, ticket: int) -> None:
        self._shapes.pop(int(ticket), None)
        _check(lib().cgs_server_cancel(self._h, int(ticket)))

    def usage(self):
        k = C.c_int64()
        f = C.c_size_t()
        _check(lib().cgs_server_usage(self._h, C.byref(k), C.byref(f)))
        return int(k.value), int(f.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().cgs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
