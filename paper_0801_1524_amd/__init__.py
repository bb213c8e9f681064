"""bfsft: butterfly sparse Fourier transform on MI355X (gfx950).

Thin ctypes binding over the C ABI in ``include/bfsft.h``: every step of the
transform runs in the HIP library ``libbfsft.so`` built from ``csrc/``;
this module only marshals torch device tensors and the current HIP stream.
There is no CPU fallback: importing the binding without the built library,
or using it without a GPU, raises.

    u_i = sum_j exp(2 pi i x_i . k_j / N) f_j        (Section 1, eq. 1)

Usage (points as [n][d] float64 arrays in [0, N]^d, numpy or torch; sources
complex128; results are complex128 tensors on the current GPU)::

    import paper_0801_1524_amd as bf
    with bf.Plan(2, N, 9, x, k, "mixed") as plan:   # trees, tables, tuning
        u = plan.execute(f)                          # steps 2-4 of Section 2.2
        v = plan.execute_adjoint(g)                  # sum_i exp(-2 pi i x_i . k_j / N) g_i
    B = bf.BatchedPlan([(N1, x1, k1), (N2, x2, k2)], 2, 7, "mixed")
    u_packed = B.execute(f_packed)                   # one graph for all transforms
    B.close()
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfsft.so")

OK, EINVAL, EDOMAIN, ENOMEM, EDEVICE = 0, -1, -2, -3, -4
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16x2": 2, "bf16x3": 3, "mixed": 4}
MAX_LEVELS = 32

_lib = None


class BfsftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bfsft status {status}: {message}")
        self.status = status


class Info(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int), ("p", ctypes.c_int), ("precision", ctypes.c_int), ("levels", ctypes.c_int),
        ("N", ctypes.c_int64), ("nx", ctypes.c_int64), ("nk", ctypes.c_int64),
        ("rho", ctypes.c_double),
        ("x_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("k_boxes", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("pairs", ctypes.c_int64 * (MAX_LEVELS + 1)),
        ("sweep_bytes", ctypes.c_double), ("sweep_flops", ctypes.c_double),
        ("device_bytes", ctypes.c_int64), ("transforms", ctypes.c_int64),
        ("lds_kb", ctypes.c_int), ("wg_per_cu", ctypes.c_int),
        ("level_kernel", ctypes.c_int * MAX_LEVELS), ("level_lds_kb", ctypes.c_int * MAX_LEVELS),
        ("start_level", ctypes.c_int),
        ("start_kernel", ctypes.c_int),
        ("start_tables", ctypes.c_int),
    ]


class Problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("x", ctypes.c_void_p), ("nx", ctypes.c_int64),
                ("k", ctypes.c_void_p), ("nk", ctypes.c_int64)]


def lib():
    """Load libbfsft.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_0801_1524_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.bfsft_plan_create.argtypes = [PP, I, I64, I, I, P, I64, P, I64, P]
    L.bfsft_plan_create.restype = I
    L.bfsft_execute.argtypes = [P, P, P]
    L.bfsft_execute.restype = I
    L.bfsft_execute_noalloc.argtypes = [P, P, P]
    L.bfsft_execute_noalloc.restype = I
    L.bfsft_execute_adjoint.argtypes = [P, P, P]
    L.bfsft_execute_adjoint.restype = I
    L.bfsft_execute_probe.argtypes = [P, P, P, I, P]
    L.bfsft_execute_probe.restype = I
    L.bfsft_destroy.argtypes = [P]
    L.bfsft_destroy.restype = None
    L.bfsft_strerror.argtypes = [I]
    L.bfsft_strerror.restype = ctypes.c_char_p
    L.bfsft_last_error.argtypes = []
    L.bfsft_last_error.restype = ctypes.c_char_p
    L.bfsft_plan_info.argtypes = [P, ctypes.POINTER(Info)]
    L.bfsft_plan_info.restype = I
    L.bfsft_plan_tables.argtypes = [P, P, P, P]
    L.bfsft_plan_tables.restype = I
    L.bfsft_plan_boxes.argtypes = [P, I, I, P]
    L.bfsft_plan_boxes.restype = I
    L.bfsft_plan_create_batched.argtypes = [PP, I, ctypes.POINTER(Problem), I, I, I, P]
    L.bfsft_plan_create_batched.restype = I
    L.bfsft_execute_batched.argtypes = [P, P, P]
    L.bfsft_execute_batched.restype = I
    L.bfsft_execute_batched_serial.argtypes = [P, P, P]
    L.bfsft_execute_batched_serial.restype = I
    L.bfsft_timing_begin.argtypes = [P, I]
    L.bfsft_timing_begin.restype = I
    L.bfsft_timing_end.argtypes = [P, ctypes.POINTER(ctypes.c_double), I]
    L.bfsft_timing_end.restype = I
    L.bfsft_copy_rate.argtypes = [I, I64, I, P, ctypes.POINTER(ctypes.c_double)]
    L.bfsft_copy_rate.restype = I
    L.bfsft_mfma_f64_rate.argtypes = [I, I, P, ctypes.POINTER(ctypes.c_double)]
    L.bfsft_mfma_f64_rate.restype = I
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        L = lib()
        raise BfsftError(rc, f"{L.bfsft_strerror(rc).decode()}: {L.bfsft_last_error().decode()}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("bfsft needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _dev_points(a, d, torch):
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    a = a.to(device="cuda", dtype=torch.float64).contiguous().reshape(-1, d)
    return a


def _dev_complex(a, torch):
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
    return a.to(device="cuda", dtype=torch.complex128).contiguous().reshape(-1)


def _sources(a, n, torch, what):
    """Device complex128 copy (or view) of a source vector, of exactly n values."""
    t = _dev_complex(a, torch)
    if t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} values, the plan expects {n}")
    return t


def _output(out, n, torch, what):
    """A caller's output tensor, checked, or a new one: complex128, contiguous,
    on the current GPU, with at least n values (the kernels write n)."""
    if out is None:
        return torch.empty(n, dtype=torch.complex128, device="cuda")
    if not isinstance(out, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if out.dtype != torch.complex128 or not out.is_cuda or not out.is_contiguous():
        raise ValueError(f"{what} must be a contiguous complex128 tensor on the GPU")
    if out.device.index != torch.cuda.current_device():
        raise ValueError(f"{what} is on another GPU than the current one")
    if out.numel() < n:
        raise ValueError(f"{what} has {out.numel()} values, the plan writes {n}")
    return out


class _Ordered:
    """Runs a call on the plan's stream in order with the caller's current
    stream: the plan stream waits for the current one (the inputs were made
    there), the current one waits for the plan stream afterwards (the
    outputs are read there), and tensors used on both are recorded on the
    plan stream so the caching allocator does not reuse them early."""

    def __init__(self, torch, plan_stream, tensors):
        self.torch, self.ps, self.tensors = torch, plan_stream, tensors

    def __enter__(self):
        self.cur = self.torch.cuda.current_stream()
        self.other = self.cur.cuda_stream != self.ps.cuda_stream
        if self.other:
            self.ps.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        if self.other:
            self.cur.wait_stream(self.ps)
            for t in self.tensors:
                if t is not None and t.numel():
                    t.record_stream(self.ps)


def _info_dict(info: Info) -> dict:
    L = info.levels
    return {
        "d": info.d, "p": info.p, "precision": info.precision, "levels": L,
        "N": info.N, "nx": info.nx, "nk": info.nk, "rho": info.rho,
        "x_boxes": list(info.x_boxes[:L + 1]), "k_boxes": list(info.k_boxes[:L + 1]),
        "pairs": list(info.pairs[:L + 1]),
        "sweep_bytes": info.sweep_bytes, "sweep_flops": info.sweep_flops,
        "device_bytes": info.device_bytes, "transforms": info.transforms,
        "lds_kb": info.lds_kb, "wg_per_cu": info.wg_per_cu,
        "level_kernel": list(info.level_kernel[:L]), "level_lds_kb": list(info.level_lds_kb[:L]),
        "start_level": info.start_level,
        "start_kernel": info.start_kernel,
        "start_tables": info.start_tables,
    }


class Plan:
    """A planned transform for fixed targets x (nx, d) and sources k (nk, d).

    ``precision``: "fp64" (FP64 state and arithmetic), "mixed" (FP32 state in
    HBM, FP64 arithmetic) or "fp32" (FP32 state and arithmetic).  Every
    execute runs on the stream that was current at creation, ordered with
    the caller's current stream.
    """

    def __init__(self, d, N, p, x, k, precision="fp64"):
        torch = _torch()
        self._L = lib()
        self.d, self.N, self.p = int(d), int(N), int(p)
        self.precision = precision
        xd = _dev_points(x, d, torch)
        kd = _dev_points(k, d, torch)
        self.nx, self.nk = int(xd.shape[0]), int(kd.shape[0])
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        # every execute runs on this stream, ordered with the caller's current one
        self._stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self._L.bfsft_plan_create(ctypes.byref(h), self.d, self.N, self.p, PRECISIONS[precision],
                                       ctypes.c_void_p(xd.data_ptr() if self.nx else 0), self.nx,
                                       ctypes.c_void_p(kd.data_ptr() if self.nk else 0), self.nk,
                                       ctypes.c_void_p(self._stream.cuda_stream))
        _check(rc)
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.bfsft_destroy(h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def execute(self, f, out=None):
        """u (complex128 device tensor, original target order) for sources f."""
        torch = _torch()
        fd = _sources(f, self.nk, torch, "f")
        u = _output(out, self.nx, torch, "out")
        with _Ordered(torch, self._stream, (fd, u)):
            _check(self._L.bfsft_execute(self._h, ctypes.c_void_p(fd.data_ptr() if self.nk else 0),
                                         ctypes.c_void_p(u.data_ptr() if self.nx else 0)))
        return u

    def execute_noalloc(self, f, out):
        """As execute, through bfsft_execute_noalloc (state in the library's
        static scratch; out must be given: nothing is allocated)."""
        torch = _torch()
        fd = _sources(f, self.nk, torch, "f")
        u = _output(out, self.nx, torch, "out")
        with _Ordered(torch, self._stream, (fd, u)):
            _check(self._L.bfsft_execute_noalloc(self._h, ctypes.c_void_p(fd.data_ptr() if self.nk else 0),
                                                 ctypes.c_void_p(u.data_ptr() if self.nx else 0)))
        return u

    def execute_adjoint(self, g, out=None):
        """v_j = sum_i exp(-2 pi i x_i . k_j / N) g_i (complex128 device tensor,
        original source order) for values g at the targets."""
        torch = _torch()
        gd = _sources(g, self.nx, torch, "g")
        v = _output(out, self.nk, torch, "out")
        with _Ordered(torch, self._stream, (gd, v)):
            _check(self._L.bfsft_execute_adjoint(self._h, ctypes.c_void_p(gd.data_ptr() if self.nx else 0),
                                                 ctypes.c_void_p(v.data_ptr() if self.nk else 0)))
        return v

    def execute_probe(self, f, level):
        """(u, pot): pot = check potentials u^{AB} of T_K level `level`,
        shape (x_boxes[L-level], k_boxes[level], p^d), boxes as in boxes()."""
        torch = _torch()
        info = self.info()
        L = info["levels"]
        nA, nB = info["x_boxes"][L - level], info["k_boxes"][level]
        fd = _sources(f, self.nk, torch, "f")
        u = torch.empty(self.nx, dtype=torch.complex128, device="cuda")
        pot = torch.empty((nA, nB, self.p ** self.d), dtype=torch.complex128, device="cuda")
        with _Ordered(torch, self._stream, (fd, u, pot)):
            _check(self._L.bfsft_execute_probe(self._h, ctypes.c_void_p(fd.data_ptr()),
                                               ctypes.c_void_p(u.data_ptr()), int(level),
                                               ctypes.c_void_p(pot.data_ptr())))
        return u, pot

    def info(self) -> dict:
        info = Info()
        _check(self._L.bfsft_plan_info(self._h, ctypes.byref(info)))
        return _info_dict(info)

    def timing_begin(self, max_execs: int):
        """Arm per-launch HIP events for the next max_execs executes."""
        _check(self._L.bfsft_timing_begin(self._h, int(max_execs)))

    def timing_end(self) -> dict:
        """Wait for the armed events; per-phase milliseconds summed over executes."""
        L = self.info()["levels"]
        out = (ctypes.c_double * (3 + L))()
        _check(self._L.bfsft_timing_end(self._h, out, 3 + L))
        return {"executes": int(out[0]), "leaf_ms": out[1], "final_ms": out[2],
                "translate_ms": [out[3 + l] for l in range(L)]}

    def tables(self):
        """(R, G, E): the device's interpolation tables (bfsft_plan_tables):
        R (2, p, p) real, G (2 s, 2 t, p) complex, E (p,) complex."""
        p = self.p
        R = np.zeros((2, p, p), dtype=np.float64)
        G = np.zeros((2, 2, p), dtype=np.complex128)
        E = np.zeros(p, dtype=np.complex128)
        _check(self._L.bfsft_plan_tables(self._h, R.ctypes.data_as(ctypes.c_void_p),
                                         G.ctypes.data_as(ctypes.c_void_p), E.ctypes.data_as(ctypes.c_void_p)))
        return R, G, E

    def boxes(self, side: str, m: int) -> np.ndarray:
        info = self.info()
        n = (info["x_boxes"] if side == "x" else info["k_boxes"])[m]
        out = np.zeros((n, self.d), dtype=np.int64)
        _check(self._L.bfsft_plan_boxes(self._h, 0 if side == "x" else 1, int(m),
                                        out.ctypes.data_as(ctypes.c_void_p)))
        return out


class BatchedPlan:
    """Many independent 2D/3D transforms of uneven N, executed as one graph
    launch of persistent per-step kernels.  ``problems`` is a list of
    (N, x, k) triples; sources and outputs are packed in problem order."""

    def __init__(self, problems, d, p, precision="mixed"):
        torch = _torch()
        self._L = lib()
        self.d, self.p, self.precision = int(d), int(p), precision
        self._keep = []
        arr = (Problem * len(problems))()
        self.nx_list, self.nk_list = [], []
        for i, (N, x, k) in enumerate(problems):
            xd = _dev_points(x, d, torch)
            kd = _dev_points(k, d, torch)
            self._keep += [xd, kd]
            arr[i].N = int(N)
            arr[i].x = xd.data_ptr()
            arr[i].nx = xd.shape[0]
            arr[i].k = kd.data_ptr()
            arr[i].nk = kd.shape[0]
            self.nx_list.append(int(xd.shape[0]))
            self.nk_list.append(int(kd.shape[0]))
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self._stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self._L.bfsft_plan_create_batched(ctypes.byref(h), len(problems), arr, self.d, self.p,
                                               PRECISIONS[precision], ctypes.c_void_p(self._stream.cuda_stream))
        self._keep = []
        _check(rc)
        self._h = h
        self.nx = sum(self.nx_list)
        self.nk = sum(self.nk_list)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.bfsft_destroy(h)
            self._h = None

    __del__ = close

    def execute(self, f_packed, out=None, serial=False):
        torch = _torch()
        fd = _sources(f_packed, self.nk, torch, "f_packed")
        u = _output(out, self.nx, torch, "out")
        fn = self._L.bfsft_execute_batched_serial if serial else self._L.bfsft_execute_batched
        with _Ordered(torch, self._stream, (fd, u)):
            _check(fn(self._h, ctypes.c_void_p(fd.data_ptr() if self.nk else 0),
                      ctypes.c_void_p(u.data_ptr() if self.nx else 0)))
        return u

    def info(self) -> dict:
        info = Info()
        _check(self._L.bfsft_plan_info(self._h, ctypes.byref(info)))
        return _info_dict(info)


def copy_rate(elem_bytes: int = 8, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s (read + write) of the library's plain streaming copy kernel on
    the current GPU and stream: the practical memory ceiling."""
    torch = _torch()
    out = ctypes.c_double()
    _check(lib().bfsft_copy_rate(int(elem_bytes), int(nbytes), int(reps),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(out)))
    return out.value


def mfma_f64_rate(waves_per_simd: int = 2, iters: int = 20000) -> float:
    """FP64 TFLOP/s of 12 independent v_mfma_f64_16x16x4f64 chains per wave
    at waves_per_simd waves per SIMD on the current GPU and stream: the
    practical ceiling of the matrix-core direct sums."""
    torch = _torch()
    out = ctypes.c_double()
    _check(lib().bfsft_mfma_f64_rate(int(waves_per_simd), int(iters),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(out)))
    return out.value


def transform(x, k, f, N, p, d=None, precision="fp64"):
    """One-shot u = B(x, k) f on the GPU (plan, execute, destroy)."""
    d = d or np.asarray(x).shape[-1]
    with Plan(d, N, p, x, k, precision) as P:
        return P.execute(f)
