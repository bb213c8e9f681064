"""CPU oracle for the butterfly sparse Fourier transform.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the library.  It
shares no code with the GPU path (see ``bfsft_oracle.c`` for the paper
passages each function follows).

* :func:`direct` - O1, eq. (1) evaluated term by term (FP64, double-double
  phase reduction), OpenMP over outputs.
* :class:`Butterfly` - O2, the f-form butterfly of Section 2.2, FP64.
* :func:`direct_numpy` - O3, a plain numpy evaluation of eq. (1) for tiny
  problems (phases small enough that FP64 reduction is exact enough).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfsft_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# another build of this source to load instead (the mutation tests point it
# at copies with one planted mistake each); never rebuilt here
_SO_OVERRIDE = os.environ.get("BFSFT_ORACLE_LIB")
_lib = None

__all__ = ["build", "direct", "direct_numpy", "Butterfly", "threads"]


def build(force: bool = True, src: str = _SRC, out: str = _SO) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math); `src` and
    `out` default to this package's source and library."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
            "-fcx-limited-range", "-fno-fast-math", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _SO_OVERRIDE:
        lib = ctypes.CDLL(_SO_OVERRIDE)
    else:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_SO)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    D = ctypes.c_double
    lib.or_direct.argtypes = [I, D, P, P, P, I64, P, I64, P]
    lib.or_direct.restype = None
    lib.or_bf_create.argtypes = [I, I64, I, P, I64, P, I64]
    lib.or_bf_create.restype = P
    lib.or_bf_destroy.argtypes = [P]
    lib.or_bf_destroy.restype = None
    lib.or_bf_levels.argtypes = [P]
    lib.or_bf_levels.restype = I
    lib.or_bf_count.argtypes = [P, I, I]
    lib.or_bf_count.restype = I64
    lib.or_bf_boxes.argtypes = [P, I, I, P]
    lib.or_bf_boxes.restype = None
    lib.or_bf_matrix_M.argtypes = [P, I64, I64, P]
    lib.or_bf_matrix_M.restype = None
    lib.or_bf_matrix_E.argtypes = [P, I64, I64, P]
    lib.or_bf_matrix_E.restype = None
    lib.or_bf_run.argtypes = [P, P, P, I, P, P, I]
    lib.or_bf_run.restype = I
    lib.or_set_threads.argtypes = [I]
    lib.or_set_threads.restype = None
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = I
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads(n: int | None = None) -> int:
    """Set (if n) and return the OpenMP thread count of the oracle."""
    lib = _load()
    if n:
        lib.or_set_threads(int(n))
    return lib.or_max_threads()


def direct(x, k, f, N, idx=None):
    """O1: u[s] = sum_j exp(2 pi i x_{idx[s]}.k_j / N) f_j (all outputs if idx is None)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.complex128)
    d = x.shape[1]
    if idx is None:
        idx = np.arange(x.shape[0], dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    u = np.zeros(idx.shape[0], dtype=np.complex128)
    lib.or_direct(d, float(N), _ptr(x), _ptr(k), _ptr(f), k.shape[0], _ptr(idx),
                  idx.shape[0], _ptr(u))
    return u


def direct_numpy(x, k, f, N):
    """O3: eq. (1) as one dense numpy product (tiny problems only)."""
    ph = (np.asarray(x, np.float64) @ np.asarray(k, np.float64).T) / float(N)
    ph = ph - np.round(ph)
    return np.exp(2j * np.pi * ph) @ np.asarray(f, np.complex128)


class Butterfly:
    """O2: the paper's butterfly (Section 2.2, steps 1-4), f-form, FP64."""

    def __init__(self, d, N, p, x, k):
        self._lib = _load()
        self.x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, d)
        self.k = np.ascontiguousarray(k, dtype=np.float64).reshape(-1, d)
        self.d, self.N, self.p = int(d), int(N), int(p)
        self._h = self._lib.or_bf_create(self.d, self.N, self.p, _ptr(self.x),
                                         self.x.shape[0], _ptr(self.k), self.k.shape[0])
        if not self._h:
            raise ValueError("oracle: invalid parameters")
        self.L = self._lib.or_bf_levels(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_bf_destroy(h)
            self._h = None

    def count(self, side: str, m: int) -> int:
        return int(self._lib.or_bf_count(self._h, 0 if side == "x" else 1, m))

    def boxes(self, side: str, m: int) -> np.ndarray:
        """Integer box coordinates (n, d) of level m, in the oracle's order."""
        n = self.count(side, m)
        out = np.zeros((n, self.d), dtype=np.int64)
        self._lib.or_bf_boxes(self._h, 0 if side == "x" else 1, m, _ptr(out))
        return out

    def matrix_M(self, iA, iB):
        out = np.zeros((self.p, self.p), dtype=np.complex128)
        self._lib.or_bf_matrix_M(self._h, int(iA), int(iB), _ptr(out))
        return out

    def matrix_E(self, iA, ic):
        out = np.zeros((self.p, self.p), dtype=np.complex128)
        self._lib.or_bf_matrix_E(self._h, int(iA), int(ic), _ptr(out))
        return out

    def run(self, f, dump_level=None, start_level=0):
        """Returns u (original target order); with dump_level, also the check
        potentials and charges of that T_K level, shape (nA, nB, p^d).
        start_level s0: the sweep begins at T_K level L - s0 with charges
        matched to directly summed potentials (0: at the leaves)."""
        f = np.ascontiguousarray(f, dtype=np.complex128)
        u = np.zeros(self.x.shape[0], dtype=np.complex128)
        du = df = None
        lvl = -1
        if dump_level is not None:
            lvl = int(dump_level)
            nA = self.count("x", self.L - lvl)
            nB = self.count("k", lvl)
            du = np.zeros((nA, nB, self.p ** self.d), dtype=np.complex128)
            df = np.zeros_like(du)
        rc = self._lib.or_bf_run(self._h, _ptr(f), _ptr(u), lvl,
                                 _ptr(du) if du is not None else None,
                                 _ptr(df) if df is not None else None, int(start_level))
        if rc != 0:
            raise RuntimeError(f"oracle butterfly failed ({rc})")
        if dump_level is None:
            return u
        return u, du, df
