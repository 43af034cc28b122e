"""Host-core comparator: plain restarted Arnoldi for exp(-tA) b with OpenMP (``plain_arnoldi.cpp``).

Neither the oracle nor the GPU product: it times the plain method on the host cores of the GPU
machine, for the sketched-versus-plain comparison.  ``build()`` compiles ``libplaincpu.so`` in place
with g++; ``expv`` calls it through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "plain_arnoldi.cpp")
LIB = os.path.join(HERE, "libplaincpu.so")
# x86-64-v3 (AVX2, FMA): every EPYC host of the GPU machines has it; the loops are memory-bound
FLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c++17"]
STATUS = {0: "converged", 1: "breakdown", 2: "max_cycles", -1: "invalid"}

_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    res = subprocess.run(["g++", *FLAGS, SRC, "-o", tmp], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"g++ failed ({res.returncode}):\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built (cpu_baseline.build())")
        lib = ctypes.CDLL(LIB)
        f = lib.cpu_plain_expv
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        lib.cpu_plain_threads.restype = ctypes.c_int
        lib.cpu_plain_threads.argtypes = []
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads a call uses."""
    return int(_load().cpu_plain_threads())


def expv(rowptr, colind, vals, b, t, m, tol, max_cycles=100, n_quad=128):
    """x ~ exp(-tA) b for the CSR matrix A (int32 indices, FP64 values); returns (x, info)."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = b.shape[0]
    if rowptr.shape[0] != n + 1 or colind.shape[0] != vals.shape[0] or rowptr[-1] != vals.shape[0]:
        raise ValueError("inconsistent CSR arrays")
    x = np.empty(n, dtype=np.float64)
    cyc, mv = ctypes.c_int(0), ctypes.c_int(0)
    st = lib.cpu_plain_expv(n, rowptr.ctypes.data, colind.ctypes.data, vals.ctypes.data, b.ctypes.data, float(t),
                            int(m), float(tol), int(max_cycles), int(n_quad), x.ctypes.data, ctypes.byref(cyc),
                            ctypes.byref(mv))
    if st < 0:
        raise ValueError("cpu_plain_expv rejected its arguments")
    return x, {"status": STATUS[st], "cycles": cyc.value, "matvecs": mv.value}
