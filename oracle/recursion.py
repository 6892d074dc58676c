"""ctypes front end of O3 (oracle/recursion.c), the plain O(N) recursion.

``build()`` compiles recursion.c with gcc (-O2, no fast-math, OpenMP across
modes only).  ``long_range`` mirrors ``soewald2d.long_range`` (all particles).
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "recursion.c")
_LIB = os.path.join(_HERE, "_o3.so")
_lib = None


def build(force=False):
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.o3_long_range.restype = ctypes.c_int
        lib.o3_long_range.argtypes = [ctypes.c_int, d, d, d, d, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, d, d, d, d, ctypes.c_int,
                                      ip, ip, d, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      d, d, d, d]
        _lib = lib
    return _lib


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def long_range(pos, q, box, alpha, w, s, modes, weights, include_self_pair=True, diag=0.0,
               nthreads=0):
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    N = len(q)
    x = np.ascontiguousarray(pos[:, 0])
    y = np.ascontiguousarray(pos[:, 1])
    z = np.ascontiguousarray(pos[:, 2])
    w = np.asarray(w, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    wr, wi = np.ascontiguousarray(w.real), np.ascontiguousarray(w.imag)
    sr, si = np.ascontiguousarray(s.real), np.ascontiguousarray(s.imag)
    modes = np.asarray(modes).reshape(-1, 2)
    mx = np.ascontiguousarray(modes[:, 0], dtype=np.int32)
    my = np.ascontiguousarray(modes[:, 1], dtype=np.int32)
    wt = np.ascontiguousarray(weights, dtype=np.float64)
    phi = np.zeros(N)
    F = np.zeros((N, 3))
    fx, fy, fz = np.zeros(N), np.zeros(N), np.zeros(N)
    rc = lib.o3_long_range(N, _p(x), _p(y), _p(z), _p(q), box[0], box[1], alpha, len(w),
                           _p(wr), _p(wi), _p(sr), _p(si), len(mx), _p(mx, ctypes.c_int),
                           _p(my, ctypes.c_int), _p(wt), int(include_self_pair), float(diag),
                           int(nthreads), _p(phi), _p(fx), _p(fy), _p(fz))
    if rc != 0:
        raise RuntimeError("o3_long_range failed")
    F[:, 0], F[:, 1], F[:, 2] = fx, fy, fz
    return dict(phi=phi, F=F, U=0.5 * float(q @ phi))
