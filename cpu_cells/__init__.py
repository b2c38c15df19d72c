"""Algorithm-matched CPU baseline (measurement only).

The paper's speedups compare like with like: its GPU cell-list code against a
CPU cell-list code. This package is that CPU side for the benchmark: the same
method (cells of side >= r_c rebuilt every step by a counting sort, the
27-cell force sum of the force-shifted LJ force, velocity Verlet) in C with
OpenMP threads and SIMD pair loops, in FP32 and FP64 (``cells_cpu.c``). It shares no code with the
GPU library or with the brute-force oracle; a CPU test pins its forces to the
oracle's. ``build()`` compiles it with gcc for the host it runs on.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cells_cpu.c")
_LIB = os.path.join(_HERE, "libcells_cpu.so")
_lib = None


class Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("box", "epsilon", "sigma", "rc", "mass", "dt")]


def build(force: bool = True, native: bool = False) -> str:
    """gcc -O3 with OpenMP; ``native`` tunes for the building host's CPU
    (for a build made where it runs), otherwise x86-64-v3 (AVX2, FMA)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        arch = "-march=native" if native else "-march=x86-64-v3"
        # no errno from sqrt and no trapping arithmetic (no FP trap is ever
        # enabled): the masked pair loop then runs in SIMD lanes; every result
        # stays IEEE
        subprocess.run(["gcc", "-O3", arch, "-fno-math-errno", "-fno-trapping-math", "-std=c11", "-fopenmp", "-fPIC",
                        "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(Params)
        for name, real in (("cc_run_f32", ctypes.c_float), ("cc_run_f64", ctypes.c_double)):
            f = getattr(lib, name)
            rp = ctypes.POINTER(real)
            f.argtypes = [P, ctypes.c_int64, rp, rp, rp, ctypes.c_int32]
            f.restype = ctypes.c_int
        lib.cc_num_threads.restype = ctypes.c_int
        lib.cc_set_threads.argtypes = [ctypes.c_int]
        lib.cc_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().cc_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following runs."""
    _load().cc_set_threads(int(n))


def run(pos, vel, box, nsteps, *, precision="f64", epsilon=1.0, sigma=1.0, rc_over_sigma=2.5, mass=1.0, dt=0.005):
    """nsteps cell-list Verlet steps from (pos, vel) ([N, >=3] arrays, user
    order). Returns (pos, vel, force) as [N, 3] arrays of the precision."""
    dtype = np.float32 if precision == "f32" else np.float64
    real = ctypes.c_float if precision == "f32" else ctypes.c_double
    x = np.ascontiguousarray(np.asarray(pos)[:, :3], dtype=dtype).copy()
    v = np.ascontiguousarray(np.asarray(vel)[:, :3], dtype=dtype).copy()
    f = np.zeros_like(x)
    p = Params(float(box), float(epsilon), float(sigma), float(rc_over_sigma * sigma), float(mass), float(dt))
    fn = getattr(_load(), "cc_run_f32" if precision == "f32" else "cc_run_f64")
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(real))
    rc = fn(ctypes.byref(p), x.shape[0], ptr(x), ptr(v), ptr(f), int(nsteps))
    if rc != 0:
        raise ValueError("the CPU cell-list baseline needs at least 3 cells per dimension")
    return x, v, f
