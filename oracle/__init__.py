"""Reference oracle (test infrastructure only).

A plain FP64 brute-force implementation of truncated-and-shifted Lennard-Jones
molecular dynamics, written from the paper (section 2 equations for the force
sum, f_LJ and the shifted f(r); velocity Verlet), in C with OpenMP
(``lj_oracle.c``) behind this ctypes wrapper.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never calls it, and the two share no
code. ``build()`` compiles the C source with gcc into ``liboracle.so`` next to
it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lj_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double),
        ("epsilon", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("rc", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("shift_mode", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(OracleParams)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_pair.argtypes = [P, ctypes.c_double, dp, dp]
        lib.oracle_pair.restype = None
        lib.oracle_forces.argtypes = [P, i64, dp, dp, dp]
        lib.oracle_forces.restype = ctypes.c_int
        lib.oracle_forces_rows.argtypes = [P, i64, dp, i64, ctypes.POINTER(i64), dp, dp, dp]
        lib.oracle_forces_rows.restype = ctypes.c_int
        lib.oracle_kinetic.argtypes = [P, i64, dp]
        lib.oracle_kinetic.restype = ctypes.c_double
        lib.oracle_neighbors.argtypes = [
            P, i64, dp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), i64,
            ctypes.c_double, ctypes.POINTER(i64)]
        lib.oracle_neighbors.restype = i64
        lib.oracle_run.argtypes = [P, i64, dp, dp, ctypes.c_int32, dp]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_hvp.argtypes = [P, i64, dp, dp, dp]
        lib.oracle_hvp.restype = ctypes.c_int
        lib.oracle_dforce_dparams.argtypes = [P, i64, dp, dp, dp]
        lib.oracle_dforce_dparams.restype = ctypes.c_int
        lib.oracle_virial_grad.argtypes = [P, i64, dp, dp, dp]
        lib.oracle_virial_grad.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def params(box, epsilon=1.0, sigma=1.0, rc=None, mass=1.0, dt=0.005, shift_mode=0):
    """Oracle parameters; rc defaults to 2.5 sigma (section 2)."""
    if rc is None:
        rc = 2.5 * sigma
    return OracleParams(float(box), float(epsilon), float(sigma), float(rc), float(mass),
                        float(dt), int(shift_mode), 0)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _xyz(a) -> np.ndarray:
    a = np.asarray(a)
    if a.ndim == 2 and a.shape[1] == 4:
        a = a[:, :3]
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def pair(p: OracleParams, r: float):
    """(phi(r), u(r)): shifted pair force magnitude and pair energy."""
    phi = ctypes.c_double()
    u = ctypes.c_double()
    _load().oracle_pair(ctypes.byref(p), float(r), ctypes.byref(phi), ctypes.byref(u))
    return phi.value, u.value


def forces(p: OracleParams, pos):
    """All forces [N,3] plus (U, W). pos may be [N,3] or [N,4] (w ignored)."""
    x = _xyz(pos)
    n = x.shape[0]
    f = np.zeros((n, 3), dtype=np.float64)
    uw = np.zeros(2, dtype=np.float64)
    rc = _load().oracle_forces(ctypes.byref(p), n, _dp(x), _dp(f), _dp(uw))
    if rc != 0:
        raise ValueError(f"oracle_forces failed ({rc})")
    return f, float(uw[0]), float(uw[1])


def forces_rows(p: OracleParams, pos, rows):
    """Forces on the listed rows only, plus their per-row (U_i, W_i) halves."""
    x = _xyz(pos)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    k = rows.shape[0]
    f = np.zeros((k, 3), dtype=np.float64)
    ur = np.zeros(k, dtype=np.float64)
    wr = np.zeros(k, dtype=np.float64)
    rc = _load().oracle_forces_rows(
        ctypes.byref(p), x.shape[0], _dp(x), k,
        rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(f), _dp(ur), _dp(wr))
    if rc != 0:
        raise ValueError(f"oracle_forces_rows failed ({rc})")
    return f, ur, wr


def kinetic(p: OracleParams, vel) -> float:
    v = _xyz(vel)
    return float(_load().oracle_kinetic(ctypes.byref(p), v.shape[0], _dp(v)))


def neighbors(p: OracleParams, pos, band: float = 1e-5):
    """Brute-force neighbour sets: (counts[N], idx flat CSR, guard-band count)."""
    x = _xyz(pos)
    n = x.shape[0]
    counts = np.zeros(n, dtype=np.int32)
    cap = max(1, int(n) * 128)
    while True:
        idx = np.zeros(cap, dtype=np.int32)
        guard = ctypes.c_int64()
        tot = _load().oracle_neighbors(
            ctypes.byref(p), n, _dp(x), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap, float(band), ctypes.byref(guard))
        if tot >= 0:
            return counts, idx[:tot].copy(), int(guard.value)
        cap = int(counts.sum()) + 1


def run(p: OracleParams, pos, vel, nsteps: int):
    """Velocity Verlet for nsteps; returns (pos, vel, thermo[(nsteps+1),3] = U,K,W)."""
    x = _xyz(pos).copy()
    v = _xyz(vel).copy()
    th = np.zeros((nsteps + 1, 3), dtype=np.float64)
    rc = _load().oracle_run(ctypes.byref(p), x.shape[0], _dp(x), _dp(v), int(nsteps), _dp(th))
    if rc != 0:
        raise ValueError(f"oracle_run failed ({rc})")
    return x, v, th


def hvp(p: OracleParams, pos, u):
    """J u, J = dF/dr of the force sum (force-shift mode)."""
    x = _xyz(pos)
    uu = _xyz(u)
    out = np.zeros_like(x)
    if _load().oracle_hvp(ctypes.byref(p), x.shape[0], _dp(x), _dp(uu), _dp(out)) != 0:
        raise ValueError("oracle_hvp needs shift_mode 0 and L >= 2 r_c")
    return out


def dforce_dparams(p: OracleParams, pos, a):
    """(sum_i a_i . dF_i/d eps, sum_i a_i . dF_i/d sigma), r_c = 2.5 sigma."""
    x = _xyz(pos)
    aa = _xyz(a)
    out = np.zeros(2)
    if _load().oracle_dforce_dparams(ctypes.byref(p), x.shape[0], _dp(x), _dp(aa), _dp(out)) != 0:
        raise ValueError("oracle_dforce_dparams needs shift_mode 0 and L >= 2 r_c")
    return float(out[0]), float(out[1])


def virial_grad(p: OracleParams, pos):
    """(dW/dr [N,3], dW/d eps, dW/d sigma)."""
    x = _xyz(pos)
    g = np.zeros_like(x)
    dw = np.zeros(2)
    if _load().oracle_virial_grad(ctypes.byref(p), x.shape[0], _dp(x), _dp(g), _dp(dw)) != 0:
        raise ValueError("oracle_virial_grad needs shift_mode 0 and L >= 2 r_c")
    return g, float(dw[0]), float(dw[1])
