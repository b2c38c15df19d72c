"""ctypes binding of the C-ABI in include/md.h.

Argument marshalling only: every step of the MD path runs in the HIP kernels
of ``libmdlj.so``. Device buffers are torch tensors on a ROCm device; the
library is handed raw pointers and torch's current HIP stream. There is no
CPU fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdlj.so")

MD_OK = 0
MD_ERR_ARG = 1
MD_ERR_BOX = 2
MD_ERR_WORKSPACE = 3
MD_ERR_HIP = 5
MD_ERR_DEVICE = 6

MD_DEV_NONFINITE = 1
MD_DEV_ORDER = 2
MD_DEV_NB_OVERFLOW = 4
MD_DEV_SKIN = 8

MD_FLAG_PAIR_LISTS = 1
MD_FLAG_ATOM_LISTS = 2

# Symbols declared in include/md.h, in declaration order.
SYMBOLS = (
    "md_workspace_bytes",
    "md_cell_grid",
    "md_tile_capacity",
    "md_build_cells",
    "md_forces",
    "md_forces_noalloc",
    "md_step",
    "md_step_every",
    "md_step_list",
    "md_step_nlist",
    "md_energy_virial",
    "md_thermo",
    "md_get_state",
    "md_neighbors",
    "md_neighbors_lists",
    "md_cell_lists",
    "md_adjoint_kick",
    "md_adjoint_drift",
    "md_adjoint_segment",
    "md_adjoint_recompute",
    "md_adjoint_path",
    "md_step_path",
    "md_loss_grad",
    "md_loss",
    "md_adjoint_seed",
    "md_batch_workspace_bytes",
    "md_batch_build",
    "md_batch_forces",
    "md_batch_step",
    "md_batch_energy_virial",
    "md_batch_get_state",
    "md_batch_graph_create",
    "md_graph_launch",
    "md_graph_destroy",
    "md_check",
    "md_last_error",
    "md_status_name",
)


class MDError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_status_name(code)}: {message}")
        self.code = code


class MDParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("box", ctypes.c_float),
        ("epsilon", ctypes.c_float),
        ("sigma", ctypes.c_float),
        ("mass", ctypes.c_float),
        ("rc_over_sigma", ctypes.c_float),
        ("dt", ctypes.c_float),
        ("cell_min", ctypes.c_float),
        ("shift_mode", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("waves_per_cell", ctypes.c_int32),
        ("list_radius", ctypes.c_float),
        ("tile_cap", ctypes.c_int32),
    ]


class MDReplica(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box", ctypes.c_float), ("cell_min", ctypes.c_float),
                ("waves_per_cell", ctypes.c_int32), ("tile_cap", ctypes.c_int32)]


def replica_table(reps):
    """ctypes array of md_replica from (n, box[, cell_min[, waves_per_cell[,
    tile_cap]]]) tuples (0 for any of the last three: the batch's shared
    cell_min and waves_per_cell, the formula's tile)."""
    arr = (MDReplica * len(reps))()
    for i, r in enumerate(reps):
        arr[i].n = int(r[0])
        arr[i].box = float(r[1])
        arr[i].cell_min = float(r[2]) if len(r) > 2 else 0.0
        arr[i].waves_per_cell = int(r[3]) if len(r) > 3 else 0
        arr[i].tile_cap = int(r[4]) if len(r) > 4 else 0
    return arr


def make_params(n, box, epsilon=1.0, sigma=1.0, mass=1.0, rc_over_sigma=2.5, dt=0.005, cell_min=0.0,
                shift_mode=0, flags=0, waves_per_cell=0, list_radius=0.0, tile_cap=0) -> MDParams:
    return MDParams(int(n), float(box), float(epsilon), float(sigma), float(mass), float(rc_over_sigma),
                    float(dt), float(cell_min), int(shift_mode), int(flags), int(waves_per_cell), float(list_radius),
                    int(tile_cap))


_lib = None


def lib():
    """Load libmdlj.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_0709_3225_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(MDParams)
        vp = ctypes.c_void_p
        sz = ctypes.c_size_t
        i32 = ctypes.c_int32
        L.md_workspace_bytes.argtypes = [P]
        L.md_workspace_bytes.restype = sz
        L.md_cell_grid.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
        L.md_tile_capacity.argtypes = [P]
        L.md_tile_capacity.restype = i32
        L.md_build_cells.argtypes = [P, vp, sz, vp, vp, vp]
        L.md_forces.argtypes = [P, vp, sz, vp, vp]
        L.md_forces_noalloc.argtypes = [P, vp, vp, vp]
        L.md_step.argtypes = [P, vp, sz, i32, i32, vp, vp]
        L.md_step_every.argtypes = [P, vp, sz, i32, i32, i32, vp, vp]
        L.md_step_list.argtypes = [P, vp, sz, i32, i32, i32, vp, vp]
        L.md_step_nlist.argtypes = [P, vp, sz, i32, i32, i32, vp, vp]
        L.md_energy_virial.argtypes = [P, vp, sz, vp, vp]
        L.md_thermo.argtypes = [P, vp, sz, vp, vp]
        L.md_get_state.argtypes = [P, vp, sz, vp, vp, vp]
        L.md_neighbors.argtypes = [P, vp, sz, vp, vp, i32, vp]
        L.md_neighbors_lists.argtypes = [P, vp, sz, vp, vp, i32, i32, vp]
        L.md_cell_lists.argtypes = [P, vp, sz, vp, vp, vp]
        L.md_check.argtypes = [vp, sz, vp, ctypes.POINTER(i32)]
        L.md_adjoint_kick.argtypes = [P, vp, sz, vp, vp, vp, ctypes.c_float, vp]
        L.md_adjoint_drift.argtypes = [P, vp, vp, vp]
        L.md_loss_grad.argtypes = [P, vp, sz, ctypes.c_float, ctypes.c_float, vp, vp, vp, vp]
        L.md_adjoint_segment.argtypes = [P, vp, sz, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.md_adjoint_recompute.argtypes = [P, vp, sz, vp, vp, i32, vp, vp, vp]
        L.md_adjoint_path.argtypes = [P, vp, sz, i32, i32, vp, vp, vp, vp, vp, vp]
        L.md_step_path.argtypes = [P, vp, sz, i32, vp, vp, vp]
        L.md_loss.argtypes = [P, vp, sz, vp, vp]
        L.md_adjoint_seed.argtypes = [P, vp, sz, ctypes.c_float, vp, vp, vp, vp]
        R = ctypes.POINTER(MDReplica)
        L.md_batch_workspace_bytes.argtypes = [P, R, i32]
        L.md_batch_workspace_bytes.restype = sz
        L.md_batch_build.argtypes = [P, R, i32, vp, sz, vp, vp, vp]
        L.md_batch_forces.argtypes = [P, R, i32, vp, sz, vp, vp]
        L.md_batch_step.argtypes = [P, R, i32, vp, sz, i32, i32, vp, vp]
        L.md_batch_energy_virial.argtypes = [P, R, i32, vp, sz, vp, vp]
        L.md_batch_get_state.argtypes = [P, R, i32, vp, sz, vp, vp, vp]
        L.md_batch_graph_create.argtypes = [P, R, i32, vp, sz, i32, i32, vp, vp, ctypes.POINTER(vp)]
        L.md_graph_launch.argtypes = [vp, vp]
        L.md_graph_destroy.argtypes = [vp]
        for name in ("md_cell_grid", "md_build_cells", "md_forces", "md_forces_noalloc", "md_step",
                     "md_step_every", "md_step_list", "md_energy_virial", "md_thermo", "md_get_state",
                     "md_neighbors", "md_neighbors_lists", "md_cell_lists", "md_check", "md_adjoint_kick",
                     "md_adjoint_drift", "md_adjoint_segment", "md_adjoint_recompute",
                     "md_adjoint_path", "md_step_path", "md_loss_grad", "md_loss", "md_adjoint_seed",
                     "md_batch_build", "md_batch_forces", "md_batch_step",
                     "md_batch_energy_virial", "md_batch_get_state", "md_batch_graph_create", "md_graph_launch",
                     "md_graph_destroy"):
            getattr(L, name).restype = ctypes.c_int
        L.md_last_error.argtypes = []
        L.md_last_error.restype = ctypes.c_char_p
        L.md_status_name.argtypes = [ctypes.c_int]
        L.md_status_name.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _status_name(code: int) -> str:
    try:
        return lib().md_status_name(int(code)).decode()
    except Exception:  # the name is only decoration for the message
        return f"status {code}"


def _check(code: int):
    if code != MD_OK:
        raise MDError(code, lib().md_last_error().decode())


# ------------------------------------------------------------------ marshalling

def _ptr(t, name, dtype=None, shape=None):
    """Raw device pointer of a CUDA/HIP tensor after shape/dtype checks."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _ws(ws):
    import torch

    p = _ptr(ws, "workspace", torch.uint8)
    return p, ctypes.c_size_t(ws.numel())


def md_workspace_bytes(p: MDParams) -> int:
    return int(lib().md_workspace_bytes(ctypes.byref(p)))


def md_cell_grid(p: MDParams):
    nc = ctypes.c_int32()
    side = ctypes.c_float()
    _check(lib().md_cell_grid(ctypes.byref(p), ctypes.byref(nc), ctypes.byref(side)))
    return nc.value, side.value


def md_tile_capacity(p: MDParams) -> int:
    """Atoms per LDS pass of the force pass for these parameters."""
    t = lib().md_tile_capacity(ctypes.byref(p))
    if t == 0:
        raise MDError(MD_ERR_ARG, lib().md_last_error().decode())
    return int(t)


def md_build_cells(p: MDParams, ws, pos4, vel4=None, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_build_cells(ctypes.byref(p), wp, wn, _ptr(pos4, "pos4", torch.float32, (p.n, 4)),
                                _ptr(vel4, "vel4", torch.float32, (p.n, 4)), _stream(stream)))


def md_forces(p: MDParams, ws, force4=None, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_forces(ctypes.byref(p), wp, wn, _ptr(force4, "force4", torch.float32, (p.n, 4)),
                           _stream(stream)))


def md_forces_noalloc(p: MDParams, pos4, force4, stream=None):
    import torch

    _check(lib().md_forces_noalloc(ctypes.byref(p), _ptr(pos4, "pos4", torch.float32, (p.n, 4)),
                                   _ptr(force4, "force4", torch.float32, (p.n, 4)), _stream(stream)))


def md_step(p: MDParams, ws, nsteps: int, thermo_every: int = 0, thermo=None, stream=None):
    import torch

    wp, wn = _ws(ws)
    tp = None
    if thermo is not None:
        rows = nsteps // thermo_every if thermo_every > 0 else 0
        if thermo.numel() < 3 * rows:
            raise ValueError(f"thermo needs {3 * rows} doubles")
        tp = _ptr(thermo, "thermo", torch.float64)
    _check(lib().md_step(ctypes.byref(p), wp, wn, int(nsteps), int(thermo_every), tp, _stream(stream)))


def md_step_every(p: MDParams, ws, nsteps: int, rebuild_every: int, thermo_every: int = 0, thermo=None,
                  stream=None):
    import torch

    wp, wn = _ws(ws)
    tp = None
    if thermo is not None:
        rows = nsteps // thermo_every if thermo_every > 0 else 0
        if thermo.numel() < 3 * rows:
            raise ValueError(f"thermo needs {3 * rows} doubles")
        tp = _ptr(thermo, "thermo", torch.float64)
    _check(lib().md_step_every(ctypes.byref(p), wp, wn, int(nsteps), int(rebuild_every), int(thermo_every), tp,
                               _stream(stream)))


def md_step_list(p: MDParams, ws, nsteps: int, rebuild_every: int, thermo_every: int = 0, thermo=None,
                 stream=None):
    import torch

    wp, wn = _ws(ws)
    tp = None
    if thermo is not None:
        rows = nsteps // thermo_every if thermo_every > 0 else 0
        if thermo.numel() < 3 * rows:
            raise ValueError(f"thermo needs {3 * rows} doubles")
        tp = _ptr(thermo, "thermo", torch.float64)
    _check(lib().md_step_list(ctypes.byref(p), wp, wn, int(nsteps), int(rebuild_every), int(thermo_every), tp,
                              _stream(stream)))


def md_step_nlist(p: MDParams, ws, nsteps: int, rebuild_every: int, thermo_every: int = 0, thermo=None,
                  stream=None):
    import torch

    wp, wn = _ws(ws)
    tp = None
    if thermo is not None:
        rows = nsteps // thermo_every if thermo_every > 0 else 0
        if thermo.numel() < 3 * rows:
            raise ValueError(f"thermo needs {3 * rows} doubles")
        tp = _ptr(thermo, "thermo", torch.float64)
    _check(lib().md_step_nlist(ctypes.byref(p), wp, wn, int(nsteps), int(rebuild_every), int(thermo_every), tp,
                               _stream(stream)))


def md_energy_virial(p: MDParams, ws, out3, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_energy_virial(ctypes.byref(p), wp, wn, _ptr(out3, "out3", torch.float64, (3,)),
                                  _stream(stream)))



def md_thermo(p: MDParams, ws, out5, stream=None):
    """out5 = (U, K, W, T, P) in FP64 on the device (md_thermo)."""
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_thermo(ctypes.byref(p), wp, wn, _ptr(out5, "out5", torch.float64, (5,)), _stream(stream)))

def md_get_state(p: MDParams, ws, pos4=None, vel4=None, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_get_state(ctypes.byref(p), wp, wn, _ptr(pos4, "pos4", torch.float32, (p.n, 4)),
                              _ptr(vel4, "vel4", torch.float32, (p.n, 4)), _stream(stream)))


def md_neighbors(p: MDParams, ws, counts, idx, max_per_atom: int, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_neighbors(ctypes.byref(p), wp, wn, _ptr(counts, "counts", torch.int32, (p.n,)),
                              _ptr(idx, "idx", torch.int32, (p.n * max_per_atom,)), int(max_per_atom),
                              _stream(stream)))


def md_neighbors_lists(p: MDParams, ws, counts, idx, max_per_atom: int, record: bool, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_neighbors_lists(ctypes.byref(p), wp, wn, _ptr(counts, "counts", torch.int32, (p.n,)),
                                    _ptr(idx, "idx", torch.int32, (p.n * max_per_atom,)), int(max_per_atom),
                                    1 if record else 0, _stream(stream)))


def md_cell_lists(p: MDParams, ws, cell_start=None, order=None, stream=None):
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_cell_lists(ctypes.byref(p), wp, wn, _ptr(cell_start, "cell_start", torch.int32),
                               _ptr(order, "order", torch.int32, (p.n,)), _stream(stream)))


def md_check(ws, stream=None, raise_on_error: bool = True) -> int:
    """Synchronise and read/clear the device error bits; returns them."""
    wp, wn = _ws(ws)
    flags = ctypes.c_int32()
    code = lib().md_check(wp, wn, _stream(stream), ctypes.byref(flags))
    if code == MD_ERR_DEVICE and not raise_on_error:
        return flags.value
    _check(code)
    return flags.value


def md_adjoint_kick(p: MDParams, ws, w4, lam_r4, theta=None, coef: float = 1.0, stream=None):
    """lam_r4 += coef * J w4 at the workspace positions; theta[0..1] += coef * w.dF/d(eps, sigma)."""
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_adjoint_kick(ctypes.byref(p), wp, wn, _ptr(w4, "w4", torch.float32, (p.n, 4)),
                                 _ptr(lam_r4, "lam_r4", torch.float32, (p.n, 4)),
                                 _ptr(theta, "theta", torch.float64, (2,)), float(coef), _stream(stream)))


def md_adjoint_drift(p: MDParams, lam_r4, lam_v4, stream=None):
    """lam_v4 += dt * lam_r4."""
    import torch

    _check(lib().md_adjoint_drift(ctypes.byref(p), _ptr(lam_r4, "lam_r4", torch.float32, (p.n, 4)),
                                  _ptr(lam_v4, "lam_v4", torch.float32, (p.n, 4)), _stream(stream)))


def md_adjoint_segment(p: MDParams, ws, ckpt_pos4, ckpt_vel4, first_step: int, nsteps: int, path4, path_start,
                       lam_r4, lam_v4, theta=None, stream=None):
    """Recompute a checkpoint segment and run its drift and kick adjoints (md_adjoint_segment)."""
    import torch

    wp, wn = _ws(ws)
    n = p.n
    nc, _ = md_cell_grid(p)
    if path4.numel() < 4 * n * nsteps:
        raise ValueError(f"path4 needs {nsteps} x {n} float4")
    if path_start.numel() < nsteps * (nc ** 3 + 1):
        raise ValueError(f"path_start needs {nsteps} x {nc ** 3 + 1} int32")
    _check(lib().md_adjoint_segment(
        ctypes.byref(p), wp, wn, _ptr(ckpt_pos4, "ckpt_pos4", torch.float32, (n, 4)),
        _ptr(ckpt_vel4, "ckpt_vel4", torch.float32, (n, 4)), int(first_step), int(nsteps),
        _ptr(path4, "path4", torch.float32), _ptr(path_start, "path_start", torch.int32),
        _ptr(lam_r4, "lam_r4", torch.float32, (n, 4)),
        _ptr(lam_v4, "lam_v4", torch.float32, (n, 4)),
        None if theta is None else _ptr(theta, "theta", torch.float64), _stream(stream)))


def _path_ptrs(p: MDParams, nsteps: int, path4, path_start):
    import torch

    nc, _ = md_cell_grid(p)
    if path4.numel() < 4 * p.n * nsteps:
        raise ValueError(f"path4 needs {nsteps} x {p.n} float4")
    if path_start.numel() < nsteps * (nc ** 3 + 1):
        raise ValueError(f"path_start needs {nsteps} x {nc ** 3 + 1} int32")
    return _ptr(path4, "path4", torch.float32), _ptr(path_start, "path_start", torch.int32)


def md_adjoint_recompute(p: MDParams, ws, ckpt_pos4, ckpt_vel4, nsteps: int, path4, path_start, stream=None):
    """The states of a checkpoint segment into a path (md_adjoint_recompute)."""
    import torch

    wp, wn = _ws(ws)
    pp, ps = _path_ptrs(p, nsteps, path4, path_start)
    _check(lib().md_adjoint_recompute(
        ctypes.byref(p), wp, wn, _ptr(ckpt_pos4, "ckpt_pos4", torch.float32, (p.n, 4)),
        _ptr(ckpt_vel4, "ckpt_vel4", torch.float32, (p.n, 4)), int(nsteps), pp, ps, _stream(stream)))


def md_adjoint_path(p: MDParams, ws, first_step: int, nsteps: int, path4, path_start, lam_r4, lam_v4, theta=None,
                    stream=None):
    """Drift and kick adjoints over a kept path, last state first (md_adjoint_path)."""
    import torch

    wp, wn = _ws(ws)
    pp, ps = _path_ptrs(p, nsteps, path4, path_start)
    _check(lib().md_adjoint_path(
        ctypes.byref(p), wp, wn, int(first_step), int(nsteps), pp, ps,
        _ptr(lam_r4, "lam_r4", torch.float32, (p.n, 4)), _ptr(lam_v4, "lam_v4", torch.float32, (p.n, 4)),
        None if theta is None else _ptr(theta, "theta", torch.float64), _stream(stream)))


def md_step_path(p: MDParams, ws, nsteps: int, path4, path_start, stream=None):
    """nsteps of md_step, keeping the state before each step as a path (md_step_path)."""
    wp, wn = _ws(ws)
    pp, ps = _path_ptrs(p, nsteps, path4, path_start)
    _check(lib().md_step_path(ctypes.byref(p), wp, wn, int(nsteps), pp, ps, _stream(stream)))


def md_loss_grad(p: MDParams, ws, k_coef: float, w_coef: float, g_r4, g_v4, theta=None, stream=None):
    """g_r4 = w_coef dW/dr, g_v4 = k_coef m v; theta += w_coef dW/d(eps, sigma)."""
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_loss_grad(ctypes.byref(p), wp, wn, float(k_coef), float(w_coef),
                              _ptr(g_r4, "g_r4", torch.float32, (p.n, 4)), _ptr(g_v4, "g_v4", torch.float32, (p.n, 4)),
                              _ptr(theta, "theta", torch.float64, (2,)), _stream(stream)))


def md_loss(p: MDParams, ws, loss, stream=None):
    """loss[0] = K/N + W/(3V) at the workspace state (FP64, on the device)."""
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_loss(ctypes.byref(p), wp, wn, _ptr(loss, "loss", torch.float64, (1,)), _stream(stream)))


def md_adjoint_seed(p: MDParams, ws, scale: float, lam_r4, lam_v4, theta=None, stream=None):
    """Seed the backward pass from scale * md_loss at the workspace (final) state."""
    import torch

    wp, wn = _ws(ws)
    _check(lib().md_adjoint_seed(ctypes.byref(p), wp, wn, float(scale), _ptr(lam_r4, "lam_r4", torch.float32, (p.n, 4)),
                                 _ptr(lam_v4, "lam_v4", torch.float32, (p.n, 4)),
                                 _ptr(theta, "theta", torch.float64, (2,)), _stream(stream)))
