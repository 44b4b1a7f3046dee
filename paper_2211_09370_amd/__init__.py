"""MI355X-native single-step simplified lattice Boltzmann solver for quasi-static MHD pipe flow
(arXiv:2211.09370).

Every step of the solver runs in the HIP kernels of libmhdlbm.so (include/mhdlbm.h). This module
is a thin binding: the functions named like the C calls marshal arguments through ctypes, and
`Sim` wraps them with PyTorch providing the device workspace and the stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (MHD_BEXT_NONE, MHD_BEXT_SIX_MAGNETS, MHD_BEXT_TANH_FRINGE_Y, MHD_BEXT_UNIFORM_Y,
                   MHD_FIELD_B_INDUCED,
                   MHD_FIELD_RHO, MHD_FIELD_U, MHD_K_BUDGET, MHD_K_CONTROL, MHD_K_FLUID,
                   MHD_K_IB, MHD_K_LORENTZ, MHD_K_MAG_SWEEP,
                   MHD_STORE_BF16, MHD_STORE_F16, MHD_STORE_F16_SPLIT, MHD_STORE_F32, MhdError,
                   mhd_budget,
                   mhd_grid_desc, mhd_params, mhd_pipe_desc)

__all__ = ["Sim", "Batch", "MhdError", "mhd_workspace_size", "mhd_create", "mhd_set_markers",
           "mhd_set_params", "mhd_set_field", "mhd_get_field", "mhd_get_time", "mhd_set_time",
           "mhd_step", "mhd_step_noalloc", "mhd_get_budgets", "mhd_record_budget", "mhd_set_profiling",
           "mhd_kernel_stats", "mhd_destroy", "mhd_get_tiles", "mhd_set_tiles", "mhd_set_graph", "mhd_tune",
           "mhd_mag_residual_curve", "mhd_choose_n_mag",
           "mhd_batch_workspace_size", "mhd_batch_create", "mhd_batch_pipe", "mhd_batch_tune",
           "mhd_batch_step", "mhd_batch_set_graph", "mhd_batch_set_profiling",
           "mhd_batch_kernel_stats", "mhd_batch_destroy", "mhd_last_error", "BUDGET_FIELDS"]

BUDGET_FIELDS = [f for f, _ in mhd_budget._fields_]
_STORAGE = {"f32": MHD_STORE_F32, "f16": MHD_STORE_F16, "bf16": MHD_STORE_BF16,
            "f16split": MHD_STORE_F16_SPLIT}
_FIELDS = {"rho": MHD_FIELD_RHO, "u": MHD_FIELD_U, "b": MHD_FIELD_B_INDUCED}
_D = C.POINTER(C.c_double)


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


# ----------------------------------------------------------------------------------------------
# Functions with the C names (handle = ctypes c_void_p)
# ----------------------------------------------------------------------------------------------

def mhd_last_error() -> str:
    return _abi.lib().mhd_last_error().decode()


def mhd_workspace_size(desc: mhd_grid_desc, n_markers: int) -> int:
    n = C.c_size_t(0)
    _abi.check(_abi.lib().mhd_workspace_size(C.byref(desc), int(n_markers), C.byref(n)),
               "mhd_workspace_size")
    return int(n.value)


def mhd_create(desc: mhd_grid_desc, n_markers: int, dev_ptr: int, nbytes: int, stream: int):
    h = C.c_void_p()
    _abi.check(_abi.lib().mhd_create(C.byref(desc), int(n_markers), C.c_void_p(dev_ptr),
                                     int(nbytes), C.c_void_p(stream), C.byref(h)), "mhd_create")
    return h


def mhd_set_markers(h, xyz: np.ndarray, u_wall=None, b_wall=None):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    M = xyz.shape[1] if xyz.size else 0
    uw = None if u_wall is None else np.ascontiguousarray(u_wall, dtype=np.float64)
    bw = None if b_wall is None else np.ascontiguousarray(b_wall, dtype=np.float64)
    _abi.check(_abi.lib().mhd_set_markers(h, _dptr(xyz) if M else None, M, _dptr(uw), _dptr(bw)),
               "mhd_set_markers")


def mhd_set_params(h, p: mhd_params):
    _abi.check(_abi.lib().mhd_set_params(h, C.byref(p)), "mhd_set_params")


def mhd_set_field(h, field: int, host: np.ndarray):
    _abi.check(_abi.lib().mhd_set_field(h, field, _dptr(host)), "mhd_set_field")


def mhd_get_field(h, field: int, host: np.ndarray) -> int:
    """Fills host; returns the status (MHD_ERR_UNSTABLE still fills the array)."""
    st = _abi.lib().mhd_get_field(h, field, _dptr(host))
    if st not in (_abi.MHD_OK, _abi.MHD_ERR_UNSTABLE):
        _abi.check(st, "mhd_get_field")
    return st


def mhd_get_time(h):
    t = C.c_int64(0)
    G = C.c_double(0)
    _abi.check(_abi.lib().mhd_get_time(h, C.byref(t), C.byref(G)), "mhd_get_time")
    return int(t.value), float(G.value)


def mhd_set_time(h, t: int, G: float):
    _abi.check(_abi.lib().mhd_set_time(h, int(t), float(G)), "mhd_set_time")


def mhd_step(h, n_steps: int, budget_every: int = 0):
    _abi.check(_abi.lib().mhd_step(h, int(n_steps), int(budget_every)), "mhd_step")


def mhd_step_noalloc(h, n_steps: int, budget_every: int = 0):
    _abi.check(_abi.lib().mhd_step_noalloc(h, int(n_steps), int(budget_every)), "mhd_step_noalloc")


def mhd_record_budget(h):
    _abi.check(_abi.lib().mhd_record_budget(h), "mhd_record_budget")


def mhd_get_budgets(h, cap: int = 4096):
    """Returns (list of dict records, status)."""
    buf = (mhd_budget * max(int(cap), 1))()
    n = C.c_int64(0)
    st = _abi.lib().mhd_get_budgets(h, buf, int(cap), C.byref(n))
    if st not in (_abi.MHD_OK, _abi.MHD_ERR_UNSTABLE):
        _abi.check(st, "mhd_get_budgets")
    recs = [{f: getattr(buf[i], f) for f in BUDGET_FIELDS} for i in range(n.value)]
    return recs, st


def mhd_set_profiling(h, enable: bool):
    _abi.check(_abi.lib().mhd_set_profiling(h, 1 if enable else 0), "mhd_set_profiling")


def mhd_kernel_stats(h, kernel: int):
    n = C.c_int64(0)
    ms = C.c_double(0)
    _abi.check(_abi.lib().mhd_kernel_stats(h, int(kernel), C.byref(n), C.byref(ms)),
               "mhd_kernel_stats")
    return int(n.value), float(ms.value)


def mhd_destroy(h):
    _abi.check(_abi.lib().mhd_destroy(h), "mhd_destroy")


def mhd_mag_residual_curve(h, n_sweeps: int) -> np.ndarray:
    out = np.zeros(int(n_sweeps))
    _abi.check(_abi.lib().mhd_mag_residual_curve(h, int(n_sweeps), _dptr(out)), "mhd_mag_residual_curve")
    return out


def mhd_choose_n_mag(h, tol: float, n_max: int, apply: bool = False) -> int:
    n = C.c_int32(0)
    _abi.check(_abi.lib().mhd_choose_n_mag(h, float(tol), int(n_max), 1 if apply else 0, C.byref(n)),
               "mhd_choose_n_mag")
    return int(n.value)


def mhd_get_tiles(h):
    t = (C.c_int32 * 4)()
    _abi.check(_abi.lib().mhd_get_tiles(h, t), "mhd_get_tiles")
    return tuple(int(v) for v in t)


def mhd_set_tiles(h, tiles):
    t = (C.c_int32 * 4)(*[int(v) for v in tiles])
    _abi.check(_abi.lib().mhd_set_tiles(h, t), "mhd_set_tiles")


def mhd_tune(h, reps=5):
    _abi.check(_abi.lib().mhd_tune(h, int(reps)), "mhd_tune")


def mhd_set_graph(h, enable):
    _abi.check(_abi.lib().mhd_set_graph(h, 1 if enable else 0), "mhd_set_graph")


def _pipe_array(pipes):
    arr = (mhd_pipe_desc * len(pipes))()
    for i, p in enumerate(pipes):
        arr[i] = p
    return arr


def mhd_batch_workspace_size(pipes) -> int:
    n = C.c_size_t(0)
    arr = _pipe_array(pipes)
    _abi.check(_abi.lib().mhd_batch_workspace_size(arr, len(pipes), C.byref(n)),
               "mhd_batch_workspace_size")
    return int(n.value)


def mhd_batch_create(pipes, dev_ptr: int, nbytes: int, stream: int):
    h = C.c_void_p()
    arr = _pipe_array(pipes)
    _abi.check(_abi.lib().mhd_batch_create(arr, len(pipes), C.c_void_p(dev_ptr), int(nbytes),
                                           C.c_void_p(stream), C.byref(h)), "mhd_batch_create")
    return h


def mhd_batch_pipe(h, i: int):
    out = C.c_void_p()
    _abi.check(_abi.lib().mhd_batch_pipe(h, int(i), C.byref(out)), "mhd_batch_pipe")
    return out


def mhd_batch_tune(h, reps: int = 5):
    _abi.check(_abi.lib().mhd_batch_tune(h, int(reps)), "mhd_batch_tune")


def mhd_batch_step(h, n_steps: int, budget_every: int = 0):
    _abi.check(_abi.lib().mhd_batch_step(h, int(n_steps), int(budget_every)), "mhd_batch_step")


def mhd_batch_set_graph(h, enable: bool):
    _abi.check(_abi.lib().mhd_batch_set_graph(h, 1 if enable else 0), "mhd_batch_set_graph")


def mhd_batch_set_profiling(h, enable: bool):
    _abi.check(_abi.lib().mhd_batch_set_profiling(h, 1 if enable else 0),
               "mhd_batch_set_profiling")


def mhd_batch_kernel_stats(h, kernel: int):
    n = C.c_int64(0)
    ms = C.c_double(0)
    _abi.check(_abi.lib().mhd_batch_kernel_stats(h, int(kernel), C.byref(n), C.byref(ms)),
               "mhd_batch_kernel_stats")
    return int(n.value), float(ms.value)


def mhd_batch_destroy(h):
    _abi.check(_abi.lib().mhd_batch_destroy(h), "mhd_batch_destroy")


# ----------------------------------------------------------------------------------------------
# Convenience wrapper: torch owns the workspace and the stream
# ----------------------------------------------------------------------------------------------

def make_params(src=None, **over) -> mhd_params:
    """mhd_params from any object / dict with the field names of the C struct, plus overrides."""
    p = mhd_params()
    p.lambda_u = 1.0
    p.fringe_w = 1.0
    p.k_c = 0.1
    p.n_mag = 1
    p.alpha = 1.0
    p.gamma = 1.0
    names = [f for f, _ in mhd_params._fields_]
    vals = {}
    if src is not None:
        alias = {"magnet_half_width": "magnet_L", "magnet_distance": "magnet_D"}
        for f in names:
            g = alias.get(f, f)
            if isinstance(src, dict):
                if f in src:
                    vals[f] = src[f]
                elif g in src:
                    vals[f] = src[g]
            elif hasattr(src, f):
                vals[f] = getattr(src, f)
            elif hasattr(src, g):
                vals[f] = getattr(src, g)
    vals.update(over)
    for f, v in vals.items():
        setattr(p, f, int(v) if f in ("n_mag", "bext_kind", "flow_control", "lattice") else float(v))
    return p


class Sim:
    """One periodic box with an immersed pipe wall, stepped on a torch CUDA stream of its own
    unless one is given (steps on such a stream replay as captured HIP graphs; the NULL stream
    cannot be captured). `get_field` and `budgets` synchronise with it; use
    `torch.cuda.synchronize()` before timing or before reading its results by other means."""

    def __init__(self, nx: int, ny: int, nz: int, n_markers: int = 0, *, rho_storage="f32",
                 u_storage="f32", b_storage="f32", u_scale: float = 1.0, b_scale: float = 1.0,
                 device=None, stream=None, _handle=None, _owner=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.desc = mhd_grid_desc(self.nx, self.ny, self.nz, _STORAGE[rho_storage],
                                  _STORAGE[u_storage], _STORAGE[b_storage], float(u_scale),
                                  float(b_scale))
        self.n_markers = int(n_markers)
        if _handle is not None:  # a pipe of a Batch: the batch owns the handle and the memory
            self._h = _handle
            self._owner = _owner
            return
        self._owner = None
        import torch

        nbytes = mhd_workspace_size(self.desc, self.n_markers)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        # 256-byte aligned workspace carved out of one uint8 tensor; the allocation is ordered on
        # torch's current stream, the solver's stream may differ
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        base = self._ws.data_ptr()
        self._ptr = (base + 255) & ~255
        self.workspace_bytes = nbytes
        self._h = mhd_create(self.desc, self.n_markers, self._ptr, nbytes, self._stream.cuda_stream)

    # -- setup -----------------------------------------------------------------------------
    def set_markers(self, xyz, u_wall=None, b_wall=None):
        mhd_set_markers(self._h, xyz, u_wall, b_wall)

    def set_params(self, params=None, **over):
        mhd_set_params(self._h, params if isinstance(params, mhd_params) else make_params(params, **over))

    def set_field(self, name: str, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        want = self.N * (1 if name == "rho" else 3)
        if a.size != want:
            raise ValueError(f"{name}: expected {want} values, got {a.size}")
        mhd_set_field(self._h, _FIELDS[name], a)

    def get_field(self, name: str) -> np.ndarray:
        shape = (self.nz, self.ny, self.nx) if name == "rho" else (3, self.nz, self.ny, self.nx)
        out = np.empty(shape, dtype=np.float64)
        self.last_status = mhd_get_field(self._h, _FIELDS[name], out)
        return out

    # -- stepping --------------------------------------------------------------------------
    def step(self, n: int = 1, budget_every: int = 0):
        mhd_step(self._h, n, budget_every)

    def step_noalloc(self, n: int = 1, budget_every: int = 0):
        """mhd_step with its kernels' scratch in the library's static device array (no allocation)."""
        mhd_step_noalloc(self._h, n, budget_every)

    def tune(self, reps: int = 5):
        """Time every valid sweep tile choice on the live fields and keep the fastest (state unchanged)."""
        mhd_tune(self._h, reps)

    def set_graph(self, on: bool):
        """Graph replay of the steps on a caller stream (default on; no effect on the default stream)."""
        mhd_set_graph(self._h, on)

    def record_budget(self):
        mhd_record_budget(self._h)

    def budgets(self):
        recs, st = mhd_get_budgets(self._h)
        self.last_status = st
        return recs

    def time(self):
        return mhd_get_time(self._h)

    def set_time(self, t: int, G: float):
        mhd_set_time(self._h, t, G)

    def set_profiling(self, on: bool):
        mhd_set_profiling(self._h, on)

    def kernel_stats(self, kernel: int):
        return mhd_kernel_stats(self._h, kernel)

    def mag_residual_curve(self, n_sweeps: int) -> np.ndarray:
        """Induction residual after each of n_sweeps sweeps from the current state (restored)."""
        return mhd_mag_residual_curve(self._h, n_sweeps)

    def choose_n_mag(self, tol: float, n_max: int, apply: bool = False) -> int:
        """Smallest sweep count whose residual is within tol of the first sweep's (Sec. 5.8)."""
        return mhd_choose_n_mag(self._h, tol, n_max, apply)

    @property
    def tiles(self):
        """Sweep tile choice (x tile, z chunk, paired form, rows of the paired form)."""
        return mhd_get_tiles(self._h)

    @tiles.setter
    def tiles(self, t):
        mhd_set_tiles(self._h, t)

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h = None
            return
        if getattr(self, "_h", None) is not None and self._h.value:
            mhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent boxes advanced together (`mhd_batch_*`); `pipes[i]` is a Sim view of
    box i for setup and read-back. Stepped on a torch CUDA stream of its own unless one is
    given (`stream.synchronize()` or `torch.cuda.synchronize()` before timing)."""

    def __init__(self, boxes, *, rho_storage="f32", u_storage="f32", b_storage="f32",
                 u_scale: float = 1.0, b_scale: float = 1.0, device=None, stream=None):
        """boxes: sequence of (nx, ny, nz, n_markers)."""
        import torch

        self.boxes = [tuple(int(v) for v in b) for b in boxes]
        kinds = (_STORAGE[rho_storage], _STORAGE[u_storage], _STORAGE[b_storage])
        descs = [mhd_pipe_desc(mhd_grid_desc(nx, ny, nz, *kinds, float(u_scale), float(b_scale)), m)
                 for nx, ny, nz, m in self.boxes]
        nbytes = mhd_batch_workspace_size(descs)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        # a stream of its own by default: the NULL stream cannot be captured into a graph
        self._stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)  # the workspace allocation is ordered on torch's stream
        self._ptr = (self._ws.data_ptr() + 255) & ~255
        self.workspace_bytes = nbytes
        self._h = mhd_batch_create(descs, self._ptr, nbytes, self._stream.cuda_stream)
        self.pipes = []
        for i, (nx, ny, nz, m) in enumerate(self.boxes):
            self.pipes.append(Sim(nx, ny, nz, m, rho_storage=rho_storage, u_storage=u_storage,
                                  b_storage=b_storage, u_scale=u_scale, b_scale=b_scale,
                                  _handle=mhd_batch_pipe(self._h, i), _owner=self))

    @property
    def n_cells(self) -> int:
        return sum(nx * ny * nz for nx, ny, nz, _ in self.boxes)

    def tune(self, reps: int = 5):
        mhd_batch_tune(self._h, reps)

    def step(self, n: int = 1, budget_every: int = 0):
        mhd_batch_step(self._h, n, budget_every)

    def set_graph(self, on: bool):
        mhd_batch_set_graph(self._h, on)

    def set_profiling(self, on: bool):
        mhd_batch_set_profiling(self._h, on)

    def kernel_stats(self, kernel: int):
        return mhd_batch_kernel_stats(self._h, kernel)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for p in self.pipes:
                p._h = None
            mhd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
