"""Batches: many independent blocks of uneven size in one persistent launch.

A ``Plan`` wraps ``fdbb_batch_plan_*``: the task table lives on the device,
one persistent kernel walks every tile of every task, and that launch is
captured once in a HIP graph and replayed.  ``run_noalloc`` is the same
launch without a plan (``fdbb_batch_run_noalloc``: the table goes into the
library's fixed device array, nothing is allocated).  Task builders take
the same tensors as the single-call functions in ``fdbb``.
"""
from __future__ import annotations

import ctypes

import torch

from . import fdbb as F


def _task(op, dim, dtype, gamma, n, direction=0):
    t = F.Task()
    t.op = F.OPS[op] if isinstance(op, str) else op
    t.dim = dim
    t.dtype = dtype
    t.dir = direction
    t.gamma = gamma
    t.n = n
    return t


def _set(t, slot, tensor, fields=None, dim=None, blocks=False):
    if tensor is None:
        return
    if blocks:
        ptr, ld = F._blocks(tensor, dim)
    elif fields is None:
        ptr, ld = F._dptr(tensor, slot), 0
    else:
        ptr, ld = F._fields(tensor, fields, slot)
    setattr(t, slot, ptr)
    setattr(t, "ld_" + slot, ld)


def fused_task(U, F_=None, A=None, R=None, gamma=1.4):
    dim = U.shape[0] - 2
    t = _task("fused", dim, F.dtype_code(U.dtype), gamma, U.shape[1])
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", F_, (dim + 2) * dim)
    _set(t, "out1", A, dim=dim, blocks=True)
    _set(t, "out2", R, 2 * dim + 1)
    return t


def flux_task(U, F_, gamma=1.4):
    dim = U.shape[0] - 2
    t = _task("flux", dim, F.dtype_code(U.dtype), gamma, U.shape[1])
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", F_, (dim + 2) * dim)
    return t


def flux_dir_task(U, Fd, direction, gamma=1.4):
    """F_direction alone (K fields) of the state U."""
    dim = U.shape[0] - 2
    t = _task("flux_dir", dim, F.dtype_code(U.dtype), gamma, U.shape[1], direction)
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", Fd, dim + 2)
    return t


def jacobian_task(U, A, gamma=1.4):
    dim = U.shape[0] - 2
    t = _task("flux_jacobian", dim, F.dtype_code(U.dtype), gamma, U.shape[1])
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", A, dim=dim, blocks=True)
    return t


def eos_task(U, p=None, c=None, gamma=1.4):
    dim = U.shape[0] - 2
    t = _task("eos", dim, F.dtype_code(U.dtype), gamma, U.shape[1])
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", p)
    _set(t, "out1", c)
    return t


def cons2prim_task(U, V, gamma=1.4):
    dim = U.shape[0] - 2
    t = _task("cons2prim", dim, F.dtype_code(U.dtype), gamma, U.shape[1])
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", V, dim + 2)
    return t


def adjoint_task(U, Fbar, Ubar, gamma=1.4, direction=-1):
    dim = U.shape[0] - 2
    t = _task("adjoint", dim, F.dtype_code(U.dtype), gamma, U.shape[1], direction)
    _set(t, "in0", U, dim + 2)
    _set(t, "in1", Fbar, (dim + 2) * dim if direction < 0 else dim + 2)
    _set(t, "out0", Ubar, dim + 2)
    return t


def roe_task(UL, UR, Uh, gamma=1.4):
    dim = UL.shape[0] - 2
    t = _task("roe_average", dim, F.dtype_code(UL.dtype), gamma, UL.shape[1])
    _set(t, "in0", UL, dim + 2)
    _set(t, "in1", UR, dim + 2)
    _set(t, "out0", Uh, dim + 2)
    return t


def riemann_task(U, R, gamma=1.4):
    dim = U.shape[0] - 2
    t = _task("riemann_invariants", dim, F.dtype_code(U.dtype), gamma, U.shape[1])
    _set(t, "in0", U, dim + 2)
    _set(t, "out0", R, 2 * dim + 1)
    return t


MAX_NOALLOC_TASKS = 1024  # FDBB_NOALLOC_MAX_TASKS


def run_noalloc(tasks, block=0, ppt=1, grid=0, nontemporal=1, stream=None):
    """One persistent launch of ``tasks`` through the allocation-free entry
    point (at most MAX_NOALLOC_TASKS tasks); ``block=0`` takes the installed
    batch configuration, as for plans."""
    arr = (F.Task * max(1, len(tasks)))(*tasks)
    F.check(F.library().fdbb_batch_run_noalloc(arr, len(tasks), block, ppt, grid, nontemporal,
                                               F._stream(stream)))


class Plan:
    """Owner of one ``fdbb_batch_plan``.  ``block=0`` (the default) takes the
    autotuned batch configuration installed for the first task's storage
    type (``fdbb_set_batch_config``); an explicit block uses the given
    ``ppt``, ``grid`` and ``nontemporal``."""

    def __init__(self, tasks, capacity=None, block=0, ppt=1, grid=0, nontemporal=1):
        lib = F.library()
        arr = (F.Task * max(1, len(tasks)))(*tasks)
        self.capacity = capacity or max(1, len(tasks))
        self._h = ctypes.c_void_p()
        F.check(lib.fdbb_batch_plan_create(arr, len(tasks), self.capacity, block, ppt, grid,
                                           nontemporal, ctypes.byref(self._h)))
        self.block, self.ppt, self.grid, self.nontemporal = self.config()

    def config(self):
        """(block, ppt, grid, nontemporal) the plan launches with."""
        b, p, g, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        F.check(F.library().fdbb_batch_plan_config(self._h, ctypes.byref(b), ctypes.byref(p), ctypes.byref(g),
                                                   ctypes.byref(t)))
        return b.value, p.value, g.value, t.value

    def update(self, tasks, stream=None):
        arr = (F.Task * max(1, len(tasks)))(*tasks)
        F.check(F.library().fdbb_batch_plan_update(self._h, arr, len(tasks), F._stream(stream)))

    def run(self, stream=None, graph=True):
        F.check(F.library().fdbb_batch_exec(self._h, F._stream(stream), 1 if graph else 0))

    def info(self):
        pts, tiles = ctypes.c_int64(), ctypes.c_int64()
        F.check(F.library().fdbb_batch_plan_info(self._h, ctypes.byref(pts), ctypes.byref(tiles)))
        return pts.value, tiles.value

    def close(self):
        if self._h and self._h.value:
            # launches of this plan may still be queued: let them finish first
            torch.cuda.synchronize()
            F.library().fdbb_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
