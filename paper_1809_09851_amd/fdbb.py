"""ctypes binding of libfdbb.so (C ABI declared in include/fdbb.h).

Argument marshalling only: every building block runs in the HIP kernels of
the library.  There is no CPU fallback; if the library is missing, loading
raises.

Field sets are 2-D tensors ``(fields, n)`` whose rows are ``ld`` elements
apart (``ld = t.stride(0) >= n``, unit stride along points), float64 or
float32, on the current HIP device.  Flux Jacobians are 4-D tensors
``(D, n, K, K)`` with strides ``(ldA*K*K, K*K, K, 1)``.  The ``fdbb_*``
functions mirror the C entry points one to one (same names, same argument
order, tensors in place of pointer/ld pairs); the lower-case helpers
allocate outputs with rows padded to a multiple of 64 elements.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libfdbb.so")

F64, F32 = 0, 1
OK, EINVAL, EALIGN, EALIAS, EHIP, ENOMEM = range(6)
OPS = {
    "cons2prim": 0, "prim2cons": 1, "eos": 2, "flux": 3, "flux_jacobian": 4,
    "riemann_invariants": 5, "cons2char": 6, "char2cons": 7, "fused": 8, "adjoint": 9,
    "v_mag2": 10, "eigenvectors": 11, "char_apply": 12, "roe_average": 13,
    "eos_pvt": 14, "viscous_flux": 15, "flux_dir": 16,
}
EOS_IDS = {"perfect_gas": 0, "stiffened_gas": 1}
ROW_ALIGN = 64  # elements; keeps every row 16-byte aligned for both dtypes

_i = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_p = ctypes.c_void_p


class FdbbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class Task(ctypes.Structure):
    """Mirror of fdbb_task."""
    _fields_ = [
        ("op", ctypes.c_int32), ("dim", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("dir", ctypes.c_int32), ("gamma", _d), ("n", _i64),
        ("in0", _p), ("ld_in0", _i64), ("in1", _p), ("ld_in1", _i64),
        ("out0", _p), ("ld_out0", _i64), ("out1", _p), ("ld_out1", _i64),
        ("out2", _p), ("ld_out2", _i64),
    ]


class Completion(ctypes.Structure):
    """Mirror of fdbb_completion."""
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("out0", _p), ("out1", _p), ("out2", _p), ("ld", _i64),
                ("t_submit_ns", _i64), ("t_admit_ns", _i64), ("t_done_ns", _i64)]


class ServerStats(ctypes.Structure):
    """Mirror of fdbb_server_stats."""
    _fields_ = [("submitted", _i64), ("completed", _i64), ("launches", _i64), ("errors", _i64),
                ("arena_bytes", _i64), ("peak_arena_bytes", _i64), ("queued", _i64)]


_lib = None


def library():
    """Load libfdbb.so (built by ``python -m paper_1809_09851_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(f"{LIBRARY} is not built; run `python -m paper_1809_09851_amd.build`")
        lib = ctypes.CDLL(LIBRARY)
        two = [_i, _d, _i, _p, _i64, _p, _i64, _i64, _p]
        for name in ("fdbb_cons2prim", "fdbb_prim2cons", "fdbb_flux", "fdbb_flux_jacobian",
                     "fdbb_riemann_invariants"):
            getattr(lib, name).argtypes = two
        lib.fdbb_eos.argtypes = [_i, _d, _i, _p, _i64, _p, _p, _i64, _p]
        lib.fdbb_flux_direction.argtypes = [_i, _i, _d, _i, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_velocity_magnitude2.argtypes = [_i, _i, _p, _i64, _p, _i64, _p]
        for name in ("fdbb_cons2char", "fdbb_char2cons"):
            getattr(lib, name).argtypes = [_i, _i, _d, _i, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_euler_fused.argtypes = [_i, _d, _i, _p, _i64, _p, _i64, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_flux_adjoint.argtypes = [_i, _i, _d, _i, _p, _i64, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_eigenvectors.argtypes = [_i, _d, _i, _p, _i64, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_char_apply.argtypes = [_i, _i, _i, _d, _i, _p, _i64, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_roe_average.argtypes = [_i, _d, _i, _p, _i64, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_eos_pvt.argtypes = [_i, _i, _p, _i, _p, _i64, _p, _p, _p, _i64, _p]
        lib.fdbb_viscous_flux.argtypes = [_i, _d, _d, _i, _p, _i64, _p, _i64, _p, _i64, _p, _i64, _i64, _p]
        lib.fdbb_set_launch_config.argtypes = [_i, _i, _i, _i, _i, _i, _i]
        lib.fdbb_get_launch_config.argtypes = [_i, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i),
                                               ctypes.POINTER(_i), ctypes.POINTER(_i)]
        lib.fdbb_set_small_launch_config.argtypes = [_i, _i, _i, _i64, _i, _i, _i, _i]
        lib.fdbb_get_small_launch_config.argtypes = [_i, _i, _i, ctypes.POINTER(_i64)] + [ctypes.POINTER(_i)] * 4
        lib.fdbb_launch_config_for.argtypes = [_i, _i, _i, _i64] + [ctypes.POINTER(_i)] * 4
        lib.fdbb_kernel_info.argtypes = [_i, _i, _i, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]
        lib.fdbb_status_string.argtypes = [_i]
        lib.fdbb_status_string.restype = ctypes.c_char_p
        lib.fdbb_last_error.argtypes = []
        lib.fdbb_last_error.restype = ctypes.c_char_p
        lib.fdbb_version.argtypes = []
        lib.fdbb_batch_plan_create.argtypes = [ctypes.POINTER(Task), _i, _i, _i, _i, _i, _i,
                                               ctypes.POINTER(_p)]
        lib.fdbb_batch_plan_update.argtypes = [_p, ctypes.POINTER(Task), _i, _p]
        lib.fdbb_batch_exec.argtypes = [_p, _p, _i]
        lib.fdbb_batch_plan_info.argtypes = [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        lib.fdbb_batch_plan_destroy.argtypes = [_p]
        lib.fdbb_set_batch_config.argtypes = [_i, _i, _i, _i, _i]
        lib.fdbb_get_batch_config.argtypes = [_i] + [ctypes.POINTER(_i)] * 4
        lib.fdbb_batch_plan_config.argtypes = [_p] + [ctypes.POINTER(_i)] * 4
        lib.fdbb_set_server_batch_config.argtypes = [_i, _i, _i, _i]
        lib.fdbb_get_server_batch_config.argtypes = [ctypes.POINTER(_i)] * 4
        lib.fdbb_batch_run_noalloc.argtypes = [ctypes.POINTER(Task), _i, _i, _i, _i, _i, _p]
        lib.fdbb_task_check.argtypes = [ctypes.POINTER(Task)]
        lib.fdbb_task_run.argtypes = [ctypes.POINTER(Task), _p]
        lib.fdbb_server_create.argtypes = [_i64, _i, _i, _d, _i, ctypes.POINTER(_p)]
        lib.fdbb_server_submit.argtypes = [_p, ctypes.POINTER(Task), ctypes.c_uint64]
        lib.fdbb_server_poll.argtypes = [_p, ctypes.POINTER(Completion), _i, ctypes.POINTER(_i)]
        lib.fdbb_server_release.argtypes = [_p, ctypes.c_uint64]
        lib.fdbb_server_get_stats.argtypes = [_p, ctypes.POINTER(ServerStats)]
        lib.fdbb_server_destroy.argtypes = [_p]
        lib.fdbb_probe_copy.argtypes = [_p, _p, _i64, _i, _p]
        lib.fdbb_probe_write.argtypes = [_p, _i64, ctypes.c_uint64, _i, _p]
        lib.fdbb_probe_read.argtypes = [_p, _i64, _p, _i, _p]
        lib.fdbb_probe_fused_stores.argtypes = [_p, _p, _p, _i64, _p]
        lib.fdbb_probe_pow.argtypes = [_p, _p, _p, _i64, _i, _p]
        _lib = lib
        if os.environ.get("FDBB_NO_TUNED_TABLE") != "1":
            from . import tune
            tune.apply_table()
    return _lib


def check(status: int) -> None:
    if status != OK:
        lib = library()
        msg = lib.fdbb_last_error().decode() or lib.fdbb_status_string(status).decode()
        raise FdbbError(status, f"fdbb status {status} ({lib.fdbb_status_string(status).decode()}): {msg}")


# ------------------------------------------------------------ marshalling
def dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return F64
    if t == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t}; use float64 or float32")


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dptr(t: torch.Tensor, name: str = "tensor") -> int:
    """Data pointer of a device tensor; a host tensor is refused here, since
    every entry point hands its pointers to kernels."""
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a tensor in device memory, got one on {t.device}")
    return t.data_ptr()


def _ptr(t):
    if t is None:
        return None
    return _dptr(t)


def _fields(t: torch.Tensor, fields: int, name: str):
    """(pointer, ld) of a field-set tensor (fields, n) with unit point stride."""
    if t.dim() != 2 or t.shape[0] != fields:
        raise ValueError(f"{name}: expected shape ({fields}, n), got {tuple(t.shape)}")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name}: points must be contiguous (stride 1)")
    ld = t.stride(0) if fields > 1 else max(t.shape[1], 1)
    return _dptr(t, name), ld


def _blocks(A: torch.Tensor, dim: int, name: str = "A"):
    K = dim + 2
    if A.dim() != 4 or A.shape[0] != dim or A.shape[2] != K or A.shape[3] != K:
        raise ValueError(f"{name}: expected shape ({dim}, n, {K}, {K}), got {tuple(A.shape)}")
    if A.stride(3) != 1 or A.stride(2) != K or A.stride(1) != K * K or A.stride(0) % (K * K):
        raise ValueError(f"{name}: blocks must be point-major row-major")
    return _dptr(A, name), A.stride(0) // (K * K)


def padded_ld(n: int) -> int:
    return max(ROW_ALIGN, (n + ROW_ALIGN - 1) // ROW_ALIGN * ROW_ALIGN)


def empty_fields(fields: int, n: int, dtype=torch.float64, device=None) -> torch.Tensor:
    """Uninitialised (fields, n) field set with rows padded to 64 elements."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    return torch.empty((fields, padded_ld(n)), dtype=dtype, device=device)[:, :n]


def empty_blocks(dim: int, n: int, dtype=torch.float64, device=None) -> torch.Tensor:
    K = dim + 2
    device = device or torch.device("cuda", torch.cuda.current_device())
    return torch.empty((dim, padded_ld(n), K, K), dtype=dtype, device=device)[:, :n]


def to_fields(x: torch.Tensor) -> torch.Tensor:
    """Copy a (fields, n) tensor into a padded field set on the same device."""
    out = empty_fields(x.shape[0], x.shape[1], x.dtype, x.device)
    out.copy_(x)
    return out


def _dim_of(U: torch.Tensor) -> int:
    dim = U.shape[0] - 2
    if dim not in (1, 2, 3):
        raise ValueError(f"a state has 3, 4 or 5 fields, got {U.shape[0]}")
    return dim


# ------------------------------------------------------------ C mirrors
def fdbb_cons2prim(dim, gamma, U, V, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    v, ldv = _fields(V, dim + 2, "V")
    n = U.shape[1] if n is None else n
    check(library().fdbb_cons2prim(dim, gamma, dtype_code(U.dtype), u, ldu, v, ldv, n, _stream(stream)))


def fdbb_prim2cons(dim, gamma, V, U, n=None, stream=None):
    v, ldv = _fields(V, dim + 2, "V")
    u, ldu = _fields(U, dim + 2, "U")
    n = V.shape[1] if n is None else n
    check(library().fdbb_prim2cons(dim, gamma, dtype_code(V.dtype), v, ldv, u, ldu, n, _stream(stream)))


def fdbb_velocity_magnitude2(dim, U, y, n=None, stream=None):
    if U.dim() != 2 or U.shape[0] < dim + 1:
        raise ValueError("U: expected a state of at least D+1 fields")
    if U.shape[1] > 1 and U.stride(1) != 1:
        raise ValueError("U: points must be contiguous (stride 1)")
    n = U.shape[1] if n is None else n
    check(library().fdbb_velocity_magnitude2(dim, dtype_code(U.dtype), _dptr(U, "U"), U.stride(0), _dptr(y, "y"),
                                             n, _stream(stream)))


def fdbb_eos(dim, gamma, U, p=None, c=None, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    n = U.shape[1] if n is None else n
    check(library().fdbb_eos(dim, gamma, dtype_code(U.dtype), u, ldu, _ptr(p), _ptr(c), n,
                             _stream(stream)))


def fdbb_flux(dim, gamma, U, F, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    f, ldf = _fields(F, (dim + 2) * dim, "F")
    n = U.shape[1] if n is None else n
    check(library().fdbb_flux(dim, gamma, dtype_code(U.dtype), u, ldu, f, ldf, n, _stream(stream)))


def fdbb_flux_direction(dim, direction, gamma, U, Fd, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    f, ldf = _fields(Fd, dim + 2, "Fd")
    n = U.shape[1] if n is None else n
    check(library().fdbb_flux_direction(dim, direction, gamma, dtype_code(U.dtype), u, ldu, f, ldf, n,
                                        _stream(stream)))


def fdbb_flux_jacobian(dim, gamma, U, A, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    a, lda = _blocks(A, dim)
    n = U.shape[1] if n is None else n
    check(library().fdbb_flux_jacobian(dim, gamma, dtype_code(U.dtype), u, ldu, a, lda, n,
                                       _stream(stream)))


def fdbb_riemann_invariants(dim, gamma, U, R, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    r, ldr = _fields(R, 2 * dim + 1, "R")
    n = U.shape[1] if n is None else n
    check(library().fdbb_riemann_invariants(dim, gamma, dtype_code(U.dtype), u, ldu, r, ldr, n,
                                            _stream(stream)))


def fdbb_cons2char(dim, direction, gamma, U, W, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    w, ldw = _fields(W, dim + 2, "W")
    n = U.shape[1] if n is None else n
    check(library().fdbb_cons2char(dim, direction, gamma, dtype_code(U.dtype), u, ldu, w, ldw, n,
                                   _stream(stream)))


def fdbb_char2cons(dim, direction, gamma, W, U, n=None, stream=None):
    w, ldw = _fields(W, dim + 2, "W")
    u, ldu = _fields(U, dim + 2, "U")
    n = W.shape[1] if n is None else n
    check(library().fdbb_char2cons(dim, direction, gamma, dtype_code(W.dtype), w, ldw, u, ldu, n,
                                   _stream(stream)))


def fdbb_euler_fused(dim, gamma, U, F=None, A=None, R=None, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    f, ldf = _fields(F, (dim + 2) * dim, "F") if F is not None else (None, 0)
    a, lda = _blocks(A, dim) if A is not None else (None, 0)
    r, ldr = _fields(R, 2 * dim + 1, "R") if R is not None else (None, 0)
    n = U.shape[1] if n is None else n
    check(library().fdbb_euler_fused(dim, gamma, dtype_code(U.dtype), u, ldu, f, ldf, a, lda, r, ldr,
                                     n, _stream(stream)))


def fdbb_flux_adjoint(dim, direction, gamma, U, Fbar, Ubar, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    fb, ldfb = _fields(Fbar, (dim + 2) * dim if direction < 0 else dim + 2, "Fbar")
    ub, ldub = _fields(Ubar, dim + 2, "Ubar")
    n = U.shape[1] if n is None else n
    check(library().fdbb_flux_adjoint(dim, direction, gamma, dtype_code(U.dtype), u, ldu, fb, ldfb,
                                      ub, ldub, n, _stream(stream)))


def fdbb_eigenvectors(dim, gamma, U, L=None, R=None, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    lp, ldl = _blocks(L, dim, "L") if L is not None else (None, 0)
    rp, ldr = _blocks(R, dim, "R") if R is not None else (None, 0)
    n = U.shape[1] if n is None else n
    check(library().fdbb_eigenvectors(dim, gamma, dtype_code(U.dtype), u, ldu, lp, ldl, rp, ldr, n,
                                      _stream(stream)))


def fdbb_char_apply(dim, direction, mode, gamma, U, X, Y, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    x, ldx = _fields(X, dim + 2, "X")
    y, ldy = _fields(Y, dim + 2, "Y")
    n = U.shape[1] if n is None else n
    check(library().fdbb_char_apply(dim, direction, mode, gamma, dtype_code(U.dtype), u, ldu, x, ldx, y, ldy,
                                    n, _stream(stream)))


def fdbb_roe_average(dim, gamma, UL, UR, Uh, n=None, stream=None):
    ul, ldl = _fields(UL, dim + 2, "UL")
    ur, ldr = _fields(UR, dim + 2, "UR")
    uh, ldh = _fields(Uh, dim + 2, "Uh")
    n = UL.shape[1] if n is None else n
    check(library().fdbb_roe_average(dim, gamma, dtype_code(UL.dtype), ul, ldl, ur, ldr, uh, ldh, n,
                                     _stream(stream)))


def fdbb_eos_pvt(dim, eos, params, U, p=None, c=None, T=None, n=None, stream=None):
    """General EOS entry: eos 'perfect_gas' (params c_p, c_v) or
    'stiffened_gas' (params gamma, p_inf, c_v)."""
    eos = EOS_IDS[eos] if isinstance(eos, str) else eos
    prm = (ctypes.c_double * 3)(*(list(params) + [0.0] * (3 - len(params))))
    u, ldu = _fields(U, dim + 2, "U")
    n = U.shape[1] if n is None else n
    ptr = [_ptr(t) for t in (p, c, T)]
    check(library().fdbb_eos_pvt(dim, eos, ctypes.cast(prm, _p), dtype_code(U.dtype), u, ldu, *ptr, n,
                                 _stream(stream)))


def fdbb_viscous_flux(dim, mu, kappa, U, G, gradT, Fv, n=None, stream=None):
    u, ldu = _fields(U, dim + 2, "U")
    g, ldg = _fields(G, dim * dim, "G")
    t, ldt = _fields(gradT, dim, "gradT")
    f, ldf = _fields(Fv, (dim + 2) * dim, "Fv")
    n = U.shape[1] if n is None else n
    check(library().fdbb_viscous_flux(dim, mu, kappa, dtype_code(U.dtype), u, ldu, g, ldg, t, ldt, f, ldf, n,
                                      _stream(stream)))


def fdbb_set_launch_config(op, dim, dtype, block, ppt, grid_cap=0, nontemporal=1):
    op = OPS[op] if isinstance(op, str) else op
    check(library().fdbb_set_launch_config(op, dim, dtype, block, ppt, grid_cap, nontemporal))


def fdbb_get_launch_config(op, dim, dtype):
    """(block, ppt, grid_cap, nontemporal) of (op, dim, dtype)."""
    op = OPS[op] if isinstance(op, str) else op
    b, p, g, t = _i(), _i(), _i(), _i()
    check(library().fdbb_get_launch_config(op, dim, dtype, ctypes.byref(b), ctypes.byref(p),
                                           ctypes.byref(g), ctypes.byref(t)))
    return b.value, p.value, g.value, t.value


def fdbb_set_small_launch_config(op, dim, dtype, max_n, block=256, ppt=1, grid_cap=0, nontemporal=1):
    """Configuration for calls of at most max_n points (max_n 0 removes it)."""
    op = OPS[op] if isinstance(op, str) else op
    check(library().fdbb_set_small_launch_config(op, dim, dtype, max_n, block, ppt, grid_cap, nontemporal))


def fdbb_get_small_launch_config(op, dim, dtype):
    """(max_n, block, ppt, grid_cap, nontemporal); max_n 0 when none is set."""
    op = OPS[op] if isinstance(op, str) else op
    m = _i64()
    b, p, g, t = _i(), _i(), _i(), _i()
    check(library().fdbb_get_small_launch_config(op, dim, dtype, ctypes.byref(m), ctypes.byref(b),
                                                 ctypes.byref(p), ctypes.byref(g), ctypes.byref(t)))
    return m.value, b.value, p.value, g.value, t.value


def fdbb_launch_config_for(op, dim, dtype, n):
    """(block, ppt, grid_cap, nontemporal) a call of n points launches with."""
    op = OPS[op] if isinstance(op, str) else op
    b, p, g, t = _i(), _i(), _i(), _i()
    check(library().fdbb_launch_config_for(op, dim, dtype, n, ctypes.byref(b), ctypes.byref(p),
                                           ctypes.byref(g), ctypes.byref(t)))
    return b.value, p.value, g.value, t.value


def fdbb_set_server_batch_config(block, ppt=1, grid_per_cu=0, nontemporal=1):
    """Batch configuration of the request server's launches (block 0 removes it)."""
    check(library().fdbb_set_server_batch_config(block, ppt, grid_per_cu, nontemporal))


def fdbb_get_server_batch_config():
    """(block, ppt, grid_per_cu, nontemporal) the request server launches with."""
    b, p, g, t = _i(), _i(), _i(), _i()
    check(library().fdbb_get_server_batch_config(ctypes.byref(b), ctypes.byref(p), ctypes.byref(g),
                                                 ctypes.byref(t)))
    return b.value, p.value, g.value, t.value


def fdbb_set_batch_config(dtype, block, ppt, grid_per_cu=0, nontemporal=1):
    check(library().fdbb_set_batch_config(dtype, block, ppt, grid_per_cu, nontemporal))


def fdbb_get_batch_config(dtype):
    """(block, ppt, grid_per_cu, nontemporal) that batch plans created with
    block 0 use for storage type `dtype`."""
    b, p, g, t = _i(), _i(), _i(), _i()
    check(library().fdbb_get_batch_config(dtype, ctypes.byref(b), ctypes.byref(p), ctypes.byref(g),
                                          ctypes.byref(t)))
    return b.value, p.value, g.value, t.value


def fdbb_kernel_info(op, dim, dtype, ppt, nontemporal=1):
    """(vector registers, private spill bytes) per thread of a kernel."""
    op = OPS[op] if isinstance(op, str) else op
    v, b = _i(), _i()
    check(library().fdbb_kernel_info(op, dim, dtype, ppt, nontemporal, ctypes.byref(v), ctypes.byref(b)))
    return v.value, b.value


def fdbb_version() -> int:
    return library().fdbb_version()


# ------------------------------------------------------------ allocating helpers
def cons2prim(U, gamma=1.4, stream=None):
    dim = _dim_of(U)
    V = empty_fields(dim + 2, U.shape[1], U.dtype, U.device)
    fdbb_cons2prim(dim, gamma, U, V, stream=stream)
    return V


def prim2cons(V, gamma=1.4, stream=None):
    dim = _dim_of(V)
    U = empty_fields(dim + 2, V.shape[1], V.dtype, V.device)
    fdbb_prim2cons(dim, gamma, V, U, stream=stream)
    return U


def velocity_magnitude2(U, stream=None):
    dim = _dim_of(U)
    n = U.shape[1]
    y = torch.empty(max(n, 1), dtype=U.dtype, device=U.device)[:n]
    fdbb_velocity_magnitude2(dim, U, y, stream=stream)
    return y


def eos(U, gamma=1.4, stream=None):
    dim = _dim_of(U)
    n = U.shape[1]
    p = torch.empty(max(n, 1), dtype=U.dtype, device=U.device)[:n]
    c = torch.empty(max(n, 1), dtype=U.dtype, device=U.device)[:n]
    fdbb_eos(dim, gamma, U, p, c, stream=stream)
    return p, c


def flux(U, gamma=1.4, stream=None, direction=None):
    """The flux tensor (K*D fields), or F_direction alone (K fields)."""
    dim = _dim_of(U)
    if direction is not None:
        Fd = empty_fields(dim + 2, U.shape[1], U.dtype, U.device)
        fdbb_flux_direction(dim, direction, gamma, U, Fd, stream=stream)
        return Fd
    F = empty_fields((dim + 2) * dim, U.shape[1], U.dtype, U.device)
    fdbb_flux(dim, gamma, U, F, stream=stream)
    return F


def flux_jacobian(U, gamma=1.4, stream=None):
    dim = _dim_of(U)
    A = empty_blocks(dim, U.shape[1], U.dtype, U.device)
    fdbb_flux_jacobian(dim, gamma, U, A, stream=stream)
    return A


def riemann_invariants(U, gamma=1.4, stream=None):
    dim = _dim_of(U)
    R = empty_fields(2 * dim + 1, U.shape[1], U.dtype, U.device)
    fdbb_riemann_invariants(dim, gamma, U, R, stream=stream)
    return R


def cons2char(U, direction, gamma=1.4, stream=None):
    dim = _dim_of(U)
    W = empty_fields(dim + 2, U.shape[1], U.dtype, U.device)
    fdbb_cons2char(dim, direction, gamma, U, W, stream=stream)
    return W


def char2cons(W, direction, gamma=1.4, stream=None):
    dim = _dim_of(W)
    U = empty_fields(dim + 2, W.shape[1], W.dtype, W.device)
    fdbb_char2cons(dim, direction, gamma, W, U, stream=stream)
    return U


def euler_fused(U, gamma=1.4, flux=True, jacobian=True, riemann=True, stream=None):
    dim = _dim_of(U)
    n = U.shape[1]
    F = empty_fields((dim + 2) * dim, n, U.dtype, U.device) if flux else None
    A = empty_blocks(dim, n, U.dtype, U.device) if jacobian else None
    R = empty_fields(2 * dim + 1, n, U.dtype, U.device) if riemann else None
    fdbb_euler_fused(dim, gamma, U, F, A, R, stream=stream)
    return F, A, R


def flux_adjoint(U, Fbar, gamma=1.4, direction=-1, stream=None):
    dim = _dim_of(U)
    Ub = empty_fields(dim + 2, U.shape[1], U.dtype, U.device)
    fdbb_flux_adjoint(dim, direction, gamma, U, Fbar, Ub, stream=stream)
    return Ub


# ------------------------------------------------------------ streaming probes
def probe_copy(src: torch.Tensor, dst: torch.Tensor, grid: int = 0, stream=None):
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    check(library().fdbb_probe_copy(_dptr(src), _dptr(dst), nbytes // 16 * 16, grid,
                                    _stream(stream)))


def probe_write(dst: torch.Tensor, pattern: int = 0x3FF0000000000000, grid: int = 0, stream=None):
    nbytes = dst.numel() * dst.element_size()
    check(library().fdbb_probe_write(_dptr(dst), nbytes // 16 * 16, pattern, grid, _stream(stream)))


def probe_fused_stores(F_: torch.Tensor, R: torch.Tensor, A: torch.Tensor, n: int, stream=None):
    """The fused 3D pass's stores alone (constant values, same layout and
    order): F (15, n), R (7, n), A (3, n, 5, 5), FP64, n a multiple of 512."""
    check(library().fdbb_probe_fused_stores(_dptr(F_), _dptr(R), _dptr(A), n, _stream(stream)))


def probe_pow(x: torch.Tensor, y: torch.Tensor, fp32_form: bool, stream=None) -> torch.Tensor:
    """x ** y elementwise on the device, by the power the building blocks
    use: the library's exp and log (FP64 storage), or the base-2 form of the
    FP32-storage kernels.  x and y: contiguous FP64 device tensors of one
    shape."""
    if x.dtype != torch.float64 or y.dtype != torch.float64 or x.shape != y.shape:
        raise ValueError("probe_pow takes two FP64 tensors of one shape")
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("probe_pow takes contiguous tensors")
    out = torch.empty_like(x)
    check(library().fdbb_probe_pow(_dptr(x), _dptr(y), _dptr(out), x.numel(),
                                   1 if fp32_form else 0, _stream(stream)))
    return out


def probe_read(src: torch.Tensor, sink: torch.Tensor, grid: int = 0, stream=None):
    nbytes = src.numel() * src.element_size()
    check(library().fdbb_probe_read(_dptr(src), nbytes // 16 * 16, _dptr(sink), grid,
                                    _stream(stream)))


def eigenvectors(U, gamma=1.4, left=True, right=True, stream=None):
    """(L, R) eigenvector blocks of every direction, (D, n, K, K) each."""
    dim = _dim_of(U)
    L = empty_blocks(dim, U.shape[1], U.dtype, U.device) if left else None
    R = empty_blocks(dim, U.shape[1], U.dtype, U.device) if right else None
    fdbb_eigenvectors(dim, gamma, U, L, R, stream=stream)
    return L, R


def viscous_flux(U, G, gradT, mu, kappa, stream=None):
    """Viscous flux tensor (K*D fields, flux tensor layout) of the state U
    with velocity gradient G (D*D fields) and temperature gradient gradT."""
    dim = _dim_of(U)
    Fv = empty_fields((dim + 2) * dim, U.shape[1], U.dtype, U.device)
    fdbb_viscous_flux(dim, mu, kappa, U, G, gradT, Fv, stream=stream)
    return Fv


def eos_pvt(U, eos="perfect_gas", params=(3.5, 2.5), stream=None):
    """(p, c, T) of the conservative state U under a runtime-selected EOS."""
    dim = _dim_of(U)
    p, c, T = (torch.empty(U.shape[1], dtype=U.dtype, device=U.device) for _ in range(3))
    fdbb_eos_pvt(dim, eos, params, U, p, c, T, stream=stream)
    return p, c, T


def roe_average(UL, UR, gamma=1.4, stream=None):
    """Roe-averaged conservative state between UL and UR."""
    dim = _dim_of(UL)
    Uh = empty_fields(dim + 2, UL.shape[1], UL.dtype, UL.device)
    fdbb_roe_average(dim, gamma, UL, UR, Uh, stream=stream)
    return Uh


def char_apply(U, X, direction, mode=0, gamma=1.4, stream=None):
    """L_dir(U) X (mode 0) or R_dir(U) X (mode 1)."""
    dim = _dim_of(U)
    Y = empty_fields(dim + 2, U.shape[1], U.dtype, U.device)
    fdbb_char_apply(dim, direction, mode, gamma, U, X, Y, stream=stream)
    return Y
