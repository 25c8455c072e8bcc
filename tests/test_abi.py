"""The C ABI without a GPU: the library loads, exports every symbol that
include/fdbb.h declares, and rejects bad arguments on the host before any
HIP call.  No call here reaches a kernel launch."""
import ctypes
import glob
import os
import re

import pytest

from conftest import ROOT
from paper_1809_09851_amd import fdbb as F

HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_symbols():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(fdbb_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return F.library()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(HEADERS) >= 2
    assert len(names) >= 23
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_required_entry_points_present():
    names = declared_symbols()
    for n in ("fdbb_cons2prim", "fdbb_prim2cons", "fdbb_eos", "fdbb_flux", "fdbb_flux_jacobian",
              "fdbb_riemann_invariants"):
        assert n in names


def test_status_strings_and_version(lib):
    assert lib.fdbb_status_string(0) == b"ok"
    assert lib.fdbb_status_string(F.EALIAS) == b"input and output overlap"
    assert lib.fdbb_version() >= 100


# Fake device addresses: validation rejects these calls before any HIP call.
A0 = 0x10000000
B0 = 0x20000000


def flux(dim=3, gamma=1.4, dtype=0, U=A0, ldU=128, Fp=B0, ldF=128, n=100):
    return F.library().fdbb_flux(dim, gamma, dtype, U, ldU, Fp, ldF, n, None)


@pytest.mark.parametrize("kw,status", [
    (dict(dim=0), F.EINVAL), (dict(dim=4), F.EINVAL),
    (dict(gamma=1.0), F.EINVAL), (dict(gamma=0.5), F.EINVAL),
    (dict(gamma=float("nan")), F.EINVAL), (dict(gamma=float("inf")), F.EINVAL),
    (dict(dtype=2), F.EINVAL), (dict(n=-1), F.EINVAL),
    (dict(U=0), F.EINVAL), (dict(Fp=0), F.EINVAL),
    (dict(ldU=99), F.EINVAL), (dict(ldF=50), F.EINVAL),
    (dict(U=A0 + 4), F.EALIGN), (dict(Fp=B0 + 2, dtype=1), F.EALIGN),
    (dict(Fp=A0 + 8 * 64), F.EALIAS),             # F starts inside U
    (dict(Fp=A0, ldF=128), F.EALIAS),             # same base as U
])
def test_flux_rejects(kw, status):
    assert flux(**kw) == status
    assert F.library().fdbb_last_error() != b""


def test_zero_points_is_a_noop():
    # n == 0 returns before any HIP call, even with NULL pointers.
    assert flux(n=0, U=0, Fp=0) == F.OK
    lib = F.library()
    assert lib.fdbb_cons2prim(2, 1.4, 0, None, 0, None, 0, 0, None) == F.OK


def test_inplace_rules():
    lib = F.library()
    # partial overlap of a K -> K transform: rejected
    assert lib.fdbb_cons2prim(2, 1.4, 0, A0, 128, A0 + 8, 128, 100, None) == F.EALIAS
    # same base, different ld: rejected
    assert lib.fdbb_prim2cons(2, 1.4, 0, A0, 128, A0, 256, 100, None) == F.EALIAS
    # exact in place is not allowed for ops whose output is not the state
    assert lib.fdbb_riemann_invariants(1, 1.4, 0, A0, 128, A0, 128, 100, None) == F.EALIAS


def test_eos_and_fused_nullable_outputs():
    lib = F.library()
    assert lib.fdbb_eos(3, 1.4, 0, A0, 128, None, None, 100, None) == F.EINVAL
    assert lib.fdbb_eos(3, 1.4, 0, A0, 128, A0 + 8, None, 100, None) == F.EALIAS
    assert lib.fdbb_euler_fused(3, 1.4, 0, A0, 128, None, 0, None, 0, None, 0, 100, None) == F.EINVAL
    # F of D = 2 spans (7 * 128 + 100) doubles; A starting inside it overlaps
    assert lib.fdbb_euler_fused(2, 1.4, 0, A0, 128, B0, 128, B0 + 8 * 64, 128, None, 0, 100,
                                None) == F.EALIAS


def test_direction_checks():
    lib = F.library()
    assert lib.fdbb_cons2char(2, 2, 1.4, 0, A0, 128, B0, 128, 100, None) == F.EINVAL
    assert lib.fdbb_char2cons(1, -1, 1.4, 0, A0, 128, B0, 128, 100, None) == F.EINVAL
    assert lib.fdbb_flux_adjoint(3, 3, 1.4, 0, A0, 128, B0, 128, A0 + 10**7, 128, 100, None) == F.EINVAL
    assert lib.fdbb_flux_adjoint(3, -2, 1.4, 0, A0, 128, B0, 128, A0 + 10**7, 128, 100, None) == F.EINVAL


def test_flux_direction_checks():
    lib = F.library()
    assert lib.fdbb_flux_direction(3, 3, 1.4, 0, A0, 128, B0, 128, 100, None) == F.EINVAL
    assert lib.fdbb_flux_direction(2, -1, 1.4, 0, A0, 128, B0, 128, 100, None) == F.EINVAL
    assert lib.fdbb_flux_direction(3, 0, 1.4, 0, A0, 128, B0, 64, 100, None) == F.EINVAL  # ld < n
    assert lib.fdbb_flux_direction(3, 1, 1.4, 0, A0, 128, A0 + 8 * 64, 128, 100, None) == F.EALIAS
    assert lib.fdbb_flux_direction(1, 0, 1.4, 0, A0, 128, B0, 128, 0, None) == F.OK


def test_noalloc_batch_rejects_before_any_hip_call():
    lib = F.library()
    t = (F.Task * 1)()
    t[0].op, t[0].dim, t[0].dtype, t[0].gamma, t[0].n = F.OPS["flux"], 3, 0, 1.4, 0
    assert lib.fdbb_batch_run_noalloc(t, 1025, 256, 1, 0, 1, None) == F.EINVAL
    assert b"1024" in lib.fdbb_last_error()
    assert lib.fdbb_batch_run_noalloc(t, -1, 256, 1, 0, 1, None) == F.EINVAL
    assert lib.fdbb_batch_run_noalloc(t, 1, 512, 1, 0, 1, None) == F.EINVAL
    assert lib.fdbb_batch_run_noalloc(t, 1, 256, 3, 0, 1, None) == F.EINVAL
    assert lib.fdbb_batch_run_noalloc(None, 2, 256, 1, 0, 1, None) == F.EINVAL


def test_batch_config_table():
    lib = F.library()
    old = F.fdbb_get_batch_config(F.F64)
    try:
        assert lib.fdbb_set_batch_config(F.F64, 128, 4, 8, 2) == F.OK
        assert F.fdbb_get_batch_config(F.F64) == (128, 4, 8, 2)
        # out of range, or 3D FP64 Jacobian staging beyond the LDS
        assert lib.fdbb_set_batch_config(F.F64, 320, 1, 0, 1) == F.EINVAL
        assert lib.fdbb_set_batch_config(F.F64, 96, 1, 0, 1) == F.EINVAL
        assert lib.fdbb_set_batch_config(F.F64, 64, 3, 0, 1) == F.EINVAL
        assert lib.fdbb_set_batch_config(F.F64, 64, 1, 0, 3) == F.EINVAL
        assert lib.fdbb_set_batch_config(F.F64, 64, 1, -1, 1) == F.EINVAL
        assert lib.fdbb_set_batch_config(F.F64, 256, 4, 0, 1) == F.EINVAL
        assert lib.fdbb_set_batch_config(F.F32, 256, 4, 0, 1) == F.OK  # half the bytes fit
        assert lib.fdbb_set_batch_config(5, 64, 1, 0, 1) == F.EINVAL
        assert F.fdbb_get_batch_config(F.F64) == (128, 4, 8, 2)
    finally:
        F.fdbb_set_batch_config(F.F64, *old)


def test_server_batch_config():
    lib = F.library()
    old64 = F.fdbb_get_batch_config(F.F64)
    saved = F.fdbb_get_server_batch_config()
    try:
        F.fdbb_set_server_batch_config(0)                     # no entry: the FP64 batch configuration
        assert F.fdbb_get_server_batch_config() == old64
        assert lib.fdbb_set_server_batch_config(256, 1, 8, 1) == F.OK
        assert F.fdbb_get_server_batch_config() == (256, 1, 8, 1)
        assert F.fdbb_get_batch_config(F.F64) == old64        # the batch table is not touched
        assert lib.fdbb_set_server_batch_config(256, 4, 0, 1) == F.EINVAL   # 3D FP64 staging beyond LDS
        assert lib.fdbb_set_server_batch_config(96, 1, 0, 1) == F.EINVAL
        assert lib.fdbb_set_server_batch_config(64, 3, 0, 1) == F.EINVAL
        assert lib.fdbb_set_server_batch_config(64, 1, 1025, 1) == F.EINVAL
        assert lib.fdbb_set_server_batch_config(64, 1, 0, 3) == F.EINVAL
        assert F.fdbb_get_server_batch_config() == (256, 1, 8, 1)
        F.fdbb_set_server_batch_config(0)
        assert F.fdbb_get_server_batch_config() == old64
    finally:
        F.fdbb_set_server_batch_config(*saved)


def test_eigen_and_char_apply_checks():
    lib = F.library()
    assert lib.fdbb_eigenvectors(3, 1.4, 0, A0, 128, None, 0, None, 0, 100, None) == F.EINVAL
    assert lib.fdbb_eigenvectors(2, 1.4, 0, A0, 128, A0, 128, None, 0, 100, None) == F.EALIAS
    assert lib.fdbb_char_apply(2, 2, 0, 1.4, 0, A0, 128, B0, 128, B0 + 10**6, 128, 100, None) == F.EINVAL
    assert lib.fdbb_char_apply(2, 0, 2, 1.4, 0, A0, 128, B0, 128, B0 + 10**6, 128, 100, None) == F.EINVAL
    assert lib.fdbb_char_apply(2, 0, 0, 1.4, 0, A0, 128, B0, 128, B0 + 8, 128, 100, None) == F.EALIAS


def test_roe_average_checks():
    lib = F.library()
    assert lib.fdbb_roe_average(4, 1.4, 0, A0, 128, B0, 128, A0 + 10**7, 128, 100, None) == F.EINVAL
    assert lib.fdbb_roe_average(2, 1.0, 0, A0, 128, B0, 128, A0 + 10**7, 128, 100, None) == F.EINVAL
    assert lib.fdbb_roe_average(2, 1.4, 0, None, 128, B0, 128, A0 + 10**7, 128, 100, None) == F.EINVAL
    # the output may not partly overlap either input
    assert lib.fdbb_roe_average(2, 1.4, 0, A0, 128, B0, 128, A0 + 8, 128, 100, None) == F.EALIAS
    assert lib.fdbb_roe_average(2, 1.4, 0, A0, 128, B0, 128, B0 + 8, 128, 100, None) == F.EALIAS
    assert lib.fdbb_roe_average(2, 1.4, 0, A0, 128, B0, 128, B0, 64, 100, None) == F.EINVAL
    t = F.Task()
    t.op, t.dim, t.dtype, t.gamma, t.n = F.OPS["roe_average"], 3, 1, 1.4, 100
    t.in0, t.ld_in0, t.in1, t.ld_in1, t.out0, t.ld_out0 = A0, 128, B0, 128, B0, 128
    assert lib.fdbb_task_check(ctypes.byref(t)) == F.OK  # in place over UR


def test_eos_pvt_checks():
    lib = F.library()
    D3 = ctypes.c_double * 3

    def call(eos, prm, p=B0, c=None, T=None, dim=3, n=100):
        return lib.fdbb_eos_pvt(dim, eos, ctypes.cast(D3(*prm), ctypes.c_void_p), 0, A0, 128, p, c, T, n, None)

    assert call(0, (2.5, 3.5, 0)) == F.EINVAL  # c_p < c_v
    assert call(0, (3.5, 0.0, 0)) == F.EINVAL
    assert call(1, (1.0, 0.1, 1.0)) == F.EINVAL  # gamma <= 1
    assert call(1, (4.4, -1.0, 1.0)) == F.EINVAL  # p_inf < 0
    assert call(1, (4.4, 0.1, 0.0)) == F.EINVAL  # c_v <= 0
    assert call(2, (4.4, 0.1, 1.0)) == F.EINVAL  # unknown id
    assert call(1, (4.4, 0.1, 1.0), p=None) == F.EINVAL  # no output
    assert call(1, (4.4, 0.1, 1.0), dim=4) == F.EINVAL
    assert call(1, (4.4, 0.1, 1.0), p=A0 + 8) == F.EALIAS
    assert lib.fdbb_eos_pvt(3, 0, None, 0, A0, 128, B0, None, None, 100, None) == F.EINVAL
    t = F.Task()
    t.op, t.dim, t.dtype, t.gamma, t.n = F.OPS["eos_pvt"], 3, 0, 1.4, 100
    t.in0, t.ld_in0, t.out0 = A0, 128, B0
    assert lib.fdbb_task_check(ctypes.byref(t)) == F.EINVAL


def test_viscous_flux_checks():
    lib = F.library()
    C0 = 0x30000000
    D0 = 0x40000000

    def call(mu=0.1, kappa=0.1, dim=3, G=B0, out=D0, n=100):
        return lib.fdbb_viscous_flux(dim, mu, kappa, 0, A0, 128, G, 128, C0, 128, out, 128, n, None)

    assert call(mu=-1.0) == F.EINVAL
    assert call(kappa=float("nan")) == F.EINVAL
    assert call(dim=0) == F.EINVAL
    assert call(G=None) == F.EINVAL
    assert call(out=C0 + 8) == F.EALIAS  # output overlaps gradT
    assert call(out=A0) == F.EALIAS  # no in-place form
    t = F.Task()
    t.op, t.dim, t.dtype, t.gamma, t.n = F.OPS["viscous_flux"], 3, 0, 1.4, 100
    t.in0, t.ld_in0, t.out0, t.ld_out0 = A0, 128, D0, 128
    assert lib.fdbb_task_check(ctypes.byref(t)) == F.EINVAL


def test_server_rejects_bad_arguments():
    lib = F.library()
    h = ctypes.c_void_p()
    assert lib.fdbb_server_create(0, 4, 64, 1e9, 0, ctypes.byref(h)) == F.EINVAL
    assert lib.fdbb_server_create(1 << 30, 0, 64, 1e9, 0, ctypes.byref(h)) == F.EINVAL
    assert lib.fdbb_server_create(1 << 30, 4, 0, 1e9, 0, ctypes.byref(h)) == F.EINVAL
    assert lib.fdbb_server_create(1 << 30, 4, 64, 0.0, 0, ctypes.byref(h)) == F.EINVAL
    assert lib.fdbb_server_create(1 << 30, 4, 64, 1e9, 2, ctypes.byref(h)) == F.EINVAL
    assert not h.value


def test_task_check_validates_without_a_gpu():
    t = F.Task()
    t.op, t.dim, t.dtype, t.gamma, t.n = 3, 3, 0, 1.4, 100
    t.in0, t.ld_in0, t.out0, t.ld_out0 = A0, 128, B0, 128
    assert F.library().fdbb_task_check(ctypes.byref(t)) == F.OK
    t.out0 = A0 + 8
    assert F.library().fdbb_task_check(ctypes.byref(t)) == F.EALIAS
    t.dim = 5
    assert F.library().fdbb_task_check(ctypes.byref(t)) == F.EINVAL


def test_points_per_call_bound():
    """Calls and tasks take fewer than 2^31 points (64-bit offsets and
    leading dimensions either way)."""
    lib = F.library()
    t = F.Task()
    big = 1 << 31
    t.op, t.dim, t.dtype, t.gamma = 0, 1, 1, 1.4
    t.in0, t.out0 = A0, A0 + 4 * 3 * (big + 64)
    t.ld_in0 = t.ld_out0 = big + 64
    t.n = big - 1
    assert lib.fdbb_task_check(ctypes.byref(t)) == F.OK
    t.n = big
    assert lib.fdbb_task_check(ctypes.byref(t)) == F.EINVAL
    assert lib.fdbb_cons2prim(1, 1.4, 1, A0, big + 64, t.out0, big + 64, big, None) == F.EINVAL
    assert b"2^31" in lib.fdbb_last_error()


def test_launch_config_table():
    lib = F.library()
    assert lib.fdbb_set_launch_config(3, 3, 0, 100, 1, 0, 1) == F.EINVAL   # not a multiple of 64
    assert lib.fdbb_set_launch_config(3, 3, 0, 256, 3, 0, 1) == F.EINVAL   # ppt
    assert lib.fdbb_set_launch_config(3, 3, 0, 2048, 1, 0, 1) == F.EINVAL
    assert lib.fdbb_set_launch_config(3, 3, 0, 256, 1, 0, 2) == F.EINVAL   # store mode
    assert lib.fdbb_set_launch_config(99, 3, 0, 256, 1, 0, 1) == F.EINVAL
    old = F.fdbb_get_launch_config("flux", 3, 0)
    F.fdbb_set_launch_config("flux", 3, 0, 512, 4, 1000, 0)
    assert F.fdbb_get_launch_config("flux", 3, 0) == (512, 4, 1000, 0)
    F.fdbb_set_launch_config("flux", 3, 0, *old)
    assert F.fdbb_get_launch_config("flux", 3, 0) == old


def test_small_launch_config_selects_by_size(lib):
    op, dim, dt = "cons2prim", 1, F.F64
    code = F.OPS[op]
    large = F.fdbb_get_launch_config(op, dim, dt)
    saved = F.fdbb_get_small_launch_config(op, dim, dt)
    assert lib.fdbb_set_small_launch_config(code, dim, dt, -1, 256, 1, 0, 1) == F.EINVAL
    assert lib.fdbb_set_small_launch_config(code, dim, dt, 100, 100, 1, 0, 1) == F.EINVAL
    assert lib.fdbb_set_small_launch_config(code, dim, dt, 100, 256, 3, 0, 1) == F.EINVAL
    assert lib.fdbb_set_small_launch_config(99, dim, dt, 100, 256, 1, 0, 1) == F.EINVAL
    assert lib.fdbb_set_small_launch_config(F.OPS["fused"], 3, dt, 100, 512, 1, 0, 1) == F.EINVAL  # staged
    assert lib.fdbb_launch_config_for(code, dim, dt, -1, None, None, None, None) == F.EINVAL
    try:
        F.fdbb_set_small_launch_config(op, dim, dt, 0)
        assert F.fdbb_get_small_launch_config(op, dim, dt) == (0, *large)
        for n in (0, 1, 1 << 20, 1 << 30):
            assert F.fdbb_launch_config_for(op, dim, dt, n) == large
        small = (128, 4, 0, 0) if large != (128, 4, 0, 0) else (64, 2, 0, 1)
        F.fdbb_set_small_launch_config(op, dim, dt, 1 << 21, *small)
        assert F.fdbb_get_small_launch_config(op, dim, dt) == (1 << 21, *small)
        assert F.fdbb_launch_config_for(op, dim, dt, 1) == small
        assert F.fdbb_launch_config_for(op, dim, dt, 1 << 21) == small
        assert F.fdbb_launch_config_for(op, dim, dt, (1 << 21) + 1) == large
        # other (op, dim, dtype) keys are untouched
        assert F.fdbb_launch_config_for(op, 2, dt, 1) == F.fdbb_get_launch_config(op, 2, dt)
        assert F.fdbb_launch_config_for(op, dim, F.F32, 1) == F.fdbb_get_launch_config(op, dim, F.F32)
        F.fdbb_set_small_launch_config(op, dim, dt, 0)
        assert F.fdbb_launch_config_for(op, dim, dt, 1) == large
    finally:
        F.fdbb_set_small_launch_config(op, dim, dt, *saved) if saved[0] else \
            F.fdbb_set_small_launch_config(op, dim, dt, 0)


def test_kernel_info_rejects_bad_arguments():
    lib = F.library()
    assert lib.fdbb_kernel_info(3, 3, 0, 3, 1, None, None) == F.EINVAL
    assert lib.fdbb_kernel_info(3, 0, 0, 1, 1, None, None) == F.EINVAL
    assert lib.fdbb_kernel_info(3, 3, 0, 1, 2, None, None) == F.EINVAL


def test_batch_plan_rejects_bad_tasks():
    lib = F.library()
    plan = ctypes.c_void_p()
    t = (F.Task * 1)()
    t[0].op, t[0].dim, t[0].dtype, t[0].gamma, t[0].n = 3, 4, 0, 1.4, 10
    assert lib.fdbb_batch_plan_create(t, 1, 1, 256, 1, 0, 1, ctypes.byref(plan)) == F.EINVAL
    assert lib.fdbb_batch_plan_create(t, 1, 0, 256, 1, 0, 1, ctypes.byref(plan)) == F.EINVAL
    assert lib.fdbb_batch_plan_create(t, 1, 1, 100, 1, 0, 1, ctypes.byref(plan)) == F.EINVAL
    assert not plan.value


def test_fused_store_probe_checks():
    lib = F.library()
    assert lib.fdbb_probe_fused_stores(A0, B0, A0 + (1 << 30), 1000, None) == F.EINVAL  # not a multiple of 512
    assert lib.fdbb_probe_fused_stores(A0 + 8, B0, A0 + (1 << 30), 1024, None) == F.EINVAL  # misaligned
    assert lib.fdbb_probe_fused_stores(A0, B0, A0 + (1 << 30), 0, None) == F.EINVAL


def test_pow_probe_checks():
    lib = F.library()
    big = A0 + (1 << 30)
    assert lib.fdbb_probe_pow(A0, B0, big, -1, 1, None) == F.EINVAL
    assert lib.fdbb_probe_pow(A0 + 4, B0, big, 16, 1, None) == F.EINVAL  # misaligned
    assert lib.fdbb_probe_pow(None, B0, big, 16, 0, None) == F.EINVAL
    assert lib.fdbb_probe_pow(A0, B0, None, 16, 0, None) == F.EINVAL
    assert lib.fdbb_probe_pow(A0, B0, big, 0, 1, None) == F.OK  # nothing to do, no launch


def test_binding_refuses_host_tensors():
    """Host tensors are refused before any pointer reaches the library."""
    import torch
    U = torch.ones(5, 64, dtype=torch.float64)
    V = torch.empty_like(U)
    with pytest.raises(ValueError, match="device memory"):
        F.fdbb_cons2prim(3, 1.4, U, V)
    with pytest.raises(ValueError, match="device memory"):
        F.probe_pow(U[0].contiguous(), U[1].contiguous(), True)


def test_headers_are_plain_c_and_cpp(tmp_path):
    """The public headers compile as strict C99 and as C++11, so that a C
    caller needs nothing but the headers and libfdbb.so."""
    import subprocess
    src = tmp_path / "use.c"
    src.write_text('#include "fdbb.h"\n#include "fdbb_server.h"\n#include "fdbb_probe.h"\n'
                   "int main(void) { return FDBB_OK; }\n")
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                    "-I", inc, str(src)], check=True)
    subprocess.run(["g++", "-std=c++11", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I", inc,
                    "-x", "c++", str(src)], check=True)
