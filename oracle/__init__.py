"""Plain CPU oracle for the compressible-Euler building blocks of FDBB.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
never loads it and shares no code with it.

The arithmetic lives in ``fdbb_oracle.c`` (plain single-threaded C, FP64,
compiled with ``-O2 -ffp-contract=off``).  This module only builds that file
with gcc and marshals numpy arrays into it; it holds none of the method's
arithmetic.  Every function takes and returns SoA arrays of shape
``(fields, n)`` (C-contiguous float64), matching the C layout with ld = n.

Sections cited below are those of the FDBB paper:
  * cons2prim / prim2cons       -- Sec. 2.2, "Variables" (conversion figure)
  * v_mag2                      -- Sec. 3, Eq. 2 (micro-benchmark expression)
  * eos                         -- Sec. 2.2, "Equations of state" (p_rhoe)
  * flux                        -- Sec. 2.2, "Inviscid Fluxes" (flux tensor)
  * flux_jacobian               -- Fig. 1 / Sec. 2.2 (derivative of the above)
  * riemann_invariants, cons2char, char2cons -- Fig. 1 (named building blocks)
  * flux_adjoint                -- transpose of the flux Jacobians
  * eigenvectors, char_apply    -- characteristic decomposition of A_d (Fig. 1,
                                   "characteristic variables", linearised)
  * roe_average                 -- Roe's averaged state between two states, the
                                   linearisation point of that decomposition
  * eos_pvt                     -- Sec. 2.2, "Equations of state": p(rho, e),
                                   T(rho, e) and c of a runtime-selected EOS
  * viscous_flux                -- Fig. 1, "viscous fluxes" (Navier-Stokes form)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "fdbb_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle_fdbb.so")

_i64 = ctypes.c_int64
_dp = ctypes.c_void_p
_int = ctypes.c_int
_dbl = ctypes.c_double

CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def compile_source(src: str, out: str) -> str:
    """Compile one oracle source file into a shared library with gcc."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIBRARY):
        compile_source(SOURCE, LIBRARY)
    return LIBRARY


def _soa(a: np.ndarray, fields: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != fields:
        raise ValueError(f"expected an array of shape ({fields}, n), got {a.shape}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _check(rc: int):
    if rc != 0:
        raise ValueError("oracle rejected dim or direction")


class Oracle:
    """numpy front end over one compiled copy of ``fdbb_oracle.c``."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        sig = [_int, _dbl, _dp, _i64, _dp, _i64, _i64]
        for name in ("oracle_cons2prim", "oracle_prim2cons", "oracle_flux",
                     "oracle_flux_jacobian", "oracle_riemann_invariants"):
            getattr(lib, name).argtypes = sig
            getattr(lib, name).restype = _int
        lib.oracle_v_mag2.argtypes = [_int, _dp, _i64, _dp, _i64]
        lib.oracle_v_mag2.restype = _int
        lib.oracle_eos.argtypes = [_int, _dbl, _dp, _i64, _dp, _dp, _i64]
        lib.oracle_eos.restype = _int
        for name in ("oracle_cons2char", "oracle_char2cons"):
            getattr(lib, name).argtypes = [_int, _int, _dbl, _dp, _i64, _dp, _i64, _i64]
            getattr(lib, name).restype = _int
        lib.oracle_flux_adjoint.argtypes = [_int, _int, _dbl, _dp, _i64, _dp, _i64,
                                            _dp, _i64, _i64]
        lib.oracle_flux_adjoint.restype = _int
        lib.oracle_eigenvectors.argtypes = [_int, _dbl, _dp, _i64, _dp, _i64, _dp, _i64, _i64]
        lib.oracle_eigenvectors.restype = _int
        lib.oracle_char_apply.argtypes = [_int, _int, _int, _dbl, _dp, _i64, _dp, _i64, _dp, _i64, _i64]
        lib.oracle_char_apply.restype = _int
        lib.oracle_roe_average.argtypes = [_int, _dbl, _dp, _i64, _dp, _i64, _dp, _i64, _i64]
        lib.oracle_roe_average.restype = _int
        lib.oracle_eos_pvt.argtypes = [_int, _int, _dp, _dp, _i64, _dp, _dp, _dp, _i64]
        lib.oracle_eos_pvt.restype = _int
        lib.oracle_viscous_flux.argtypes = [_int, _dbl, _dbl, _dp, _i64, _dp, _i64, _dp, _i64, _dp, _i64, _i64]
        lib.oracle_viscous_flux.restype = _int
        self.lib = lib
        self.path = path

    def cons2prim(self, dim, gamma, U):
        U = _soa(U, dim + 2)
        n = U.shape[1]
        V = np.empty_like(U)
        _check(self.lib.oracle_cons2prim(dim, gamma, _ptr(U), n, _ptr(V), n, n))
        return V

    def prim2cons(self, dim, gamma, V):
        V = _soa(V, dim + 2)
        n = V.shape[1]
        U = np.empty_like(V)
        _check(self.lib.oracle_prim2cons(dim, gamma, _ptr(V), n, _ptr(U), n, n))
        return U

    def v_mag2(self, dim, U):
        """|v|^2 of each point, shape (n,)."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        y = np.empty(n)
        _check(self.lib.oracle_v_mag2(dim, _ptr(U), n, _ptr(y), n))
        return y

    def eos(self, dim, gamma, U):
        """Returns (p, c), each of shape (n,)."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        p = np.empty(n)
        c = np.empty(n)
        _check(self.lib.oracle_eos(dim, gamma, _ptr(U), n, _ptr(p), _ptr(c), n))
        return p, c

    def flux(self, dim, gamma, U):
        """Returns F with shape (K*D, n); field r*D + d is row r of F_d."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        F = np.empty(((dim + 2) * dim, n))
        _check(self.lib.oracle_flux(dim, gamma, _ptr(U), n, _ptr(F), n, n))
        return F

    def flux_jacobian(self, dim, gamma, U):
        """Returns A with shape (D, n, K, K): A[d, i] is the Jacobian block of
        point i in direction d (point-major, row-major blocks)."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        K = dim + 2
        A = np.empty((dim, n, K, K))
        _check(self.lib.oracle_flux_jacobian(dim, gamma, _ptr(U), n, _ptr(A), n, n))
        return A

    def riemann_invariants(self, dim, gamma, U):
        """Returns R with shape (2*D+1, n): (w-_0, w+_0, ..., s)."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        R = np.empty((2 * dim + 1, n))
        _check(self.lib.oracle_riemann_invariants(dim, gamma, _ptr(U), n, _ptr(R), n, n))
        return R

    def cons2char(self, dim, direction, gamma, U):
        U = _soa(U, dim + 2)
        n = U.shape[1]
        W = np.empty_like(U)
        _check(self.lib.oracle_cons2char(dim, direction, gamma, _ptr(U), n, _ptr(W), n, n))
        return W

    def char2cons(self, dim, direction, gamma, W):
        W = _soa(W, dim + 2)
        n = W.shape[1]
        U = np.empty_like(W)
        _check(self.lib.oracle_char2cons(dim, direction, gamma, _ptr(W), n, _ptr(U), n, n))
        return U

    def flux_adjoint(self, dim, direction, gamma, U, Fbar):
        """Ubar = sum_d A_d^T Fbar_d (direction == -1, Fbar of shape (K*D, n))
        or A_dir^T Fbar (direction >= 0, Fbar of shape (K, n))."""
        K = dim + 2
        U = _soa(U, K)
        n = U.shape[1]
        Fbar = _soa(Fbar, K * dim if direction < 0 else K)
        if Fbar.shape[1] != n:
            raise ValueError("Fbar and U differ in length")
        Ub = np.empty_like(U)
        _check(self.lib.oracle_flux_adjoint(dim, direction, gamma, _ptr(U), n,
                                            _ptr(Fbar), n, _ptr(Ub), n, n))
        return Ub

    def eigenvectors(self, dim, gamma, U):
        """(L, R), each of shape (D, n, K, K): R_d holds the right
        eigenvectors of A_d as columns, L_d = R_d^{-1}."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        K = dim + 2
        L = np.empty((dim, n, K, K))
        R = np.empty((dim, n, K, K))
        rc = self.lib.oracle_eigenvectors(dim, gamma, _ptr(U), n, _ptr(L), n, _ptr(R), n, n)
        if rc == -2:
            raise ValueError("singular eigenvector matrix")
        _check(rc)
        return L, R

    def char_apply(self, dim, direction, mode, gamma, U, X):
        """Y = L_dir X (mode 0) or R_dir X (mode 1), X and Y of shape (K, n)."""
        K = dim + 2
        U = _soa(U, K)
        X = _soa(X, K)
        n = U.shape[1]
        Y = np.empty_like(U)
        rc = self.lib.oracle_char_apply(dim, direction, mode, gamma, _ptr(U), n, _ptr(X), n, _ptr(Y), n, n)
        if rc == -2:
            raise ValueError("singular eigenvector matrix")
        _check(rc)
        return Y

    def roe_average(self, dim, gamma, UL, UR):
        """Roe-averaged conservative state between UL and UR, shape (K, n)."""
        UL = _soa(UL, dim + 2)
        UR = _soa(UR, dim + 2)
        if UL.shape != UR.shape:
            raise ValueError("UL and UR differ in shape")
        n = UL.shape[1]
        Uh = np.empty_like(UL)
        _check(self.lib.oracle_roe_average(dim, gamma, _ptr(UL), n, _ptr(UR), n, _ptr(Uh), n, n))
        return Uh

    def eos_pvt(self, dim, eos, params, U):
        """(p, c, T), each of shape (n,), of EOS `eos` (0 perfect gas with
        params (c_p, c_v); 1 stiffened gas with params (gamma, p_inf, c_v))."""
        U = _soa(U, dim + 2)
        n = U.shape[1]
        prm = np.zeros(3)
        prm[:len(params)] = params
        p, c, T = np.empty(n), np.empty(n), np.empty(n)
        _check(self.lib.oracle_eos_pvt(dim, eos, _ptr(prm), _ptr(U), n, _ptr(p), _ptr(c), _ptr(T), n))
        return p, c, T

    def viscous_flux(self, dim, mu, kappa, U, G, gT):
        """F^v with shape (K*D, n) from U (K, n), the velocity gradient G
        (D*D, n; field i*D + j = dv_i/dx_j) and gT (D, n)."""
        U = _soa(U, dim + 2)
        G = _soa(G, dim * dim)
        gT = _soa(gT, dim)
        n = U.shape[1]
        if G.shape[1] != n or gT.shape[1] != n:
            raise ValueError("inputs differ in length")
        Fv = np.empty(((dim + 2) * dim, n))
        _check(self.lib.oracle_viscous_flux(dim, mu, kappa, _ptr(U), n, _ptr(G), n, _ptr(gT), n, _ptr(Fv), n, n))
        return Fv

    def fused(self, dim, gamma, U):
        """The fused pass is, by definition, the flux, the flux Jacobians and
        the Riemann invariants of the same state."""
        return (self.flux(dim, gamma, U), self.flux_jacobian(dim, gamma, U),
                self.riemann_invariants(dim, gamma, U))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIBRARY):
            build(force=True)
        _default = Oracle(LIBRARY)
    return _default


def cons2prim(dim, gamma, U):
    return default().cons2prim(dim, gamma, U)


def prim2cons(dim, gamma, V):
    return default().prim2cons(dim, gamma, V)


def eos(dim, gamma, U):
    return default().eos(dim, gamma, U)


def v_mag2(dim, U):
    return default().v_mag2(dim, U)


def flux(dim, gamma, U):
    return default().flux(dim, gamma, U)


def flux_jacobian(dim, gamma, U):
    return default().flux_jacobian(dim, gamma, U)


def riemann_invariants(dim, gamma, U):
    return default().riemann_invariants(dim, gamma, U)


def cons2char(dim, direction, gamma, U):
    return default().cons2char(dim, direction, gamma, U)


def char2cons(dim, direction, gamma, W):
    return default().char2cons(dim, direction, gamma, W)


def flux_adjoint(dim, direction, gamma, U, Fbar):
    return default().flux_adjoint(dim, direction, gamma, U, Fbar)


def fused(dim, gamma, U):
    return default().fused(dim, gamma, U)


def eigenvectors(dim, gamma, U):
    return default().eigenvectors(dim, gamma, U)


def char_apply(dim, direction, mode, gamma, U, X):
    return default().char_apply(dim, direction, mode, gamma, U, X)


def roe_average(dim, gamma, UL, UR):
    return default().roe_average(dim, gamma, UL, UR)


def eos_pvt(dim, eos, params, U):
    return default().eos_pvt(dim, eos, params, U)


def viscous_flux(dim, mu, kappa, U, G, gT):
    return default().viscous_flux(dim, mu, kappa, U, G, gT)
