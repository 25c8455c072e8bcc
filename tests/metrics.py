"""Group-normwise error used by every parity test.

Plain relative error is ill-posed at outputs that are zero or cancel (for
example A_d[1+d][0] = phi - v_d^2), so errors are measured per point and per
group of outputs that share a physical scale:

    err = max over points i and groups G of |x_iG - y_iG|_inf / |y_iG|_inf

where y is the oracle.  A group whose reference is exactly zero must be
exactly zero.  Non-finite values (NaN or Inf) must occur at the same places;
for those points the kind of non-finite value is not compared.

Tolerances: 1e-12 for FP64 storage, 1e-5 for FP32 storage (outputs are
rounded to FP32, about 6e-8 relative, and the FP64 arithmetic adds nothing
visible).
"""
from __future__ import annotations

import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5}


def group_error(x: np.ndarray, y: np.ndarray, groups, denom: np.ndarray | None = None) -> float:
    """x, y: (fields, n) arrays; groups: list of lists of field indices.
    denom, if given, is an (n,) per-point scale used for every group."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    assert x.shape == y.shape, (x.shape, y.shape)
    # Non-admissible states (rho <= 0, p < 0) have no defined value; which of
    # NaN or +-Inf comes out depends on the order of operations, so only the
    # places where results stop being finite must agree.
    if not np.array_equal(np.isfinite(x), np.isfinite(y)):
        return float("inf")
    worst = 0.0
    for g in groups:
        xg = x[g]
        yg = y[g]
        fin = np.isfinite(yg).all(axis=0)
        if not fin.any():
            continue
        xg = xg[:, fin]
        yg = yg[:, fin]
        num = np.max(np.abs(xg - yg), axis=0)
        den = np.max(np.abs(yg), axis=0) if denom is None else np.asarray(denom)[fin]
        zero = den == 0
        if zero.any() and np.any(num[zero] != 0):
            return float("inf")
        if (~zero).any():
            worst = max(worst, float(np.max(num[~zero] / den[~zero])))
    return worst


def state_groups(dim):
    """U or V: {rho}, {m or v}, {E or p}."""
    return [[0], list(range(1, dim + 1)), [dim + 1]]


def flux_groups(dim):
    """Each column F_d of the flux tensor (fields r*D + d)."""
    return [[r * dim + d for r in range(dim + 2)] for d in range(dim)]


def riemann_groups(dim):
    return [[2 * d, 2 * d + 1] for d in range(dim)] + [[2 * dim]]


def char_groups(dim):
    """W = (w-, s, tangential v, w+): {w-, w+}, {s}, {tangential}."""
    g = [[0, dim + 1], [1]]
    if dim > 1:
        g.append(list(range(2, dim + 1)))
    return g


def blocks_error(x: np.ndarray, y: np.ndarray) -> float:
    """Jacobian blocks (D, n, K, K): one group per block."""
    D, n, K, _ = y.shape
    xf = np.asarray(x, dtype=np.float64).reshape(D * n, K * K).T
    yf = np.asarray(y, dtype=np.float64).reshape(D * n, K * K).T
    return group_error(xf, yf, [list(range(K * K))])


def roe_error(x: np.ndarray, y: np.ndarray, UL: np.ndarray, UR: np.ndarray) -> float:
    """Roe-averaged states: groups {rho}, {m}, {E}.  The averaged velocity
    (a v_L + b v_R) / (a + b), a = sqrt(rho_L), b = sqrt(rho_R), cancels
    when v_L and v_R point apart, so the momentum group is measured against
    the size of its terms, rho^ max_k (a |v_L,k| + b |v_R,k|) / (a + b)."""
    dim = UL.shape[0] - 2
    a, b = np.sqrt(UL[0]), np.sqrt(UR[0])
    vL, vR = np.abs(UL[1:dim + 1] / UL[0]), np.abs(UR[1:dim + 1] / UR[0])
    den = (a * b) * ((a * vL + b * vR) / (a + b)).max(axis=0)
    e = group_error(x, y, [[0], [dim + 1]])
    return max(e, group_error(x, y, [list(range(1, dim + 1))], denom=den))
