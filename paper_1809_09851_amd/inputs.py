"""Seeded synthetic workloads.

This module draws random numbers and nothing else: it holds none of the
Euler arithmetic.  States are returned in primitive form V = (rho, v_1..v_D,
p) as float64 numpy arrays of shape (D+2, n); each consumer converts them to
conservative variables with its own prim->cons.  The recipes mirror the
paper's workloads (physical states, Sec. 3, "Mini-application"; sizes 2^10
to 2^28 points) at the sizes used for measurement:

  * ``uniform_1d``  -- rho ~ U[0.5, 2], u ~ U[-1, 1], p ~ U[0.5, 2]
  * ``gaussian``    -- rho ~ U[0.5, 2], each v_i ~ N(0, 0.5^2), p ~ U[0.5, 2]
  * ``gaussian`` with ``vacuum_fraction`` -- as above, and each point is
    independently near-vacuum with that probability, its rho then redrawn
    from U[1e-3, 1e-2] (v and p unchanged)

Draw order is fixed: rho, then the velocity components in order, then p,
then (if requested) the vacuum mask and the vacuum densities.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4  # c_p / c_v = (7/2) / (5/2), the paper's perfect gas


def uniform_1d(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    V = np.empty((3, n))
    V[0] = rng.uniform(0.5, 2.0, n)
    V[1] = rng.uniform(-1.0, 1.0, n)
    V[2] = rng.uniform(0.5, 2.0, n)
    return V


def gaussian(dim: int, n: int, seed: int = 1, vacuum_fraction: float = 0.0,
             rng: np.random.Generator | None = None) -> np.ndarray:
    if rng is None:
        rng = np.random.default_rng(seed)
    V = np.empty((dim + 2, n))
    V[0] = rng.uniform(0.5, 2.0, n)
    for k in range(dim):
        V[1 + k] = rng.normal(0.0, 0.5, n)
    V[dim + 1] = rng.uniform(0.5, 2.0, n)
    if vacuum_fraction > 0.0:
        mask = rng.random(n) < vacuum_fraction
        V[0, mask] = rng.uniform(1e-3, 1e-2, int(mask.sum()))
    return V


def block_sizes(nblocks: int = 512, seed: int = 2, lo_exp: float = 3.0,
                hi_exp: float = 6.0) -> np.ndarray:
    """Block sizes log-uniform in [10^lo_exp, 10^hi_exp] points."""
    rng = np.random.default_rng(seed)
    return np.rint(10.0 ** rng.uniform(lo_exp, hi_exp, nblocks)).astype(np.int64)


def batched(dim: int = 3, nblocks: int = 512, seed: int = 2,
            vacuum_fraction: float = 0.05):
    """Block sizes first, then one gaussian state over all points, split into
    blocks in order.  Returns (sizes, list of V blocks)."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(10.0 ** rng.uniform(3.0, 6.0, nblocks)).astype(np.int64)
    total = int(sizes.sum())
    V = gaussian(dim, total, vacuum_fraction=vacuum_fraction, rng=rng)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return sizes, [V[:, offs[b]:offs[b + 1]] for b in range(nblocks)]


def cotangent(dim: int, n: int, seed: int, fields: int | None = None) -> np.ndarray:
    """Weights w ~ N(0, 1) with the flux tensor's shape (K*D fields), or with
    ``fields`` fields."""
    rng = np.random.default_rng(seed)
    f = (dim + 2) * dim if fields is None else fields
    return rng.normal(0.0, 1.0, (f, n))


SERVE_OPS = ("cons2prim", "flux", "flux_jacobian", "adjoint")


def request_stream(rate: float, count: int, seed: int = 4, pool: int = 10_000_000,
                   lo_exp: float = 3.0, hi_exp: float = 7.0):
    """Poisson arrivals at ``rate`` requests/s.  Each request draws its op
    uniformly from SERVE_OPS, D uniformly from {1, 2, 3}, N log-uniform in
    [10^lo_exp, 10^hi_exp], dtype uniformly from {"f64", "f32"} and an offset
    uniform in [0, pool - N].  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    ops = rng.integers(0, len(SERVE_OPS), count)
    dims = rng.integers(1, 4, count)
    ns = np.rint(10.0 ** rng.uniform(lo_exp, hi_exp, count)).astype(np.int64)
    ns = np.minimum(ns, pool)
    dts = rng.integers(0, 2, count)
    offs = (rng.random(count) * (pool - ns + 1)).astype(np.int64)
    out = []
    for i in range(count):
        out.append({"t": float(t[i]), "op": SERVE_OPS[int(ops[i])], "dim": int(dims[i]),
                    "n": int(ns[i]), "dtype": "f64" if dts[i] == 0 else "f32",
                    "offset": int(offs[i])})
    return out
