"""Shared helpers of the GPU parity tests: seeded states, transfers, and the
oracle on exactly the values the GPU saw."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1809_09851_amd import fdbb as F
from paper_1809_09851_amd import inputs

GAMMA = 1.4
DTYPES = {"f64": torch.float64, "f32": torch.float32}
NP = {"f64": np.float64, "f32": np.float32}


def require_gpu():
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    F.library()  # raises if the HIP library is not built


def states(dim, n, seed, dt="f64", vacuum=0.0):
    """(U for the oracle in FP64, U on the GPU in storage type dt).  The
    GPU state holds the oracle's prim->cons of a seeded primitive state,
    rounded to the storage type; the oracle sees those rounded values."""
    if dim == 1 and vacuum == 0.0:
        V = inputs.uniform_1d(n, seed)
    else:
        V = inputs.gaussian(dim, n, seed, vacuum_fraction=vacuum)
    U = oracle.prim2cons(dim, GAMMA, V)
    Us = U.astype(NP[dt])
    Ug = F.to_fields(torch.from_numpy(Us).cuda())
    return Us.astype(np.float64), Ug


def prim_states(dim, n, seed, dt="f64"):
    V = inputs.gaussian(dim, n, seed) if dim > 1 else inputs.uniform_1d(n, seed)
    Vs = V.astype(NP[dt])
    return Vs.astype(np.float64), F.to_fields(torch.from_numpy(Vs).cuda())


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def device_group_error(x: torch.Tensor, y: torch.Tensor, groups, denom: torch.Tensor | None = None,
                       chunk: int = 1 << 21) -> float:
    """The group-normwise error of metrics.group_error, on the device, over
    every point: max over points and groups of max_g |x - y| / max_g |y|
    (or / denom[point]).  x, y: (fields, n) tensors; a zero denominator
    requires a zero difference.  Both must be finite everywhere."""
    n = y.shape[1]
    worst = 0.0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        xs = x[:, a:b].double()
        ys = y[:, a:b].double()
        assert bool(torch.isfinite(xs).all()) and bool(torch.isfinite(ys).all())
        for g in groups:
            num = (xs[g] - ys[g]).abs().amax(0)
            den = ys[g].abs().amax(0) if denom is None else denom[a:b].double()
            zero = den == 0
            if bool((num[zero] != 0).any()):
                return float("inf")
            if bool((~zero).any()):
                worst = max(worst, float((num[~zero] / den[~zero]).max()))
    return worst


def device_blocks_error(x: torch.Tensor, y: torch.Tensor, chunk: int = 1 << 20) -> float:
    """Jacobian blocks (D, n, K, K): one group per block, every block."""
    D, n, K, _ = y.shape
    worst = 0.0
    for d in range(D):
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            xs = x[d, a:b].reshape(b - a, K * K).double().T
            ys = y[d, a:b].reshape(b - a, K * K).double().T
            worst = max(worst, device_group_error(xs, ys, [list(range(K * K))], chunk=chunk))
    return worst


def adjoint_denominator(U: torch.Tensor, Fbar: torch.Tensor, gamma: float = GAMMA,
                        chunk: int = 1 << 20) -> torch.Tensor:
    """Per-point scale of the adjoint Ubar = sum_d A_d^T Fbar_d: the largest
    component of sum_d |A_d|^T |Fbar_d| (the adjoint's group denominator),
    with A_d from the library's Jacobian kernel, on the device."""
    dim = U.shape[0] - 2
    K = dim + 2
    n = U.shape[1]
    out = torch.empty(n, dtype=torch.float64, device=U.device)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        A = F.flux_jacobian(U[:, a:b], gamma).double().abs()           # (D, m, K, K)
        fb = Fbar[:, a:b].double().abs().reshape(K, dim, b - a)         # field r*D + d
        fb = fb.permute(1, 2, 0)                                        # (D, m, K): [d, m, r]
        out[a:b] = (A * fb[..., None]).sum(dim=(0, 2)).amax(1)
    return out
