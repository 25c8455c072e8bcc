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
