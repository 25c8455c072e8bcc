"""EulerFlux: forward = flux kernel, backward = hand-written adjoint kernel."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import host, require_gpu
from metrics import TOL, group_error
from paper_1809_09851_amd import fdbb as F
from paper_1809_09851_amd import inputs
from paper_1809_09851_amd.autograd import EulerFlux, euler_flux

pytestmark = pytest.mark.gpu
GAMMA = 1.4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("dim", (1, 2, 3))
@pytest.mark.parametrize("direction", (None, 0, -1))
def test_gradcheck(dim, direction):
    d = None if direction is None else (dim - 1 if direction == -1 else 0)
    V = inputs.gaussian(dim, 6, 5)
    U = torch.from_numpy(oracle.prim2cons(dim, GAMMA, V)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: EulerFlux.apply(x, GAMMA, d), (U,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6)


@pytest.mark.parametrize("dim", (2, 3))
def test_loss_gradient_matches_oracle_adjoint(dim):
    n = 4096
    V = inputs.gaussian(dim, n, 3)
    U = oracle.prim2cons(dim, GAMMA, V)
    w = inputs.cotangent(dim, n, 4)
    Ug = F.to_fields(torch.from_numpy(U).cuda()).requires_grad_(True)
    wg = torch.from_numpy(w).cuda()
    loss = (euler_flux(Ug, GAMMA) * wg).sum()
    loss.backward()
    ref = oracle.flux_adjoint(dim, -1, GAMMA, U, w)
    K = dim + 2
    A = np.abs(oracle.flux_jacobian(dim, GAMMA, U))
    den = np.zeros((K, n))
    for d in range(dim):
        den += np.einsum("nrc,rn->cn", A[d], np.abs(np.array([w[r * dim + d] for r in range(K)])))
    assert group_error(host(Ug.grad), ref, [list(range(K))], denom=den.max(axis=0)) <= TOL["f64"]


def test_expanded_cotangent():
    """sum() hands backward an expanded (stride 0) cotangent."""
    dim, n = 3, 1000
    U = torch.from_numpy(oracle.prim2cons(dim, GAMMA, inputs.gaussian(dim, n, 8))).cuda().requires_grad_(True)
    euler_flux(U, GAMMA).sum().backward()
    ref = oracle.flux_adjoint(dim, -1, GAMMA, host(U), np.ones((15, n)))
    assert np.max(np.abs(host(U.grad) - ref)) <= 1e-12 * np.max(np.abs(ref))
