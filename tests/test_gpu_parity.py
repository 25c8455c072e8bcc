"""HIP kernels against the CPU oracle, element by element, through the C ABI.

Sizes span several tiles (256 threads x up to 4 points) and ragged tails.
Tolerances and the error metric are those of tests/metrics.py.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import DTYPES, GAMMA, NP, host, prim_states, require_gpu, states
from metrics import (TOL, blocks_error, char_groups, flux_groups, group_error, riemann_groups, roe_error,
                     state_groups)
from paper_1809_09851_amd import fdbb as F

pytestmark = pytest.mark.gpu

DIMS = (1, 2, 3)
DTS = ("f64", "f32")
SIZES = (1, 63, 64, 65, 1000, 5003, 12305)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _seed(dim, n, dt, k=0):
    return 1000 * dim + (n % 997) + (0 if dt == "f64" else 500) + 7 * k


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_cons2prim(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt), dt)
    V = F.cons2prim(Ug, GAMMA)
    assert group_error(host(V), oracle.cons2prim(dim, GAMMA, Uo), state_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_prim2cons(dim, dt, n):
    Vo, Vg = prim_states(dim, n, _seed(dim, n, dt, 1), dt)
    U = F.prim2cons(Vg, GAMMA)
    assert group_error(host(U), oracle.prim2cons(dim, GAMMA, Vo), state_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_eos(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 2), dt)
    p, c = F.eos(Ug, GAMMA)
    po, co = oracle.eos(dim, GAMMA, Uo)
    assert group_error(host(p)[None], po[None], [[0]]) <= TOL[dt]
    assert group_error(host(c)[None], co[None], [[0]]) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_velocity_magnitude2(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 13), dt)
    y = F.velocity_magnitude2(Ug)
    assert group_error(host(y)[None], oracle.v_mag2(dim, Uo)[None], [[0]]) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_eos_single_output(dim, dt):
    n = 777
    Uo, Ug = states(dim, n, 3, dt)
    po, co = oracle.eos(dim, GAMMA, Uo)
    c = torch.empty(n, dtype=DTYPES[dt], device="cuda")
    F.fdbb_eos(dim, GAMMA, Ug, None, c)
    assert group_error(host(c)[None], co[None], [[0]]) <= TOL[dt]
    p = torch.empty(n, dtype=DTYPES[dt], device="cuda")
    F.fdbb_eos(dim, GAMMA, Ug, p, None)
    assert group_error(host(p)[None], po[None], [[0]]) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_flux(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 3), dt)
    Fg = F.flux(Ug, GAMMA)
    assert group_error(host(Fg), oracle.flux(dim, GAMMA, Uo), flux_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_flux_jacobian(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 4), dt)
    A = F.flux_jacobian(Ug, GAMMA)
    assert blocks_error(host(A), oracle.flux_jacobian(dim, GAMMA, Uo)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_riemann_invariants(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 5), dt)
    R = F.riemann_invariants(Ug, GAMMA)
    assert group_error(host(R), oracle.riemann_invariants(dim, GAMMA, Uo), riemann_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", (1, 65, 5003))
def test_characteristic_transforms(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 6), dt)
    for d in range(dim):
        W = F.cons2char(Ug, d, GAMMA)
        Wo = oracle.cons2char(dim, d, GAMMA, Uo)
        assert group_error(host(W), Wo, char_groups(dim)) <= TOL[dt]
        # inverse, on the exact W the GPU holds
        Wh = host(W)
        U2 = F.char2cons(W, d, GAMMA)
        assert group_error(host(U2), oracle.char2cons(dim, d, GAMMA, Wh), state_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_flux_direction(dim, dt, n):
    """F_d alone equals column d of the oracle's flux block (fields r*D + d)."""
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 8), dt)
    Fo = oracle.flux(dim, GAMMA, Uo)
    for d in range(dim):
        Fd = F.flux(Ug, GAMMA, direction=d)
        assert Fd.shape == (dim + 2, n)
        assert group_error(host(Fd), Fo[d::dim], [list(range(dim + 2))]) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_fused(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 7), dt)
    Fg, A, R = F.euler_fused(Ug, GAMMA)
    Fo, Ao, Ro = oracle.fused(dim, GAMMA, Uo)
    assert group_error(host(Fg), Fo, flux_groups(dim)) <= TOL[dt]
    assert blocks_error(host(A), Ao) <= TOL[dt]
    assert group_error(host(R), Ro, riemann_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_fused_equals_single_ops(dim, dt):
    n = 4099
    _, Ug = states(dim, n, 11, dt)
    Fg, A, R = F.euler_fused(Ug, GAMMA)
    # Same formulas in separate kernels: equal up to the compiler's choice of
    # contractions, far inside the oracle tolerance.
    tol = 1e-14 if dt == "f64" else 1.2e-7
    assert group_error(host(Fg), host(F.flux(Ug, GAMMA)), flux_groups(dim)) <= tol
    assert blocks_error(host(A), host(F.flux_jacobian(Ug, GAMMA))) <= tol
    assert group_error(host(R), host(F.riemann_invariants(Ug, GAMMA)), riemann_groups(dim)) <= tol


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_fused_partial_outputs(dim, dt):
    n = 3001
    Uo, Ug = states(dim, n, 12, dt)
    Fo, Ao, Ro = oracle.fused(dim, GAMMA, Uo)
    for want in ((True, False, False), (False, True, False), (False, False, True), (True, False, True)):
        Fg, A, R = F.euler_fused(Ug, GAMMA, *want)
        if Fg is not None:
            assert group_error(host(Fg), Fo, flux_groups(dim)) <= TOL[dt]
        if A is not None:
            assert blocks_error(host(A), Ao) <= TOL[dt]
        if R is not None:
            assert group_error(host(R), Ro, riemann_groups(dim)) <= TOL[dt]


def _adjoint_scale(dim, Uo, Fb, direction):
    """Per-point |sum_d |A_d|^T |Fbar_d| |_inf from the oracle's Jacobians."""
    A = np.abs(oracle.flux_jacobian(dim, GAMMA, Uo))
    K = dim + 2
    s = np.zeros((K, Uo.shape[1]))
    for d in range(dim):
        if direction >= 0 and d != direction:
            continue
        fb = Fb if direction >= 0 else np.array([Fb[r * dim + d] for r in range(K)])
        s += np.einsum("nrc,rn->cn", A[d], np.abs(fb))
    return s.max(axis=0)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_adjoint(dim, dt, n):
    from paper_1809_09851_amd import inputs
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 8), dt)
    K = dim + 2
    for direction in [-1] + list(range(dim)):
        fields = K * dim if direction < 0 else K
        Fb = inputs.cotangent(dim, n, _seed(dim, n, dt, 9) + direction, fields)
        Fb = Fb.astype(np.float32 if dt == "f32" else np.float64).astype(np.float64)
        Fbg = F.to_fields(torch.from_numpy(Fb).to(DTYPES[dt]).cuda())
        Ub = F.flux_adjoint(Ug, Fbg, GAMMA, direction)
        ref = oracle.flux_adjoint(dim, direction, GAMMA, Uo, Fb)
        err = group_error(host(Ub), ref, [list(range(K))], denom=_adjoint_scale(dim, Uo, Fb, direction))
        assert err <= TOL[dt], (direction, err)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_eigenvectors(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 14), dt)
    L, R = F.eigenvectors(Ug, GAMMA)
    Lo, Ro = oracle.eigenvectors(dim, GAMMA, Uo)
    assert blocks_error(host(L), Lo) <= TOL[dt]
    assert blocks_error(host(R), Ro) <= TOL[dt]
    Lg, _ = F.eigenvectors(Ug, GAMMA, right=False)
    assert blocks_error(host(Lg), Lo) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", (1, 65, 5003))
def test_char_apply(dim, dt, n):
    from paper_1809_09851_amd import inputs
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 15), dt)
    K = dim + 2
    X = inputs.cotangent(dim, n, _seed(dim, n, dt, 16), fields=K)
    X = X.astype(np.float32 if dt == "f32" else np.float64).astype(np.float64)
    Xg = F.to_fields(torch.from_numpy(X).to(DTYPES[dt]).cuda())
    Lo, Ro = oracle.eigenvectors(dim, GAMMA, Uo)
    for d in range(dim):
        for mode, M in ((0, Lo[d]), (1, Ro[d])):
            Y = F.char_apply(Ug, Xg, d, mode, GAMMA)
            ref = oracle.char_apply(dim, d, mode, GAMMA, Uo, X)
            den = np.einsum("nrc,cn->rn", np.abs(M), np.abs(X)).max(axis=0)
            assert group_error(host(Y), ref, [list(range(K))], denom=den) <= TOL[dt], (d, mode)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_roe_average(dim, dt, n):
    ULo, ULg = states(dim, n, _seed(dim, n, dt, 17), dt)
    URo, URg = states(dim, n, _seed(dim, n, dt, 18), dt, vacuum=0.05 if dim > 1 else 0.0)
    Uh = F.roe_average(ULg, URg, GAMMA)
    assert roe_error(host(Uh), oracle.roe_average(dim, GAMMA, ULo, URo), ULo, URo) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_roe_average_in_place_and_of_equal_states(dim, dt):
    n = 3001
    ULo, ULg = states(dim, n, 71, dt)
    URo, URg = states(dim, n, 72, dt)
    ref = oracle.roe_average(dim, GAMMA, ULo, URo)
    F.fdbb_roe_average(dim, GAMMA, ULg, URg, URg)  # Uh written over UR
    assert roe_error(host(URg), ref, ULo, URo) <= TOL[dt]
    same = F.roe_average(ULg, ULg, GAMMA)
    assert group_error(host(same), ULo, state_groups(dim)) <= TOL[dt]


EOS_CASES = (("perfect_gas", (3.5, 2.5)), ("perfect_gas", (1.0, 0.6)), ("stiffened_gas", (4.4, 0.3, 0.7)),
             ("stiffened_gas", (1.9, 0.0, 2.5)))


@pytest.mark.parametrize("case", range(len(EOS_CASES)))
@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", (1, 65, 5003))
def test_eos_pvt(dim, dt, n, case):
    eos, prm = EOS_CASES[case]
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 19 + case), dt)
    p, c, T = F.eos_pvt(Ug, eos, prm)
    rp, rc, rT = oracle.eos_pvt(dim, F.EOS_IDS[eos], prm, Uo)
    for x, y, what in ((p, rp, "p"), (c, rc, "c"), (T, rT, "T")):
        # p and T of the stiffened gas are differences (rho e against p_inf):
        # measure them against the size of their terms
        den = None
        if eos == "stiffened_gas" and what != "c":
            e_abs = np.abs(oracle.eos_pvt(dim, 0, (prm[0], 1.0), Uo)[2])  # |e| via c_v = 1
            den = (prm[0] - 1) * Uo[0] * e_abs + prm[0] * prm[1] if what == "p" else (e_abs + prm[1] / Uo[0]) / prm[2]
        assert group_error(host(x)[None], y[None], [[0]], denom=den) <= TOL[dt], what


def test_eos_pvt_partial_outputs():
    Uo, Ug = states(3, 777, 5)
    T = torch.full((777,), 7.0, dtype=torch.float64, device="cuda")
    F.fdbb_eos_pvt(3, "stiffened_gas", (4.4, 0.3, 0.7), Ug, None, None, T)
    rT = oracle.eos_pvt(3, 1, (4.4, 0.3, 0.7), Uo)[2]
    assert group_error(host(T)[None], rT[None], [[0]]) <= TOL["f64"]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
@pytest.mark.parametrize("n", SIZES)
def test_viscous_flux(dim, dt, n):
    Uo, Ug = states(dim, n, _seed(dim, n, dt, 23), dt)
    rng = np.random.default_rng(_seed(dim, n, dt, 24))
    G = rng.normal(size=(dim * dim, n)).astype(NP[dt]).astype(np.float64)
    gT = rng.normal(size=(dim, n)).astype(NP[dt]).astype(np.float64)
    Gg = F.to_fields(torch.from_numpy(G).to(DTYPES[dt]).cuda())
    gTg = F.to_fields(torch.from_numpy(gT).to(DTYPES[dt]).cuda())
    mu, kappa = 0.01, 0.02
    Fv = F.viscous_flux(Ug, Gg, gTg, mu, kappa)
    ref = oracle.viscous_flux(dim, mu, kappa, Uo, G, gT)
    # stresses and energy fluxes are sums of signed terms: measure each
    # direction against the size of its terms
    K = dim + 2
    v = np.abs(Uo[1:dim + 1] / Uo[0])
    gabs = np.abs(G).max(axis=0)
    den = mu * 4 * gabs * (1 + v.sum(axis=0)) + kappa * np.abs(gT).max(axis=0)
    got = host(Fv)
    assert np.all(got[[d for d in range(dim)]] == 0.0)  # mass row
    assert group_error(got, ref, [[r * dim + d for r in range(1, K)] for d in range(dim)], denom=den) <= TOL[dt]


# ------------------------------------------------------------ edge cases

def test_zero_points_leave_outputs_untouched():
    _, Ug = states(3, 10, 1)
    out = torch.full((15, 64), 7.0, dtype=torch.float64, device="cuda")
    F.fdbb_flux(3, GAMMA, Ug, out[:, :10], n=0)
    assert torch.all(out == 7.0)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_unpadded_and_offset_views(dim, dt):
    """Rows of odd length and views starting at an odd element take the
    scalar path; results must not change."""
    n = 1001
    Uo, Ug = states(dim, n + 1, 21, dt)
    K = dim + 2
    tight = torch.from_numpy(Uo.astype(np.float32 if dt == "f32" else np.float64)).cuda().contiguous()
    assert tight.stride(0) == n + 1
    for U_view, Uref in ((tight, Uo), (tight[:, 1:], Uo[:, 1:])):
        Fo = oracle.flux(dim, GAMMA, Uref)
        Fg = F.flux(U_view, GAMMA)
        assert group_error(host(Fg), Fo, flux_groups(dim)) <= TOL[dt]
        A = F.flux_jacobian(U_view, GAMMA)
        assert blocks_error(host(A), oracle.flux_jacobian(dim, GAMMA, Uref)) <= TOL[dt]
        # outputs with odd rows too
        Fo2 = torch.empty((K * dim, U_view.shape[1]), dtype=DTYPES[dt], device="cuda")
        F.fdbb_flux(dim, GAMMA, U_view, Fo2)
        assert group_error(host(Fo2), Fo, flux_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_scalar_path_equals_vector_path(dim, dt):
    """Inputs one element off alignment make every load and store of a call
    take the scalar path (4- and 8-byte accesses, in every store and load
    flavour the kernels use); the per-point arithmetic is shared, so each
    result must equal, bit for bit, the 16-byte path's on an aligned copy of
    the same data."""
    from paper_1809_09851_amd import inputs
    n = 1001
    K = dim + 2
    npdt = np.float32 if dt == "f32" else np.float64

    def pair(a):
        tight = torch.from_numpy(np.ascontiguousarray(a, dtype=npdt)).cuda()
        view = tight[:, 1:]                      # base one element past a 16-byte boundary
        return view, F.to_fields(view)           # unaligned view, padded aligned copy

    Uo, _ = states(dim, n + 1, 23, dt)
    URo, _ = states(dim, n + 1, 24, dt)
    Uu, Ua = pair(Uo)
    URu, URa = pair(URo)
    Fbu, Fba = pair(inputs.cotangent(dim, n + 1, 25))
    Xu, Xa = pair(inputs.cotangent(dim, n + 1, 26, fields=K))
    Vu, Va = pair(host(F.cons2prim(Ua, GAMMA)))
    assert Uu.data_ptr() % 16 != 0 and Ua.data_ptr() % 16 == 0

    def same(name, fn, *args):
        a, b = fn(*[x[0] for x in args]), fn(*[x[1] for x in args])
        for x, y in zip(a if isinstance(a, tuple) else (a,), b if isinstance(b, tuple) else (b,)):
            assert torch.equal(x, y), name

    same("cons2prim", lambda U: F.cons2prim(U, GAMMA), (Uu, Ua))
    same("prim2cons", lambda V: F.prim2cons(V, GAMMA), (Vu, Va))
    same("v_mag2", F.velocity_magnitude2, (Uu, Ua))
    same("flux", lambda U: F.flux(U, GAMMA), (Uu, Ua))
    same("riemann_invariants", lambda U: F.riemann_invariants(U, GAMMA), (Uu, Ua))
    same("fused", lambda U: F.euler_fused(U, GAMMA), (Uu, Ua))
    same("adjoint", lambda U, Fb: F.flux_adjoint(U, Fb, GAMMA), (Uu, Ua), (Fbu, Fba))
    same("roe_average", lambda U, UR: F.roe_average(U, UR, GAMMA), (Uu, Ua), (URu, URa))
    same("char_apply", lambda U, X: F.char_apply(U, X, dim - 1, 1, GAMMA), (Uu, Ua), (Xu, Xa))
    same("eigenvectors", lambda U: F.eigenvectors(U, GAMMA), (Uu, Ua))


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("dim", DIMS)
def test_in_place_transforms(dim, dt):
    n = 2049
    Uo, Ug = states(dim, n, 31, dt)
    rho_before = Ug[0].clone()
    F.fdbb_cons2prim(dim, GAMMA, Ug, Ug)
    assert torch.equal(Ug[0], rho_before)
    assert group_error(host(Ug), oracle.cons2prim(dim, GAMMA, Uo), state_groups(dim)) <= TOL[dt]
    Vh = host(Ug)
    F.fdbb_prim2cons(dim, GAMMA, Ug, Ug)
    assert torch.equal(Ug[0], rho_before)
    assert group_error(host(Ug), oracle.prim2cons(dim, GAMMA, Vh), state_groups(dim)) <= TOL[dt]
    Uh = host(Ug)
    F.fdbb_cons2char(dim, dim - 1, GAMMA, Ug, Ug)
    assert group_error(host(Ug), oracle.cons2char(dim, dim - 1, GAMMA, Uh), char_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("dim", DIMS)
def test_near_vacuum_states(dim):
    n = 20000
    Uo, Ug = states(dim, n, 41, "f64", vacuum=0.05)
    Fg, A, R = F.euler_fused(Ug, GAMMA)
    Fo, Ao, Ro = oracle.fused(dim, GAMMA, Uo)
    assert group_error(host(Fg), Fo, flux_groups(dim)) <= TOL["f64"]
    assert blocks_error(host(A), Ao) <= TOL["f64"]
    assert group_error(host(R), Ro, riemann_groups(dim)) <= TOL["f64"]


@pytest.mark.parametrize("dim", DIMS)
def test_non_admissible_states_propagate_like_the_oracle(dim):
    """rho < 0 or p < 0 is not an error: NaN/Inf land where the oracle's do."""
    n = 512
    Uo, _ = states(dim, n, 51)
    Uo[0, ::7] *= -1.0                       # negative density
    Uo[dim + 1, 3::11] *= -1.0               # negative energy -> negative p
    Uo[0, 5] = 0.0                           # zero density
    Ug = F.to_fields(torch.from_numpy(Uo).cuda())
    p, c = F.eos(Ug, GAMMA)
    po, co = oracle.eos(dim, GAMMA, Uo)
    assert group_error(host(p)[None], po[None], [[0]]) <= TOL["f64"]
    assert group_error(host(c)[None], co[None], [[0]]) <= TOL["f64"]
    R = F.riemann_invariants(Ug, GAMMA)
    assert np.isnan(host(R)).any()
    assert group_error(host(R), oracle.riemann_invariants(dim, GAMMA, Uo), riemann_groups(dim)) <= TOL["f64"]


def test_other_gammas():
    for g in (5.0 / 3.0, 1.1, 1.3):
        Uo, Ug = states(3, 3000, 61)
        Fg, A, R = F.euler_fused(Ug, g)
        Fo, Ao, Ro = oracle.fused(3, g, Uo)
        assert group_error(host(Fg), Fo, flux_groups(3)) <= TOL["f64"]
        assert blocks_error(host(A), Ao) <= TOL["f64"]
        assert group_error(host(R), Ro, riemann_groups(3)) <= TOL["f64"]
