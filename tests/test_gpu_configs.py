"""Every launch configuration the tuner may pick gives oracle-matching
results (LDS staging races or tail bugs would show up here)."""
import pytest

import oracle
from gpu_common import GAMMA, host, require_gpu, states
from metrics import TOL, blocks_error, flux_groups, group_error, riemann_groups, state_groups
from paper_1809_09851_amd import fdbb as F

pytestmark = pytest.mark.gpu

CONFIGS = [(b, p, g, t) for b in (64, 128, 256, 512, 1024) for p in (1, 2, 4) for g, t in ((0, 1), (7, 0))]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _with_config(op, dim, dt_code, cfg, fn):
    """Run fn with cfg as the only configuration of (op, dim, dtype): the
    small-launch entry, which would take over at these sizes, is lifted for
    the call."""
    old = F.fdbb_get_launch_config(op, dim, dt_code)
    small = F.fdbb_get_small_launch_config(op, dim, dt_code)
    F.fdbb_set_launch_config(op, dim, dt_code, *cfg)
    F.fdbb_set_small_launch_config(op, dim, dt_code, 0)
    try:
        assert F.fdbb_launch_config_for(op, dim, dt_code, 1) == tuple(cfg)
        return fn()
    finally:
        F.fdbb_set_launch_config(op, dim, dt_code, *old)
        if small[0]:
            F.fdbb_set_small_launch_config(op, dim, dt_code, *small)


@pytest.mark.parametrize("block,ppt,grid,nt", CONFIGS)
def test_fused_all_configs(block, ppt, grid, nt):
    n = 7001
    for dt, code, es in (("f64", F.F64, 8), ("f32", F.F32, 4)):
        for dim in (1, 2, 3):
            Uo, Ug = states(dim, n, 70 + dim, dt)
            K = dim + 2
            lds = block * ppt * K * K * es
            try:
                Fg, A, R = _with_config("fused", dim, code, (block, ppt, grid, nt),
                                        lambda: F.euler_fused(Ug, GAMMA))
            except F.FdbbError as e:
                assert e.status == F.EINVAL and (lds > 65536 or block > 256), (dt, dim, str(e))
                continue
            Fo, Ao, Ro = oracle.fused(dim, GAMMA, Uo)
            assert group_error(host(Fg), Fo, flux_groups(dim)) <= TOL[dt]
            assert blocks_error(host(A), Ao) <= TOL[dt]
            assert group_error(host(R), Ro, riemann_groups(dim)) <= TOL[dt]


@pytest.mark.parametrize("block,ppt,grid,nt", CONFIGS)
def test_pointwise_all_configs(block, ppt, grid, nt):
    n = 5003
    for dt, code in (("f64", F.F64), ("f32", F.F32)):
        dim = 3
        Uo, Ug = states(dim, n, 80, dt)
        Fg = _with_config("flux", dim, code, (block, ppt, grid, nt), lambda: F.flux(Ug, GAMMA))
        assert group_error(host(Fg), oracle.flux(dim, GAMMA, Uo), flux_groups(dim)) <= TOL[dt]
        V = _with_config("cons2prim", dim, code, (block, ppt, grid, nt), lambda: F.cons2prim(Ug, GAMMA))
        assert group_error(host(V), oracle.cons2prim(dim, GAMMA, Uo), state_groups(dim)) <= TOL[dt]
        try:
            A = _with_config("flux_jacobian", dim, code, (block, ppt, grid, nt), lambda: _try_jac(Ug))
        except F.FdbbError as e:
            assert e.status == F.EINVAL and block > 256
            A = None
        if A is not None:
            assert blocks_error(host(A), oracle.flux_jacobian(dim, GAMMA, Uo)) <= TOL[dt]


def _try_jac(Ug):
    try:
        return F.flux_jacobian(Ug, GAMMA)
    except F.FdbbError as e:
        assert e.status == F.EINVAL
        return None


@pytest.mark.parametrize("block,ppt,grid,nt", CONFIGS)
def test_eigen_adjoint_roe_all_configs(block, ppt, grid, nt):
    """The other LDS-staged kernel (eigenvector blocks) and the kernels with
    two inputs (adjoint, Roe average) in every configuration."""
    import numpy as np
    from metrics import roe_error
    from paper_1809_09851_amd import inputs
    n = 3001
    dim, K = 3, 5
    for dt, code, es in (("f64", F.F64, 8), ("f32", F.F32, 4)):
        Uo, Ug = states(dim, n, 90, dt)
        cfg = (block, ppt, grid, nt)
        try:
            L, R = _with_config("eigenvectors", dim, code, cfg, lambda: F.eigenvectors(Ug, GAMMA))
        except F.FdbbError as e:
            # refused: more than 256 threads, or more LDS than a workgroup has
            assert e.status == F.EINVAL and (block > 256 or block * ppt * K * K * es > 160 * 1024)
        else:
            Lo, Ro = oracle.eigenvectors(dim, GAMMA, Uo)
            assert blocks_error(host(L), Lo) <= TOL[dt]
            assert blocks_error(host(R), Ro) <= TOL[dt]
        fb = inputs.cotangent(dim, n, 91).astype(np.float32 if dt == "f32" else np.float64)
        import torch
        Fbg = F.to_fields(torch.from_numpy(fb).cuda())
        Ub = _with_config("adjoint", dim, code, cfg, lambda: F.flux_adjoint(Ug, Fbg, GAMMA))
        fb = fb.astype(np.float64)
        A = np.abs(oracle.flux_jacobian(dim, GAMMA, Uo))
        den = np.zeros((K, n))
        for d in range(dim):
            den += np.einsum("nrc,rn->cn", A[d], np.abs(np.array([fb[q * dim + d] for q in range(K)])))
        assert group_error(host(Ub), oracle.flux_adjoint(dim, -1, GAMMA, Uo, fb), [list(range(K))],
                           denom=den.max(axis=0)) <= TOL[dt]
        URo, URg = states(dim, n, 92, dt)
        Uh = _with_config("roe_average", dim, code, cfg, lambda: F.roe_average(Ug, URg, GAMMA))
        assert roe_error(host(Uh), oracle.roe_average(dim, GAMMA, Uo, URo), Uo, URo) <= TOL[dt]


def test_shipped_small_entries_are_what_small_calls_use():
    """The shipped table gives calls of up to max_n points their own launch
    configuration, and calls above it the large one."""
    from paper_1809_09851_amd import tune
    entries = (tune.load_table() or {}).get(tune.arch_key(), {})
    small = {k: v for k, v in entries.items() if k.startswith("small/")}
    assert len(small) > 50
    for name, e in small.items():
        _, op, dim, dt = name.split("/")
        code, dim = tune.DT[dt][0], int(dim)
        assert F.fdbb_get_small_launch_config(op, dim, code) == (
            e["max_n"], e["block"], e["ppt"], e["grid_cap"], e["nt"]), name
        assert F.fdbb_launch_config_for(op, dim, code, e["max_n"] + 1) == F.fdbb_get_launch_config(op, dim, code)


@pytest.mark.parametrize("op", ["cons2prim", "eos", "flux"])
def test_1d_ops_on_both_sides_of_the_small_bound(op):
    """The 1D ops of a step at the last size of the small class and the
    first of the large one, every point against the oracle."""
    m = F.fdbb_get_small_launch_config(op, 1, F.F64)[0]
    assert m > 0
    for n in (m, m + 1):
        Uo, Ug = states(1, n, 90 + (n & 1), "f64")
        if op == "cons2prim":
            assert group_error(host(F.cons2prim(Ug, GAMMA)), oracle.cons2prim(1, GAMMA, Uo), state_groups(1)) <= TOL["f64"]
        elif op == "eos":
            p, c = F.eos(Ug, GAMMA)
            po, co = oracle.eos(1, GAMMA, Uo)
            assert group_error(host(p)[None], po[None], [[0]]) <= TOL["f64"]
            assert group_error(host(c)[None], co[None], [[0]]) <= TOL["f64"]
        else:
            assert group_error(host(F.flux(Ug, GAMMA)), oracle.flux(1, GAMMA, Uo), flux_groups(1)) <= TOL["f64"]


@pytest.fixture
def large_configs_only():
    """Lift every small-launch entry for the test, so that calls of any size
    run with the large (2 GB-tuned) configurations; restored afterwards."""
    saved = []
    for op in F.OPS:
        for dim in (1, 2, 3):
            for code in (F.F64, F.F32):
                entry = F.fdbb_get_small_launch_config(op, dim, code)
                if entry[0]:
                    saved.append((op, dim, code, entry))
                    F.fdbb_set_small_launch_config(op, dim, code, 0)
    yield
    for op, dim, code, entry in saved:
        F.fdbb_set_small_launch_config(op, dim, code, *entry)


@pytest.mark.parametrize("dt", ("f64", "f32"))
@pytest.mark.parametrize("dim", (1, 2, 3))
def test_every_op_with_its_installed_large_configuration(large_configs_only, dim, dt):
    """The parity checks of every entry point, on a ragged multi-tile size,
    with the configurations calls above the small-launch bound use."""
    import test_gpu_parity as P
    n = 5003
    assert F.fdbb_launch_config_for("cons2char", dim, F.F64 if dt == "f64" else F.F32, n) == \
        F.fdbb_get_launch_config("cons2char", dim, F.F64 if dt == "f64" else F.F32)
    for fn in (P.test_cons2prim, P.test_prim2cons, P.test_eos, P.test_velocity_magnitude2, P.test_flux,
               P.test_flux_jacobian, P.test_riemann_invariants, P.test_characteristic_transforms,
               P.test_flux_direction, P.test_fused, P.test_adjoint, P.test_eigenvectors, P.test_char_apply,
               P.test_roe_average, P.test_viscous_flux):
        fn(dim, dt, n)
    for case in range(len(P.EOS_CASES)):
        P.test_eos_pvt(dim, dt, n, case)
