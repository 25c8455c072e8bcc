"""The allocation-free batch entry point (fdbb_batch_run_noalloc) against
the plan-based batch launch it mirrors: same tasks, same kernel, results
equal to the plan's within the FP64 / FP32 contract, on two calls in a row
(the second with fewer, smaller tasks), checked only after both ran."""
import numpy as np
import pytest
import torch

from gpu_common import GAMMA, host, require_gpu, states
from metrics import TOL, blocks_error, flux_groups, group_error, riemann_groups, state_groups
from paper_1809_09851_amd import batch as B
from paper_1809_09851_amd import fdbb as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _mixed(nb, seed, dt, lo, hi):
    """Blocks of random sizes and dims, each with the op it will run."""
    rng = np.random.default_rng(seed)
    spec = []
    for b in range(nb):
        n = int(rng.integers(lo, hi))
        dim = int(rng.integers(1, 4))
        _, Ug = states(dim, n, seed * 977 + b, dt)
        spec.append((b % 4, dim, Ug))
    return spec


def _build(spec):
    """Tasks over the blocks of `spec`, writing into fresh NaN-filled outputs."""
    tasks, outs = [], []
    for kind, dim, Ug in spec:
        n, K = Ug.shape[1], dim + 2
        if kind == 0:
            o = (F.empty_fields(K * dim, n, Ug.dtype), F.empty_blocks(dim, n, Ug.dtype),
                 F.empty_fields(2 * dim + 1, n, Ug.dtype))
            tasks.append(B.fused_task(Ug, *o, gamma=GAMMA))
        elif kind == 1:
            o = (F.empty_fields(K * dim, n, Ug.dtype),)
            tasks.append(B.flux_task(Ug, *o, gamma=GAMMA))
        elif kind == 2:
            o = (F.empty_fields(K, n, Ug.dtype),)
            tasks.append(B.cons2prim_task(Ug, *o, gamma=GAMMA))
        else:
            o = (F.empty_fields(2 * dim + 1, n, Ug.dtype),)
            tasks.append(B.riemann_task(Ug, *o, gamma=GAMMA))
        for t in o:
            t.fill_(float("nan"))
        outs.append((kind, dim, o))
    return tasks, outs


def _check(outs, ref, dt):
    tol = TOL[dt]
    for (kind, dim, o), (_, _, r) in zip(outs, ref):
        if kind == 0:
            assert group_error(host(o[0]), host(r[0]), flux_groups(dim)) <= tol
            assert blocks_error(host(o[1]), host(r[1])) <= tol
            assert group_error(host(o[2]), host(r[2]), riemann_groups(dim)) <= tol
        elif kind == 1:
            assert group_error(host(o[0]), host(r[0]), flux_groups(dim)) <= tol
        elif kind == 2:
            assert group_error(host(o[0]), host(r[0]), state_groups(dim)) <= tol
        else:
            assert group_error(host(o[0]), host(r[0]), riemann_groups(dim)) <= tol


@pytest.mark.parametrize("dt", ("f64", "f32"))
def test_noalloc_matches_plan_on_two_calls(dt):
    print(f"noalloc: dt {dt}", flush=True)
    s1 = _mixed(48, 11, dt, 1000, 60000)
    s2 = _mixed(9, 12, dt, 1, 3000)
    t1, o1 = _build(s1)
    t2, o2 = _build(s2)
    r1t, r1 = _build(s1)
    r2t, r2 = _build(s2)
    # reference: the plan path, each list in its own plan
    for tl in (r1t, r2t):
        p = B.Plan(tl, block=256, ppt=1)
        p.run(graph=False)
        torch.cuda.synchronize()
        p.close()
    # two allocation-free calls back to back on one stream, checked after both
    B.run_noalloc(t1, block=256, ppt=1)
    B.run_noalloc(t2, block=256, ppt=1)
    torch.cuda.synchronize()
    _check(o1, r1, dt)
    _check(o2, r2, dt)


def test_noalloc_limits_and_empty_list():
    print("noalloc: limits", flush=True)
    with pytest.raises(F.FdbbError) as e:
        B.run_noalloc([B._task("flux", 3, 0, GAMMA, 0)] * (B.MAX_NOALLOC_TASKS + 1))
    assert e.value.status == F.EINVAL
    B.run_noalloc([])  # nothing to do
    with pytest.raises(F.FdbbError):
        B.run_noalloc([B._task("flux", 3, 0, GAMMA, 10)], block=512)
    torch.cuda.synchronize()
