"""Launch-configuration autotuner.

Searches workgroup size x points per thread x grid cap x store mode for an
(op, dim, dtype) at a given problem size, timing each candidate with HIP
events on the launch stream (median of repeated launches), and installs the
fastest with ``fdbb_set_launch_config``.  Results are kept in a JSON table
keyed by device architecture, HIP runtime version and (op, dim, dtype); the
binding applies the table shipped next to the library when it loads it.

    python -m paper_1809_09851_amd.tune --ops fused,flux_jacobian --dims 3 \\
        --dtypes f64,f32 --n 16777216 --write paper_1809_09851_amd/tuned_gfx950.json

The op ``batch`` tunes the persistent batch kernel (block x points per
thread x workgroups per compute unit x store mode) on the 512-block batched
workload and stores it as ``batch/3/<dtype>``; plans created without an
explicit configuration, and the request server, use it.

The op ``serve`` tunes the request server's batch configuration on
batches packed from the serving request mix (``serve_batch/0/mix``).

``--small N`` tunes the small-launch class instead: each candidate runs
back to back over rotating copies of an N-point workload (about 1 GB in
all, so that the last-level cache does not hold them), and a winner more
than 2 % faster than the large configuration at that size is stored as
``small/<op>/<dim>/<dtype>`` with max_n = 2N; calls of up to max_n points
then launch with it (``fdbb_set_small_launch_config``).
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import statistics
import sys

import torch

from . import fdbb as F

GAMMA = 1.4
BLOCKS = (64, 128, 256, 512, 1024)
PPTS = (1, 2, 4)
GRID_CAPS = (0, 2048, 4096, 8192)
STORE_MODES = (1, 0)
# the persistent batch kernel: block x points per thread x workgroups per
# compute unit x store mode (0 regular, 1 nt, 2 nt + sc1)
BATCH_BLOCKS = (64, 128, 256)
BATCH_PPTS = (1, 2, 4, 8)
BATCH_GRID_PER_CU = (1, 2, 4, 8, 16, 64, 256, 1024)
BATCH_STORE_MODES = (1, 2, 0)
DEFAULT_TABLE = os.environ.get(
    "FDBB_TUNED_TABLE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json"))
DT = {"f64": (F.F64, torch.float64), "f32": (F.F32, torch.float32)}


def arch_key() -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}/hip{torch.version.hip}"


def _state(dim, n, dtype, seed=1234):
    """A valid conservative state built on the device (no host data needed)."""
    V = F.empty_fields(dim + 2, n, dtype)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    V[0].uniform_(0.5, 2.0, generator=g)
    for k in range(dim):
        V[1 + k].normal_(0.0, 0.5, generator=g)
    V[dim + 1].uniform_(0.5, 2.0, generator=g)
    U = F.empty_fields(dim + 2, n, dtype)
    F.fdbb_prim2cons(dim, GAMMA, V, U)
    return U


def workload(op: str, dim: int, dtype, n: int):
    """Inputs and outputs resident on the device; returns one launch as a
    closure."""
    K = dim + 2
    U = _state(dim, n, dtype)
    if op == "fused":
        Fo, A, R = (F.empty_fields(K * dim, n, dtype), F.empty_blocks(dim, n, dtype),
                    F.empty_fields(2 * dim + 1, n, dtype))
        return lambda: F.fdbb_euler_fused(dim, GAMMA, U, Fo, A, R)
    if op == "flux_jacobian":
        A = F.empty_blocks(dim, n, dtype)
        return lambda: F.fdbb_flux_jacobian(dim, GAMMA, U, A)
    if op == "flux":
        Fo = F.empty_fields(K * dim, n, dtype)
        return lambda: F.fdbb_flux(dim, GAMMA, U, Fo)
    if op == "flux_dir":
        Fd = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_flux_direction(dim, dim - 1, GAMMA, U, Fd)
    if op == "cons2prim":
        V = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_cons2prim(dim, GAMMA, U, V)
    if op == "prim2cons":
        V = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_prim2cons(dim, GAMMA, U, V)
    if op == "v_mag2":
        y = torch.empty(n, dtype=dtype, device="cuda")
        return lambda: F.fdbb_velocity_magnitude2(dim, U, y)
    if op == "eos":
        p = torch.empty(n, dtype=dtype, device="cuda")
        c = torch.empty(n, dtype=dtype, device="cuda")
        return lambda: F.fdbb_eos(dim, GAMMA, U, p, c)
    if op == "riemann_invariants":
        R = F.empty_fields(2 * dim + 1, n, dtype)
        return lambda: F.fdbb_riemann_invariants(dim, GAMMA, U, R)
    if op == "cons2char":
        W = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_cons2char(dim, 0, GAMMA, U, W)
    if op == "char2cons":
        W = F.empty_fields(K, n, dtype)
        F.fdbb_cons2char(dim, 0, GAMMA, U, W)
        return lambda: F.fdbb_char2cons(dim, 0, GAMMA, W, U)
    if op == "eigenvectors":
        L, R = F.empty_blocks(dim, n, dtype), F.empty_blocks(dim, n, dtype)
        return lambda: F.fdbb_eigenvectors(dim, GAMMA, U, L, R)
    if op == "char_apply":
        X = F.empty_fields(K, n, dtype).normal_()
        Y = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_char_apply(dim, 0, 0, GAMMA, U, X, Y)
    if op == "viscous_flux":
        G = F.empty_fields(dim * dim, n, dtype).normal_()
        gT = F.empty_fields(dim, n, dtype).normal_()
        Fv = F.empty_fields(K * dim, n, dtype)
        return lambda: F.fdbb_viscous_flux(dim, 1e-3, 2e-3, U, G, gT, Fv)
    if op == "eos_pvt":
        p, c, T = (torch.empty(n, dtype=dtype, device="cuda") for _ in range(3))
        return lambda: F.fdbb_eos_pvt(dim, 1, (4.4, 0.1, 2.5), U, p, c, T)
    if op == "roe_average":
        UR = _state(dim, n, dtype, seed=4321)
        Uh = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_roe_average(dim, GAMMA, U, UR, Uh)
    if op == "adjoint":
        Fb = F.empty_fields(K * dim, n, dtype).normal_()
        Ub = F.empty_fields(K, n, dtype)
        return lambda: F.fdbb_flux_adjoint(dim, -1, GAMMA, U, Fb, Ub)
    raise ValueError(op)


def bytes_per_point(op: str, dim: int, elem: int) -> int:
    """Algorithmic HBM bytes per point of one launch of `op`."""
    K = dim + 2
    per = {"cons2prim": 2 * K, "prim2cons": 2 * K, "cons2char": 2 * K, "char2cons": 2 * K,
           "eos": K + 2, "v_mag2": dim + 2, "flux": K + K * dim, "flux_dir": 2 * K, "flux_jacobian": K + dim * K * K,
           "riemann_invariants": K + 2 * dim + 1, "fused": K + K * dim + dim * K * K + 2 * dim + 1,
           "adjoint": K * K, "eigenvectors": K + 2 * dim * K * K, "char_apply": 3 * K,
           "roe_average": 3 * K, "eos_pvt": K + 3, "viscous_flux": K + dim * dim + dim + K * dim}[op]
    return per * elem


def auto_size(op: str, dim: int, elem: int, target_bytes: float = 2e9) -> int:
    """A size whose working set (about 2 GB) is far larger than the 256 MB
    last-level cache, so that the search sees HBM behaviour."""
    n = target_bytes / bytes_per_point(op, dim, elem)
    e = min(27, max(22, int(round(math.log2(n)))))
    return 1 << e


def time_launch(fn, reps: int = 7, warmup: int = 2) -> float:
    """Median milliseconds of one launch, HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def time_queued(fns, launches: int = 256, rounds: int = 2) -> float:
    """Milliseconds per launch of `launches` back-to-back launches cycling
    over `fns` (one event pair around all of them; best of `rounds`)."""
    for f in fns:
        f()
    stream = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(rounds):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for k in range(launches):
            fns[k % len(fns)]()
        b.record(stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b) / launches)
    return best


SMALL_GRID_CAPS = (0, 2048)
SMALL_MIN_GAIN = 0.02


def search_small(op: str, dim: int, dt: str, n: int, verbose=False, target_bytes: float = 1e9):
    """Tune the small-launch class at n points.  Returns (results sorted as
    [(ms, cfg)], the large configuration's ms at this size, max_n installed
    or 0).  Installs the winner for n <= 2n when it beats the large
    configuration by more than SMALL_MIN_GAIN, else removes the entry."""
    code, dtype = DT[dt]
    es = 8 if dt == "f64" else 4
    sets = max(1, min(64, math.ceil(target_bytes / (bytes_per_point(op, dim, es) * n))))
    fns = [workload(op, dim, dtype, n) for _ in range(sets)]
    large = F.fdbb_get_launch_config(op, dim, code)
    F.fdbb_set_small_launch_config(op, dim, code, 0)
    large_ms = time_queued(fns)
    results = []
    for cfg in itertools.product(BLOCKS, PPTS, SMALL_GRID_CAPS, STORE_MODES):
        if F.fdbb_kernel_info(op, dim, code, cfg[1], cfg[3])[1] > 0:
            continue
        try:
            F.fdbb_set_small_launch_config(op, dim, code, n, *cfg)
            ms = time_queued(fns)
        except F.FdbbError:
            continue
        results.append((ms, cfg))
        if verbose:
            print(f"  small {op} {dim}d {dt} n={n} cfg={cfg} {ms * 1e3:.2f} us", file=sys.stderr, flush=True)
    results.sort()
    max_n = 0
    if results and results[0][0] < large_ms * (1 - SMALL_MIN_GAIN) and results[0][1] != large:
        max_n = 2 * n
        F.fdbb_set_small_launch_config(op, dim, code, max_n, *results[0][1])
    else:
        F.fdbb_set_small_launch_config(op, dim, code, 0)
    del fns
    torch.cuda.empty_cache()
    return results, large_ms, max_n


def search(op: str, dim: int, dt: str, n: int, reps: int = 7, space=None, verbose=False):
    """Time every candidate; returns [(ms, (block, ppt, grid_cap, nt))] sorted,
    and leaves the fastest installed."""
    code, dtype = DT[dt]
    fn = workload(op, dim, dtype, n)
    space = space or list(itertools.product(BLOCKS, PPTS, GRID_CAPS, STORE_MODES))
    old = F.fdbb_get_launch_config(op, dim, code)
    # a small-launch entry covering n would take over every candidate: lift it
    small = F.fdbb_get_small_launch_config(op, dim, code)
    if small[0] >= n:
        F.fdbb_set_small_launch_config(op, dim, code, 0)
    results = []
    for cfg in space:
        # kernels that spill registers move extra bytes through HBM; skip them
        if F.fdbb_kernel_info(op, dim, code, cfg[1], cfg[3])[1] > 0:
            continue
        try:
            F.fdbb_set_launch_config(op, dim, code, *cfg)
            ms = time_launch(fn, reps)
        except F.FdbbError:
            continue  # a configuration this kernel cannot take (block size, LDS)
        results.append((ms, cfg))
        if verbose:
            print(f"  {op} {dim}d {dt} n={n} cfg={cfg} {ms:.4f} ms", file=sys.stderr, flush=True)
    results.sort()
    F.fdbb_set_launch_config(op, dim, code, *(results[0][1] if results else old))
    if small[0] >= n:
        F.fdbb_set_small_launch_config(op, dim, code, *small)
    return results


def batch_workload(dtype, nblocks: int = 512, seed: int = 2):
    """The batched workload: `nblocks` 3D blocks of sizes log-uniform in
    [10^3, 10^6] points with 5 % near-vacuum points (seeded), each a fused
    pass (flux, Jacobians, invariants) into its own outputs on the device.
    Returns (tasks, points, the tensors the tasks point into)."""
    from . import batch as B
    from . import inputs
    sizes, Vs = inputs.batched(3, nblocks, seed=seed)
    keep, tasks = [], []
    for V in Vs:
        n = V.shape[1]
        Vg = F.to_fields(torch.from_numpy(V).to(dtype).cuda())
        U = F.empty_fields(5, n, dtype)
        F.fdbb_prim2cons(3, GAMMA, Vg, U)
        out = (F.empty_fields(15, n, dtype), F.empty_blocks(3, n, dtype), F.empty_fields(7, n, dtype))
        tasks.append(B.fused_task(U, *out, gamma=GAMMA))
        keep.append((U, out))
        del Vg
    torch.cuda.synchronize()
    return tasks, int(sizes.sum()), keep


def search_batch(dt: str, reps: int = 5, space=None, verbose=False, nblocks: int = 512):
    """Time every batch configuration on the batched workload (one
    persistent graph-captured launch each); returns [(ms, (block, ppt,
    grid_per_cu, nt))] sorted and installs the fastest for `dt`."""
    from . import batch as B
    code, dtype = DT[dt]
    es = 8 if dt == "f64" else 4
    tasks, points, keep = batch_workload(dtype, nblocks)
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    space = space or list(itertools.product(BATCH_BLOCKS, BATCH_PPTS, BATCH_GRID_PER_CU, BATCH_STORE_MODES))
    results = []
    for block, ppt, gpc, nt in space:
        if block * ppt * 25 * es > 160 * 1024:  # 3D Jacobian staging must fit in LDS
            continue
        try:
            plan = B.Plan(tasks, block=block, ppt=ppt, grid=cus * gpc, nontemporal=nt)
        except F.FdbbError:
            continue
        ms = time_launch(lambda: plan.run(graph=True), reps)
        plan.close()
        results.append((ms, (block, ppt, gpc, nt)))
        if verbose:
            print(f"  batch {dt} cfg={(block, ppt, gpc, nt)} {ms:.4f} ms", file=sys.stderr, flush=True)
    results.sort()
    if results:
        F.fdbb_set_batch_config(code, *results[0][1])
    del keep, tasks
    torch.cuda.empty_cache()
    return results, points


def serve_workload(batches: int = 24, seed: int = 7, max_batch: int = 64, max_bytes: float = 64e6):
    """Batches as the request server packs them from the serving request mix
    (inputs.request_stream: the server's ops, D in {1, 2, 3}, N log-uniform
    in [10^3, 10^7], FP64 or FP32, inputs viewed from device-resident state
    pools): consecutive requests while a batch holds at most max_batch
    requests and max_bytes moved bytes.  A request larger than that runs
    alone in the server, not in a batch, and is left out.  Returns (task
    lists, moved bytes of one pass, what the tasks point into)."""
    from . import inputs
    from . import serve
    pools = serve.StatePools(pool=10_000_000, seed=4)
    specs = inputs.request_stream(1e6, 40 * batches * max_batch, seed=seed, pool=pools.pool)
    lists, keep, total = [], [pools], 0
    cur, cur_bytes = [], 0
    for spec in specs:
        r = pools.request(spec)
        m = serve.moved_bytes(r.op, r.dim, r.n, r.elem)
        if m > max_bytes:
            continue
        if cur and (len(cur) == max_batch or cur_bytes + m > max_bytes):
            lists.append(cur)
            total += cur_bytes
            cur, cur_bytes = [], 0
            if len(lists) == batches:
                break
        r.out = serve.allocate_output(r, torch.cuda.current_stream())
        keep.append(r)
        cur.append(serve.batch_task(r))
        cur_bytes += m
    torch.cuda.synchronize()
    return lists, total, keep


def search_serve(reps: int = 3, space=None, verbose=False, batches: int = 24):
    """Time every batch configuration on the server's batches (each a direct
    launch of an empty-created plan updated with the batch, as the server
    runs them); returns [(ms per pass over the batches, (block, ppt,
    grid_per_cu, nt))] sorted, the FP64 batch configuration's ms, and the
    moved bytes of one pass, and installs the fastest as the server's."""
    from . import batch as B
    lists, total, keep = serve_workload(batches)
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    space = space or list(itertools.product(BATCH_BLOCKS, BATCH_PPTS, BATCH_GRID_PER_CU, BATCH_STORE_MODES))
    cap = max(len(t) for t in lists)

    def one(cfg):
        block, ppt, gpc, nt = cfg
        plan = B.Plan([], capacity=cap, block=block, ppt=ppt, grid=cus * (gpc or max(1, 2048 // block)),
                      nontemporal=nt)

        def run():
            for tasks in lists:
                plan.update(tasks)
                plan.run(graph=False)
        try:
            return time_launch(run, reps, 1)
        finally:
            plan.close()

    results = []
    for cfg in space:
        if cfg[0] * cfg[1] * 25 * 8 > 160 * 1024:  # 3D FP64 Jacobian staging must fit in LDS
            continue
        try:
            ms = one(cfg)
        except F.FdbbError:
            continue
        results.append((ms, cfg))
        if verbose:
            print(f"  serve cfg={cfg} {ms:.4f} ms", file=sys.stderr, flush=True)
    results.sort()
    base = F.fdbb_get_batch_config(F.F64)
    base_ms = dict((c, ms) for ms, c in results).get(tuple(base))
    if results:
        F.fdbb_set_server_batch_config(*results[0][1])
    del keep, lists
    torch.cuda.empty_cache()
    return results, base_ms, total


def load_table(path: str = DEFAULT_TABLE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def apply_table(path: str = DEFAULT_TABLE, key: str | None = None) -> int:
    """Install the table's configurations for this device; returns how many."""
    table = load_table(path)
    if not table:
        return 0
    if key is None:
        try:
            key = arch_key()
        except Exception:
            return 0
    entries = table.get(key) or {}
    count = 0
    for name, e in entries.items():
        parts = name.split("/")
        try:
            if parts[0] == "serve_batch":
                F.fdbb_set_server_batch_config(e["block"], e["ppt"], e["grid_per_cu"], e["nt"])
                count += 1
                continue
            if parts[0] == "small" and len(parts) == 4:
                _, op, dim, dt = parts
                F.fdbb_set_small_launch_config(op, int(dim), DT[dt][0], e["max_n"], e["block"], e["ppt"],
                                               e["grid_cap"], e["nt"])
                count += 1
                continue
            op, dim, dt = parts
            code = DT[dt][0]
            if op == "batch":
                F.fdbb_set_batch_config(code, e["block"], e["ppt"], e["grid_per_cu"], e["nt"])
            else:
                F.fdbb_set_launch_config(op, int(dim), code, e["block"], e["ppt"], e["grid_cap"], e["nt"])
        except (F.FdbbError, KeyError, ValueError) as exc:  # an entry this library does not take
            print(f"fdbb: ignoring tuned entry {name}: {exc}", file=sys.stderr)
            continue
        count += 1
    return count


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--ops", default="fused")
    ap.add_argument("--dims", default="3")
    ap.add_argument("--dtypes", default="f64,f32")
    ap.add_argument("--n", default="auto",
                    help="points per launch, or 'auto' for a working set of about 2 GB per op")
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--small", type=int, default=0,
                    help="tune the small-launch class at this many points instead of the large one")
    ap.add_argument("--write", default=None, help="merge results into this JSON table")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    key = arch_key()
    table = (load_table(args.write) if args.write else None) or {}
    entries = table.setdefault(key, {})
    for op in args.ops.split(","):
        if op == "serve":
            res, base_ms, total = search_serve(max(3, args.reps - 4), verbose=args.verbose)
            if res:
                best_ms, (block, ppt, gpc, nt) = res[0]
                entries["serve_batch/0/mix"] = {"block": block, "ppt": ppt, "grid_per_cu": gpc, "nt": nt,
                                                "ms": round(best_ms, 5), "bytes": total,
                                                "fp64_batch_config_ms": round(base_ms, 5) if base_ms else None,
                                                "top5": [[round(ms, 5), list(c)] for ms, c in res[:5]]}
                print(json.dumps({"serve_batch/0/mix": entries["serve_batch/0/mix"]}), flush=True)
            continue
        if op == "batch":
            # the batched workload is 3D whatever --dims says
            for dt in args.dtypes.split(","):
                res, points = search_batch(dt, max(3, args.reps - 2), verbose=args.verbose)
                if not res:
                    continue
                best_ms, (block, ppt, gpc, nt) = res[0]
                base = [ms for ms, cfg in res if cfg == (256, 1, 8, 1)]
                entries[f"batch/3/{dt}"] = {"block": block, "ppt": ppt, "grid_per_cu": gpc, "nt": nt,
                                            "ms": round(best_ms, 5), "n": points,
                                            "default_ms": round(base[0], 5) if base else None,
                                            "top5": [[round(ms, 5), list(c)] for ms, c in res[:5]]}
                print(json.dumps({f"batch/3/{dt}": entries[f"batch/3/{dt}"]}), flush=True)
            continue
        for dim in (int(d) for d in args.dims.split(",")):
            for dt in args.dtypes.split(","):
                if args.small:
                    res, large_ms, max_n = search_small(op, dim, dt, args.small, verbose=args.verbose)
                    name = f"small/{op}/{dim}/{dt}"
                    info = {"n": args.small, "large_us": round(large_ms * 1e3, 3),
                            "top5": [[round(ms * 1e3, 3), list(c)] for ms, c in res[:5]]}
                    if max_n:
                        block, ppt, cap, nt = res[0][1]
                        entries[name] = {"max_n": max_n, "block": block, "ppt": ppt, "grid_cap": cap, "nt": nt,
                                         "us": round(res[0][0] * 1e3, 3), **info}
                    else:
                        entries.pop(name, None)
                    print(json.dumps({name: entries.get(name, {"kept_large": True, **info})}), flush=True)
                    continue
                n = (auto_size(op, dim, 8 if dt == "f64" else 4) if args.n == "auto" else int(args.n))
                res = search(op, dim, dt, n, args.reps, verbose=args.verbose)
                if not res:
                    print(f"fdbb: no usable configuration for {op}/{dim}/{dt} (all spill or are refused)",
                          file=sys.stderr, flush=True)
                    continue
                best_ms, (block, ppt, cap, nt) = res[0]
                base = [ms for ms, cfg in res if cfg == (256, 1 if op in ("fused", "flux_jacobian", "viscous_flux") else
                                                         (2 if dt == "f64" else 4), 0, 1)]
                entries[f"{op}/{dim}/{dt}"] = {"block": block, "ppt": ppt, "grid_cap": cap, "nt": nt,
                                               "ms": round(best_ms, 5), "n": n,
                                               "default_ms": round(base[0], 5) if base else None,
                                               "top5": [[round(ms, 5), list(c)] for ms, c in res[:5]]}
                print(json.dumps({f"{op}/{dim}/{dt}": entries[f"{op}/{dim}/{dt}"]}), flush=True)
    if args.write:
        with open(args.write, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
