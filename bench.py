"""Throughput of the fused 3D Euler pass (flux tensor + three 5x5 flux
Jacobians + Riemann invariants) on one MI355X, against the HBM roofline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--extras]

One step is one fused pass over N = 2^24 points of a seeded synthetic 3D
state (rho, p ~ U[0.5, 2], v_i ~ N(0, 0.5^2)), FP64 storage, inputs and
outputs resident in HBM.  Prints one JSON line with the roofline (HIP-event
time, HBM traffic from the committed counter record), the CPU oracle's rate
and the served p50/p99 latencies of the request server.  ``--extras`` adds
the other building blocks (FP32 storage, the three-launch form, 1D ops,
adjoint, autograd, batches, HBM probes, every single-op entry point);
``--paper-sweeps`` the paper's two experiments over N = 2^10..2^28.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "3D Euler flux+Jacobian Gpoints/s, % HBM roofline; served p50/p99 latency"
GAMMA = 1.4

# Algorithmic bytes per point (each input read once, each output written once).
def fused_bytes(dim: int, es: int) -> int:
    K = dim + 2
    return es * (K + K * dim + dim * K * K + 2 * dim + 1)


PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "fused3d_f64_2p24_traffic.json")


def measured_traffic(n: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    from paper_1809_09851_amd import traffic
    return traffic.load_bytes_per_launch(PROFILE_TRAFFIC, n)


def box_state(root: str = "/sys/class/drm"):
    """The GPU's clock, power and partition settings from sysfs (read-only
    files of the amdgpu driver), so that a bench line says which machine
    state it was measured in.  Missing files are left out."""
    import glob

    def read(path):
        try:
            with open(path) as f:
                return f.read().strip()
        except OSError:
            return None

    def current_level(text):
        # "0: 2000Mhz *" -> "2000Mhz" (the level marked current)
        for ln in (text or "").splitlines():
            if ln.strip().endswith("*"):
                return ln.split(":", 1)[1].replace("*", "").strip()
        return None

    for dev in sorted(glob.glob(os.path.join(root, "card*", "device"))):
        if read(os.path.join(dev, "vendor")) != "0x1002":
            continue
        out = {"pci": os.path.basename(os.path.realpath(dev))}
        mp = read(os.path.join(dev, "current_memory_partition"))
        cp = read(os.path.join(dev, "current_compute_partition"))
        if mp:
            out["memory_partition"] = mp
        if cp:
            out["compute_partition"] = cp
        mclk = current_level(read(os.path.join(dev, "pp_dpm_mclk")))
        if mclk:
            out["hbm_clock"] = mclk
        sclk = read(os.path.join(dev, "pp_dpm_sclk"))
        if sclk:
            levels = [ln.split(":", 1)[1].replace("*", "").strip() for ln in sclk.splitlines() if ":" in ln]
            out["gfx_clock_levels"] = levels
        perf = read(os.path.join(dev, "power_dpm_force_performance_level"))
        if perf:
            out["performance_level"] = perf
        for hw in sorted(glob.glob(os.path.join(dev, "hwmon", "hwmon*"))):
            cap = read(os.path.join(hw, "power1_cap"))
            if cap and cap.isdigit():
                out["power_cap_w"] = int(cap) / 1e6
                break
        vram = read(os.path.join(dev, "mem_info_vram_total"))
        if vram and vram.isdigit():
            out["vram_gib"] = round(int(vram) / 2 ** 30, 1)
        used = read(os.path.join(dev, "mem_info_vram_used"))
        if used and used.isdigit():
            out["vram_used_at_start_gib"] = round(int(used) / 2 ** 30, 3)
        # pages the driver has retired for memory errors (one line each)
        bad = read(os.path.join(dev, "ras", "gpu_vram_bad_pages"))
        if bad is not None:
            out["retired_vram_pages"] = sum(1 for ln in bad.splitlines() if ln.strip())
        fclk = current_level(read(os.path.join(dev, "pp_dpm_fclk")))
        if fclk:
            out["fabric_clock"] = fclk
        return out
    return None


def timed_launches(fn, steps: int, warmup: int):
    """Run fn() warmup + steps times; returns (wall ms per step, mean HIP-event
    ms per launch), events recorded on the stream the kernels run on."""
    import torch
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        fn()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ev = sum(s.elapsed_time(e) for s, e in zip(starts, ends)) / steps
    return wall, ev


def queued_launches(fn, launches: int):
    """Mean HIP-event milliseconds per launch of `launches` back-to-back
    calls of fn() (one event pair around all of them, after one warm-up
    pass): the device's rate when the host keeps the stream fed."""
    import torch
    for _ in range(launches):
        fn()
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(launches):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / launches


def device_state(dim: int, n: int, seed: int, dtype):
    """Seeded primitive state -> GPU -> conservative state via the library."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    from paper_1809_09851_amd import inputs
    V = inputs.gaussian(dim, n, seed) if dim > 1 else inputs.uniform_1d(n, seed)
    Vg = F.to_fields(torch.from_numpy(V).to(dtype).cuda())
    Ug = F.empty_fields(dim + 2, n, dtype)
    F.fdbb_prim2cons(dim, GAMMA, Vg, Ug)
    torch.cuda.synchronize()
    del Vg
    return Ug


def cpu_baseline(n_sample: int = 1 << 24, seed: int = 1):
    """The oracle's fused pass (flux, Jacobians, invariants) on the first
    n_sample points of the same workload, split over host threads, each
    calling the unchanged single-threaded oracle on its own range."""
    import numpy as np
    import oracle
    from paper_1809_09851_amd import inputs
    V = inputs.gaussian(3, n_sample, seed)
    U = oracle.prim2cons(3, GAMMA, V)
    threads = max(1, min(16, os.cpu_count() or 1))
    chunk = 1 << 14
    ranges = [(s, min(s + chunk, n_sample)) for s in range(0, n_sample, chunk)]
    lock = threading.Lock()
    todo = list(ranges)

    def worker():
        while True:
            with lock:
                if not todo:
                    return
                a, b = todo.pop()
            Us = np.ascontiguousarray(U[:, a:b])
            oracle.flux(3, GAMMA, Us)
            oracle.flux_jacobian(3, GAMMA, Us)
            oracle.riemann_invariants(3, GAMMA, Us)

    # whole passes over the sample until about 10 s of CPU work is done
    passes, wall = 0, 0.0
    while passes < 20 and (passes == 0 or wall * threads < 10.0):
        todo[:] = list(ranges)
        t0 = time.perf_counter()
        ts = [threading.Thread(target=worker) for _ in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        wall += time.perf_counter() - t0
        passes += 1
    # one core, best of 3 over the first 2^20 points, for reference
    n1 = min(n_sample, 1 << 20)
    U1 = np.ascontiguousarray(U[:, :n1])
    best = float("inf")
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.flux(3, GAMMA, U1)
        oracle.flux_jacobian(3, GAMMA, U1)
        oracle.riemann_invariants(3, GAMMA, U1)
        best = min(best, time.perf_counter() - t0)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
    except OSError:
        pass
    return {"value": round(passes * n_sample / wall / 1e9, 6), "unit": "Gpoints/s", "cores": threads,
            "kind": "oracle", "single_core_value": round(n1 / best / 1e9, 6), "cpu": model,
            "host_cpus": os.cpu_count(),
            "sample": f"{passes} passes over the first {n_sample} points of the 3D N=2^24 workload "
                      f"(seed 1), fused flux+Jacobians+invariants, {threads} threads on disjoint "
                      f"2^14-point ranges, {wall:.2f} s wall"}


def bench_fused(n: int, steps: int, warmup: int, dtype, label: str):
    import torch
    from paper_1809_09851_amd import fdbb as F
    dim = 3
    U = device_state(dim, n, 1, dtype)
    Fg = F.empty_fields(15, n, dtype)
    A = F.empty_blocks(dim, n, dtype)
    R = F.empty_fields(7, n, dtype)

    def step():
        F.fdbb_euler_fused(dim, GAMMA, U, Fg, A, R)

    wall, ev = timed_launches(step, steps, warmup)
    es = 8 if dtype == torch.float64 else 4
    nbytes = fused_bytes(dim, es) * n
    out = {"label": label, "n": n, "wall_ms": wall, "kernel_ms": ev,
           "gpoints_s": n / (wall * 1e-3) / 1e9, "kernel_gpoints_s": n / (ev * 1e-3) / 1e9,
           "algorithmic_bytes": nbytes, "achieved_gbs": nbytes / (ev * 1e-3) / 1e9}
    del U, Fg, A, R
    torch.cuda.empty_cache()
    return out


def bench_reallocations(n: int, count: int, steps: int = 5, warmup: int = 2):
    """The fused 3D FP64 pass on `count` fresh sets of buffers (inputs and
    outputs allocated anew each time, the allocator's cache emptied first):
    mean HIP-event ms per launch for each allocation.  On this device the
    pass's time depends on the allocation it runs in."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    V = device_state(3, n, 1, torch.float64)
    out = []
    for _ in range(count):
        torch.cuda.empty_cache()
        U = F.empty_fields(5, n, torch.float64)
        U.copy_(V)
        Fo, A, R = F.empty_fields(15, n), F.empty_blocks(3, n), F.empty_fields(7, n)
        _, ev = timed_launches(lambda: F.fdbb_euler_fused(3, GAMMA, U, Fo, A, R), steps, warmup)
        out.append(round(ev, 4))
        print(f"# fused 3D f64 on allocation {len(out)}: {ev:.4f} ms", file=sys.stderr, flush=True)
        del U, Fo, A, R
    del V
    torch.cuda.empty_cache()
    return out


def bench_separate(n: int, steps: int, warmup: int, dtype):
    """The plain form: flux, Jacobian and invariants as three launches."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    dim = 3
    U = device_state(dim, n, 1, dtype)
    Fg = F.empty_fields(15, n, dtype)
    A = F.empty_blocks(dim, n, dtype)
    R = F.empty_fields(7, n, dtype)

    def step():
        F.fdbb_flux(dim, GAMMA, U, Fg)
        F.fdbb_flux_jacobian(dim, GAMMA, U, A)
        F.fdbb_riemann_invariants(dim, GAMMA, U, R)

    wall, ev = timed_launches(step, steps, warmup)
    del U, Fg, A, R
    torch.cuda.empty_cache()
    return {"label": "3d_f64_three_launches", "n": n, "wall_ms": wall,
            "gpoints_s": n / (wall * 1e-3) / 1e9}


def bench_1d(steps: int, warmup: int):
    """1D ops at N = 2^20, FP64; 32 rotating buffer sets so that the working
    set (~1.6 GB) exceeds the 256 MB last-level cache.  Each op is timed one
    launch per event pair (what a single call costs, launch latency
    included) and as back-to-back launches (`queued_*`: the device's rate
    while the host keeps the stream fed)."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    n = 1 << 20
    sets = 32
    base = device_state(1, n, 0, torch.float64)
    Us = [base.clone() for _ in range(sets)]
    Vs = [F.empty_fields(3, n) for _ in range(sets)]
    Fs = [F.empty_fields(3, n) for _ in range(sets)]
    ps = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(sets)]
    cs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(sets)]
    res = {}
    for name, bpp, fn in (
        ("cons2prim", 48, lambda k: F.fdbb_cons2prim(1, GAMMA, Us[k], Vs[k])),
        ("eos", 40, lambda k: F.fdbb_eos(1, GAMMA, Us[k], ps[k], cs[k])),
        ("flux", 48, lambda k: F.fdbb_flux(1, GAMMA, Us[k], Fs[k])),
    ):
        ctr = [0]

        def step():
            fn(ctr[0] % sets)
            ctr[0] += 1

        wall, ev = timed_launches(step, max(steps, sets), warmup)
        q = queued_launches(step, 8 * sets)
        res[name] = {"gpoints_s": round(n / (ev * 1e-3) / 1e9, 3),
                     "achieved_gbs": round(bpp * n / (ev * 1e-3) / 1e9, 1),
                     "queued_us": round(q * 1e3, 2), "queued_gbs": round(bpp * n / (q * 1e-3) / 1e9, 1),
                     "config": list(F.fdbb_launch_config_for(name, 1, F.F64, n))}
    # the three ops of one step (136 B/pt together) as three launches, as a
    # HIP graph of the three launches, and as one persistent batch launch
    from paper_1809_09851_amd import batch as B
    ctr = [0]

    def three():
        k = ctr[0] % sets
        ctr[0] += 1
        F.fdbb_cons2prim(1, GAMMA, Us[k], Vs[k])
        F.fdbb_eos(1, GAMMA, Us[k], ps[k], cs[k])
        F.fdbb_flux(1, GAMMA, Us[k], Fs[k])

    graphs = []
    for k in range(sets):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            F.fdbb_cons2prim(1, GAMMA, Us[k], Vs[k])
            F.fdbb_eos(1, GAMMA, Us[k], ps[k], cs[k])
            F.fdbb_flux(1, GAMMA, Us[k], Fs[k])
        graphs.append(g)
    plans = [B.Plan([B.cons2prim_task(Us[k], Vs[k], GAMMA), B.eos_task(Us[k], ps[k], cs[k], GAMMA),
                     B.flux_task(Us[k], Fs[k], GAMMA)]) for k in range(sets)]

    def rotate(fns):
        c = [0]

        def step():
            fns[c[0] % sets]()
            c[0] += 1
        return step

    for name, step in (("three_launches", three), ("graph_of_three", rotate([g.replay for g in graphs])),
                       ("one_persistent_launch", rotate([(lambda p=p: p.run(graph=True)) for p in plans]))):
        wall, ev = timed_launches(step, max(steps, sets), warmup)
        res[name] = {"us_per_step": round(ev * 1e3, 2), "gpoints_s": round(n / (ev * 1e-3) / 1e9, 3),
                     "achieved_gbs": round(136 * n / (ev * 1e-3) / 1e9, 1)}
    for p in plans:
        p.close()
    del graphs, plans
    del Us, Vs, Fs, ps, cs
    torch.cuda.empty_cache()
    return res


def bench_adjoint(steps: int, warmup: int):
    import torch
    from paper_1809_09851_amd import fdbb as F
    from paper_1809_09851_amd import inputs
    n = 1 << 22
    res = {}
    for dim in (2, 3):
        K = dim + 2
        U = device_state(dim, n, 3, torch.float64)
        Fb = F.to_fields(torch.from_numpy(inputs.cotangent(dim, n, 3)).cuda())
        Ub = F.empty_fields(K, n)
        wall, ev = timed_launches(lambda: F.fdbb_flux_adjoint(dim, -1, GAMMA, U, Fb, Ub), steps, warmup)
        res[f"{dim}d"] = {"gpoints_s": round(n / (ev * 1e-3) / 1e9, 3),
                          "achieved_gbs": round(K * K * 8 * n / (ev * 1e-3) / 1e9, 1)}
        del U, Fb, Ub
    torch.cuda.empty_cache()
    return res


def bench_autograd(steps: int, warmup: int):
    """Forward + backward of EulerFlux (flux kernel, then adjoint kernel) on
    the 3D N = 2^22 state with loss sum(w . F)."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    from paper_1809_09851_amd import inputs
    from paper_1809_09851_amd.autograd import euler_flux
    n, dim = 1 << 22, 3
    U = device_state(dim, n, 3, torch.float64).requires_grad_(True)
    w = F.to_fields(torch.from_numpy(inputs.cotangent(dim, n, 3)).cuda())

    def step():
        U.grad = None
        (euler_flux(U, GAMMA) * w).sum().backward()

    wall, ev = timed_launches(step, steps, warmup)
    # the library's share: the flux kernel of the forward pass and the
    # adjoint kernel of the backward pass (the loss's product, sum and
    # broadcast gradient are PyTorch's own kernels)
    Ud = U.detach()
    Fo = F.empty_fields(15, n, torch.float64)
    Ub = F.empty_fields(5, n, torch.float64)

    def kernels():
        F.fdbb_flux(dim, GAMMA, Ud, Fo)
        F.fdbb_flux_adjoint(dim, -1, GAMMA, Ud, w, Ub)

    _, ev_k = timed_launches(kernels, steps, warmup)
    del U, w, Ud, Fo, Ub
    torch.cuda.empty_cache()
    return {"n": n, "ms_per_fwd_bwd": round(wall, 4), "gpoints_s": round(n / (wall * 1e-3) / 1e9, 3),
            "flux_and_adjoint_kernels_ms": round(ev_k, 4),
            "kernel_gbs": round(360 * n / (ev_k * 1e-3) / 1e9, 1)}


def bench_serving(rates, count: int, warmup: int, slots: int = 8, batch_mb: float = 64.0,
                  engine: str = "native", budget: int = 200 * 10 ** 9):
    """Poisson request streams: continuous batching against one launch per
    request on a single stream (same requests, same pools), through the
    native server, the Python scheduler, or both."""
    import torch
    from paper_1809_09851_amd import serve as S
    torch.cuda.empty_cache()  # the native server takes its whole budget up front
    pools = S.StatePools()
    out = []
    engines = ("native", "python") if engine == "both" else (engine,)
    for rate in rates:
        for eng in engines:
            for baseline in (False, True):
                if eng == "native":
                    r = S.native_serve_benchmark(rate, count, warmup=warmup, pools=pools, slots=slots,
                                                 mode="single" if baseline else "batched", budget=budget,
                                                 max_batch_bytes=batch_mb * 1e6)
                else:
                    r = S.serve_benchmark(rate, count, warmup=warmup, pools=pools, baseline=baseline,
                                          slots=slots, budget=budget, max_batch_bytes=batch_mb * 1e6)
                r["engine"] = eng
                print(f"# serving {eng} rate={rate:g} {'baseline' if baseline else 'batched'}: "
                      f"p50 {r['p50_ms']} ms p99 {r['p99_ms']} ms, {r['req_s']} req/s",
                      file=sys.stderr, flush=True)
                out.append(r)
    # saturating load: a fixed number of requests outstanding, so that the
    # device never waits for arrivals and the two modes' throughput differs
    sat = {}
    if engine in ("native", "both"):
        for baseline in (False, True):
            mode = "single" if baseline else "batched"
            r = S.native_serve_closed_loop(count, concurrency=64, warmup=warmup, pools=pools, slots=slots,
                                           mode=mode, budget=budget, max_batch_bytes=batch_mb * 1e6)
            print(f"# serving saturated ({r['concurrency']} outstanding) {mode}: {r['req_s']} req/s, "
                  f"{r['gpoints_s']} Gpoints/s, p50 {r['p50_ms']} ms p99 {r['p99_ms']} ms",
                  file=sys.stderr, flush=True)
            sat[mode] = r
    del pools
    return out, sat


def bench_batched(steps: int, warmup: int, dtype, nblocks: int = 512):
    """512 uneven 3D blocks (sizes log-uniform in [1e3, 1e6], 5 % near-vacuum
    points), fused pass: 512 stream launches, one 512-node HIP graph, and one
    persistent graph-captured launch with the autotuned configuration."""
    import torch
    from paper_1809_09851_amd import batch as B
    from paper_1809_09851_amd import fdbb as F
    from paper_1809_09851_amd import inputs
    sizes, Vs = inputs.batched(3, nblocks, seed=2)
    blocks = []
    for V in Vs:
        n = V.shape[1]
        Vg = F.to_fields(torch.from_numpy(V).to(dtype).cuda())
        U = F.empty_fields(5, n, dtype)
        F.fdbb_prim2cons(3, GAMMA, Vg, U)
        blocks.append((U, F.empty_fields(15, n, dtype), F.empty_blocks(3, n, dtype), F.empty_fields(7, n, dtype)))
        del Vg
    del Vs
    torch.cuda.synchronize()
    points = int(sizes.sum())
    es = 8 if dtype == torch.float64 else 4
    nbytes = fused_bytes(3, es) * points
    res = {"blocks": nblocks, "points": points, "algorithmic_gb": round(nbytes / 1e9, 2)}

    def launches():
        for U, Fo, A, R in blocks:
            F.fdbb_euler_fused(3, GAMMA, U, Fo, A, R)

    wall, ev = timed_launches(launches, steps, warmup)
    res["stream_launches"] = {"ms": round(ev, 4), "gpoints_s": round(points / ev / 1e6, 3),
                              "frac": round(nbytes / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        launches()
    wall, ev = timed_launches(g.replay, steps, warmup)
    res["graph_of_launches"] = {"ms": round(ev, 4), "gpoints_s": round(points / ev / 1e6, 3),
                                "frac": round(nbytes / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del g
    tasks = [B.fused_task(U, Fo, A, R, GAMMA) for U, Fo, A, R in blocks]
    # the autotuned batch configuration for this storage type (tune.py's
    # batch entry, installed when the library loads)
    plan = B.Plan(tasks)
    block, ppt, grid, nt = plan.config()
    wall, ev = timed_launches(lambda: plan.run(graph=True), steps, warmup)
    res["persistent_graph"] = {"ms": round(ev, 4), "gpoints_s": round(points / ev / 1e6, 3),
                               "frac": round(nbytes / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "config": {"block": block, "ppt": ppt, "grid": grid, "nontemporal": nt}}
    plan.close()
    del blocks, tasks
    torch.cuda.empty_cache()
    return res


def bench_paper_sweeps(steps: int = 20, warmup: int = 3, lo: int = 10, hi: int = 28):
    """The paper's two experiments on this GPU, over N = 2^lo..2^hi:
    the micro-benchmark expression |v|^2 = (m.m)/(rho rho) of Sec. 3, Eq. 2
    (3D, FP32 storage as in the paper; 20 B and 7 flops per point), and the
    mini-application's repeated evaluation of the 3D inviscid flux tensor
    (FP32 storage, 80 B per point), as time per evaluation."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    from paper_1809_09851_amd import tune
    rows = []
    for e in range(lo, hi + 1):
        n = 1 << e
        U = tune._state(3, n, torch.float32)
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        Fo = F.empty_fields(15, n, torch.float32)
        _, ev_v = timed_launches(lambda: F.fdbb_velocity_magnitude2(3, U, y), steps, warmup)
        _, ev_f = timed_launches(lambda: F.fdbb_flux(3, GAMMA, U, Fo), steps, warmup)
        rows.append({"n": n, "vmag2_us": round(ev_v * 1e3, 2),
                     "vmag2_gbs": round(20 * n / (ev_v * 1e-3) / 1e9, 1),
                     "vmag2_gflops": round(7 * n / (ev_v * 1e-3) / 1e9, 1),
                     "flux_us": round(ev_f * 1e3, 2),
                     "flux_gbs": round(80 * n / (ev_f * 1e-3) / 1e9, 1)})
        print(f"# sweep n=2^{e}: v_mag2 {rows[-1]['vmag2_us']} us, flux {rows[-1]['flux_us']} us",
              file=sys.stderr, flush=True)
        del U, y, Fo
        torch.cuda.empty_cache()
    return rows


def bench_ops(steps: int, warmup: int, dims=(3,), dtypes=("f64", "f32")):
    """Every single-op entry point on its own, at a size whose working set is
    about 2 GB (far above the 256 MB last-level cache): ms per launch and
    algorithmic GB/s against the HBM peak."""
    import torch
    from paper_1809_09851_amd import tune
    out = {}
    ops = ("cons2prim", "prim2cons", "eos", "v_mag2", "flux", "flux_dir", "flux_jacobian", "riemann_invariants",
           "cons2char", "char2cons", "adjoint", "eigenvectors", "char_apply", "roe_average", "eos_pvt",
           "viscous_flux")
    for dim in dims:
        for dt in dtypes:
            dtype = torch.float64 if dt == "f64" else torch.float32
            es = 8 if dt == "f64" else 4
            for op in ops:
                n = tune.auto_size(op, dim, es)
                fn = tune.workload(op, dim, dtype, n)
                _, ev = timed_launches(fn, steps, warmup)
                gbs = tune.bytes_per_point(op, dim, es) * n / (ev * 1e-3) / 1e9
                out[f"{op}/{dim}d/{dt}"] = {"n": n, "kernel_ms": round(ev, 4), "achieved_gbs": round(gbs, 1),
                                            "frac": round(gbs / HBM_PEAK_GBS, 4)}
                del fn
                torch.cuda.empty_cache()
    return out


def write_ceiling(gib: float = 4.0, steps: int = 10, warmup: int = 3) -> float:
    """GB/s of the plain write probe (16-byte non-temporal stores, one per
    thread, over a grid covering the buffer)."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    nbytes = int(gib * (1 << 30))
    b = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    _, ev = timed_launches(lambda: F.probe_write(b, grid=nbytes // 16 // 256), steps, warmup)
    del b
    torch.cuda.empty_cache()
    return nbytes / (ev * 1e-3) / 1e9


def bench_fused_stores(steps: int, warmup: int, n: int = 1 << 24):
    """GB/s of the fused 3D pass's stores alone (constant values in its
    layout, order and tiling; no loads, no arithmetic): the ceiling of its
    store pattern on this device."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    Fo = torch.empty((15, n), dtype=torch.float64, device="cuda")
    R = torch.empty((7, n), dtype=torch.float64, device="cuda")
    A = torch.empty((3, n, 5, 5), dtype=torch.float64, device="cuda")
    _, ev = timed_launches(lambda: F.probe_fused_stores(Fo, R, A, n), steps, warmup)
    del Fo, R, A
    torch.cuda.empty_cache()
    return round(776 * n / (ev * 1e-3) / 1e9, 1)


def bench_probes(steps: int, warmup: int, gib: float = 4.0):
    """What HBM delivers to plain streaming kernels (read, write, copy of
    16-byte accesses): with one access per thread over a grid covering the
    buffer ("flat"), and as a grid-stride loop over 8 workgroups per compute
    unit ("stride")."""
    import torch
    from paper_1809_09851_amd import fdbb as F
    nbytes = int(gib * (1 << 30))
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    flat = nbytes // 16 // 256
    sink = torch.empty(max(flat, 1 << 16), dtype=torch.int64, device="cuda")
    res = {}
    for form, grid in (("flat", flat), ("stride", 0)):
        for name, moved, fn in (("read", nbytes, lambda: F.probe_read(a, sink, grid)),
                                ("write", nbytes, lambda: F.probe_write(b, grid=grid)),
                                ("copy", 2 * nbytes, lambda: F.probe_copy(a, b, grid))):
            _, ev = timed_launches(fn, steps, warmup)
            res[f"{name}_{form}"] = round(moved / (ev * 1e-3) / 1e9, 1)
    del a, b, sink
    torch.cuda.empty_cache()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--extras", action="store_true", help="also time the other building blocks")
    ap.add_argument("--reallocs", type=int, default=6,
                    help="also time the fused pass on this many fresh buffer allocations (0 skips)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve-rates", default="100,300,1000,3000,10000",
                    help="comma-separated Poisson rates (req/s) for the serving measurement; '' skips it")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-engine", choices=("native", "python", "both"), default="native",
                    help="the C++ server (fdbb_server.h), the Python scheduler, or both")
    ap.add_argument("--serve-batch-mb", type=float, default=64.0,
                    help="HBM megabytes one batched launch may move")
    ap.add_argument("--paper-sweeps", action="store_true",
                    help="also run the paper's micro-benchmark and mini-application sweeps (N = 2^10..2^28)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run the 1 GiB copy probe 3 times (hardware byte-counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: every building block is pointwise and one GPU's "
              "share of a sharded run is exactly the single-GPU kernel on N/G points; "
              "use --gpus 1", file=sys.stderr)
        return 2

    box = box_state()  # before the process's first GPU call
    import torch
    from paper_1809_09851_amd import fdbb as F
    if not os.path.exists(F.LIBRARY):
        import __graft_entry__
        __graft_entry__.build()
    F.library()
    torch.cuda.set_device(0)

    main_run = bench_fused(args.n, args.steps, args.warmup, torch.float64, "3d_f64_fused")
    print(f"# fused 3D f64: {main_run['kernel_ms']:.3f} ms/launch, "
          f"{main_run['achieved_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    achieved = main_run["achieved_gbs"]
    traffic = measured_traffic(args.n)
    line = {
        "metric": METRIC,
        "value": round(main_run["gpoints_s"], 4),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["wall_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "euler3d_fused_flux_jacobians_riemann", "n_points": args.n, "dim": 3,
                   "gamma": GAMMA, "storage": "f64",
                   "state": "rho,p~U[0.5,2], v_i~N(0,0.5^2), seed 1"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_point": fused_bytes(3, 8), "kernel_ms": round(main_run["kernel_ms"], 4)},
    }
    if box:
        line["box"] = box
    # the device's own ceiling for a plain write stream (95 % of the fused
    # pass's bytes are writes), measured in the same process
    ceiling = write_ceiling()
    line["roofline"]["measured_write_ceiling_gbs"] = round(ceiling, 1)
    line["roofline"]["frac_of_measured_ceiling"] = round(achieved / ceiling, 4)
    if args.reallocs > 0:
        ms = bench_reallocations(args.n, args.reallocs)
        nbytes = fused_bytes(3, 8) * args.n
        line["allocation_spread"] = {
            "what": "the same pass on freshly allocated buffers, one entry per allocation",
            "kernel_ms": ms, "frac": [round(nbytes / (m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) for m in ms]}
    if args.extras:
        ex = {}
        f32 = bench_fused(args.n, args.steps, args.warmup, torch.float32, "3d_f32_fused")
        ex["fused_3d_f32"] = {"gpoints_s": round(f32["kernel_gpoints_s"], 3),
                              "achieved_gbs": round(f32["achieved_gbs"], 1),
                              "frac": round(f32["achieved_gbs"] / HBM_PEAK_GBS, 4)}
        sep = bench_separate(args.n, max(5, args.steps // 5), 2, torch.float64)
        ex["three_launches_3d_f64"] = {"gpoints_s": round(sep["gpoints_s"], 3)}
        ex["ops_1d_f64_2p20"] = bench_1d(args.steps, args.warmup)
        ex["adjoint_f64_2p22"] = bench_adjoint(args.steps, args.warmup)
        ex["autograd_3d_f64_2p22"] = bench_autograd(max(5, args.steps // 5), 2)
        ex["batched_512_f64"] = bench_batched(5, 2, torch.float64)
        ex["batched_512_f32"] = bench_batched(5, 2, torch.float32)
        ex["hbm_probes_gbs"] = bench_probes(max(10, args.steps // 5), 3)
        ex["fused_store_pattern_gbs"] = bench_fused_stores(max(10, args.steps // 5), 3)
        ex["single_ops_2gb"] = bench_ops(max(10, args.steps // 5), 3)
        line["extras"] = ex
    if args.paper_sweeps:
        line["paper_sweeps"] = bench_paper_sweeps()
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
    if rates:
        sweep, sat = bench_serving(rates, args.serve_count, args.serve_warmup, args.serve_slots,
                                   args.serve_batch_mb, args.serve_engine)
        line["serving"] = sweep
        if sat:
            line["serving_saturated"] = sat
    if args.probe_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            F.probe_copy(a, b)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
