"""Request serving with continuous batching.

Requests (cons2prim, flux, flux Jacobian or adjoint over a view of a
device-resident state, any dim, FP64 or FP32 storage) arrive over time.  A
scheduler admits them in arrival order as soon as a launch slot is free and
their outputs fit in the HBM budget, packs every admitted request of a tick
into one persistent batch launch (one batch plan per slot, each slot on its
own stream), and retires requests when their slot's completion event fires,
giving their bytes back to the budget.  Work of different slots overlaps on
the device, so requests that arrive while others run are started as slots
and memory free up.

Two implementations share these rules.  ``NativeServer`` drives the C++
server of fdbb_server.h (scheduler thread, HBM arena, completion events
polled without sleeping); ``native_serve_benchmark`` measures it.
``Server`` is the same scheduler in plain Python over an executor interface
(allocate / launch / done), so its logic is tested on the CPU with a fake
executor and a virtual clock; ``GpuBatchExecutor`` is its GPU executor,
``SingleLaunchExecutor`` the one-launch-per-request FIFO baseline on a
single stream.
"""
from __future__ import annotations

import collections
import dataclasses
import time

OPS = ("cons2prim", "flux", "flux_jacobian", "adjoint")


def out_shape(op: str, dim: int, n: int):
    K = dim + 2
    if op in ("cons2prim", "flux_dir"):
        return ("fields", K)
    if op == "flux":
        return ("fields", K * dim)
    if op == "flux_jacobian":
        return ("blocks", dim)
    if op == "adjoint":
        return ("fields", K)
    raise ValueError(op)


def out_bytes(op: str, dim: int, n: int, elem: int) -> int:
    K = dim + 2
    per_pt = {"cons2prim": K, "flux": K * dim, "flux_jacobian": dim * K * K, "adjoint": K, "flux_dir": K}[op]
    return per_pt * n * elem


def moved_bytes(op: str, dim: int, n: int, elem: int) -> int:
    """Algorithmic HBM bytes of one request (inputs read + outputs written)."""
    K = dim + 2
    per_pt = {"cons2prim": 2 * K, "flux": K + K * dim, "flux_jacobian": K + dim * K * K,
              "adjoint": K + K * dim + K, "flux_dir": 2 * K}[op]
    return per_pt * n * elem


@dataclasses.dataclass(eq=False)
class Request:
    op: str
    dim: int
    n: int
    elem: int                 # bytes per stored value (8 or 4)
    U: object = None          # (K, n) state view on the device
    Fbar: object = None       # (K*D, n) cotangent view (adjoint only)
    gamma: float = 1.4
    t_arrival: float = 0.0    # scheduled arrival, seconds on the server clock
    t_admit: float | None = None
    t_done: float | None = None
    out: object = None
    rid: int = -1

    @property
    def out_bytes(self) -> int:
        return out_bytes(self.op, self.dim, self.n, self.elem)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Server:
    """Continuous-batching scheduler.

    budget_bytes     HBM the outputs of in-flight requests may hold together
    slots            launch slots (batches in flight at once); None = unlimited
    max_batch        requests per launch
    max_batch_bytes  HBM bytes one launch may move; a request that would
                     push a non-empty batch past it starts the next batch,
                     so small requests are not held behind a large one
    """

    def __init__(self, executor, budget_bytes: int, slots: int | None, max_batch: int = 64,
                 clock=time.perf_counter, on_complete=None, max_batch_bytes: float = float("inf")):
        self.ex = executor
        self.max_batch_bytes = max_batch_bytes
        self.on_complete = on_complete  # called with each request as it completes
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak_used = 0
        self.slots = slots
        self.max_batch = max_batch
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.busy: dict[int, list[Request]] = {}
        self.free = list(range(slots))[::-1] if slots is not None else []
        self._fresh_slot = 0 if slots is None else None
        self.completed: list[Request] = []
        self.launches = 0
        self._next_id = 0

    # ---------------------------------------------------------------- intake
    def submit(self, req: Request) -> Request:
        if req.out_bytes > self.budget:
            raise ValueError(f"request needs {req.out_bytes} B of outputs, budget is {self.budget} B")
        req.rid = self._next_id
        self._next_id += 1
        self.queue.append(req)
        return req

    # ---------------------------------------------------------------- ticks
    def poll(self) -> int:
        """Retire every batch whose completion event has fired."""
        done = [s for s in self.busy if self.ex.done(s)]
        if not done:
            return 0
        now = self.clock()
        for s in done:
            for r in self.busy.pop(s):
                r.t_done = now
                self.used -= r.out_bytes
                self.completed.append(r)
                if self.on_complete is not None:
                    self.on_complete(r)
            release = getattr(self.ex, "release", None)
            if release:
                release(s)
            if self.slots is not None:
                self.free.append(s)
        return len(done)

    def _slot_available(self) -> bool:
        return self.slots is None or bool(self.free)

    def _take_slot(self) -> int:
        if self.slots is None:
            self._fresh_slot += 1
            return self._fresh_slot
        return self.free.pop()

    def admit(self) -> int:
        """Start queued requests, oldest first, while a slot is free and the
        next request's outputs fit in what is left of the budget."""
        started = 0
        while self.queue and self._slot_available():
            batch, moved = [], 0
            while (self.queue and len(batch) < self.max_batch
                   and self.used + self.queue[0].out_bytes <= self.budget):
                r = self.queue[0]
                m = moved_bytes(r.op, r.dim, r.n, r.elem)
                if batch and moved + m > self.max_batch_bytes:
                    break
                self.queue.popleft()
                self.used += r.out_bytes
                moved += m
                batch.append(r)
            if not batch:
                break
            self.peak_used = max(self.peak_used, self.used)
            slot = self._take_slot()
            now = self.clock()
            for r in batch:
                r.t_admit = now
            self.ex.launch(slot, batch)
            self.busy[slot] = batch
            self.launches += 1
            started += len(batch)
        return started

    def step(self):
        self.poll()
        self.admit()

    @property
    def idle(self) -> bool:
        return not self.queue and not self.busy

    def drain(self, timeout: float = 60.0):
        t_end = self.clock() + timeout
        while not self.idle:
            self.step()
            if self.clock() > t_end:
                raise TimeoutError("server did not drain")

    def run_arrivals(self, requests, t0: float | None = None):
        """Release each request at its scheduled arrival time (t_arrival
        seconds after t0 on the server clock), run the scheduler until every
        request has completed; returns the completed requests."""
        t0 = self.clock() if t0 is None else t0
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        for r in pending:
            r.t_arrival += t0
        while pending or not self.idle:
            now = self.clock()
            while pending and pending[0].t_arrival <= now:
                self.submit(pending.popleft())
            self.step()
        return self.completed


# -------------------------------------------------------------------- GPU
def allocate_output(r: Request, stream):
    """The request's output tensor, allocated in `stream`'s memory pool."""
    import torch

    from . import fdbb as F
    dtype = torch.float64 if r.elem == 8 else torch.float32
    kind, count = out_shape(r.op, r.dim, r.n)
    with torch.cuda.stream(stream):
        if kind == "fields":
            return F.empty_fields(count, r.n, dtype)
        return F.empty_blocks(r.dim, r.n, dtype)


def batch_task(r: Request):
    """The batch task of an admitted request (its output allocated)."""
    from . import batch as B
    if r.op == "cons2prim":
        return B.cons2prim_task(r.U, r.out, r.gamma)
    if r.op == "flux":
        return B.flux_task(r.U, r.out, r.gamma)
    if r.op == "flux_jacobian":
        return B.jacobian_task(r.U, r.out, r.gamma)
    return B.adjoint_task(r.U, r.Fbar, r.out, r.gamma)


class GpuBatchExecutor:
    """One batch plan and one stream per slot; a launch packs all of its
    requests into the plan's task table and launches the plan directly, with
    the LDS its task list stages."""

    def __init__(self, slots: int, capacity: int = 256, block: int = 0, ppt: int = 1):
        import torch

        from . import batch as B
        from . import fdbb as F
        self.torch = torch
        self.B = B
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        # empty plans reserve LDS for any task (3D FP64 Jacobian staging);
        # block 0 takes the server's batch configuration, as the native server
        if block == 0:
            block, ppt, gpc, nt = F.fdbb_get_server_batch_config()
            cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
            grid = cus * (gpc if gpc > 0 else max(1, 2048 // block))
        else:
            grid, nt = 0, 1
        self.plans = [B.Plan([], capacity=capacity, block=block, ppt=ppt, grid=grid, nontemporal=nt)
                      for _ in range(slots)]
        self.events = [None] * slots

    def allocate(self, r: Request, stream):
        return allocate_output(r, stream)

    def task(self, r: Request):
        return batch_task(r)

    def launch(self, slot: int, batch):
        s = self.streams[slot]
        for r in batch:
            r.out = self.allocate(r, s)
        if len(batch) == 1:
            # a lone request gains nothing from the task table: launch it
            # directly (same per-point code, so the same result bits)
            single_launch(batch[0], s)
        else:
            plan = self.plans[slot]
            plan.update([self.task(r) for r in batch], stream=s)
            plan.run(stream=s, graph=False)
        ev = self.torch.cuda.Event()
        ev.record(s)
        self.events[slot] = ev

    def done(self, slot: int) -> bool:
        return self.events[slot].query()

    def close(self):
        for p in self.plans:
            p.close()


def single_launch(r: Request, stream):
    """Run one request through its single-call entry point on `stream`
    (outputs already allocated in r.out)."""
    from . import fdbb as F
    if r.op == "cons2prim":
        F.fdbb_cons2prim(r.dim, r.gamma, r.U, r.out, stream=stream)
    elif r.op == "flux":
        F.fdbb_flux(r.dim, r.gamma, r.U, r.out, stream=stream)
    elif r.op == "flux_jacobian":
        F.fdbb_flux_jacobian(r.dim, r.gamma, r.U, r.out, stream=stream)
    else:
        F.fdbb_flux_adjoint(r.dim, -1, r.gamma, r.U, r.Fbar, r.out, stream=stream)


class SingleLaunchExecutor:
    """Baseline: each request is its own launch of the single-call entry
    point, all on one stream in arrival order."""

    def __init__(self):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.events = {}

    def launch(self, slot: int, batch):
        torch = self.torch
        s = self.stream
        ev = None
        for r in batch:
            r.out = allocate_output(r, s)
            single_launch(r, s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot] = ev

    def done(self, slot: int) -> bool:
        return self.events[slot].query()

    def release(self, slot: int):
        self.events.pop(slot, None)

    def close(self):
        pass


# -------------------------------------------------------------------- workload
class StatePools:
    """Device-resident states of ``pool`` points for every (dim, dtype), plus
    cotangent pools for the adjoint, generated once from the seeded recipe."""

    def __init__(self, pool: int = 10_000_000, seed: int = 4, dims=(1, 2, 3), elems=(8, 4), gamma=1.4):
        import torch

        from . import fdbb as F
        from . import inputs
        self.pool = pool
        self.U = {}
        self.Fbar = {}
        for dim in dims:
            V = inputs.gaussian(dim, pool, seed + dim)
            W = inputs.cotangent(dim, pool, seed + 10 + dim)
            for elem in elems:
                dtype = torch.float64 if elem == 8 else torch.float32
                Vg = F.to_fields(torch.from_numpy(V).to(dtype).cuda())
                Ug = F.empty_fields(dim + 2, pool, dtype)
                F.fdbb_prim2cons(dim, gamma, Vg, Ug)
                del Vg
                self.U[(dim, elem)] = Ug
                self.Fbar[(dim, elem)] = F.to_fields(torch.from_numpy(W).to(dtype).cuda())
        torch.cuda.synchronize()

    def request(self, spec: dict, gamma: float = 1.4) -> Request:
        """A Request for one entry of inputs.request_stream; the view starts
        at the drawn offset rounded down to a multiple of 64 points so that
        every row stays 16-byte aligned."""
        elem = 8 if spec["dtype"] == "f64" else 4
        dim, n = spec["dim"], spec["n"]
        off = (spec["offset"] // 64) * 64
        U = self.U[(dim, elem)][:, off:off + n]
        Fb = self.Fbar[(dim, elem)][:, off:off + n] if spec["op"] == "adjoint" else None
        return Request(op=spec["op"], dim=dim, n=n, elem=elem, U=U, Fbar=Fb, gamma=gamma,
                       t_arrival=spec["t"])


def summarize(done, t_span: float | None = None):
    import numpy as np
    lat = np.array([r.latency for r in done])
    pts = sum(r.n for r in done)
    moved = sum(moved_bytes(r.op, r.dim, r.n, r.elem) for r in done)
    if t_span is None:
        t_span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
    return {"requests": len(done), "seconds": round(t_span, 4),
            "req_s": round(len(done) / t_span, 1), "gpoints_s": round(pts / t_span / 1e9, 3),
            "gb_s": round(moved / t_span / 1e9, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4)}


def serve_benchmark(rate: float, count: int, warmup: int = 200, slots: int = 8, max_batch: int = 64,
                    budget: int = 200 * 10 ** 9, pools: StatePools | None = None, baseline: bool = False,
                    seed: int = 4, max_batch_bytes: float = 64e6):
    """Poisson arrivals at `rate`; the first `warmup` requests are served but
    not measured.  Returns the summary of the measured requests."""
    import torch

    from . import inputs
    pools = pools or StatePools()
    specs = inputs.request_stream(rate, warmup + count, seed=seed, pool=pools.pool)
    reqs = [pools.request(s) for s in specs]
    def release(r):
        # a served result is handed on; the benchmark drops it at once, so
        # HBM held by outputs is what the budget accounts for
        r.out = None

    if baseline:
        ex = SingleLaunchExecutor()
        srv = Server(ex, budget, slots=None, max_batch=1, on_complete=release)
    else:
        ex = GpuBatchExecutor(slots)
        srv = Server(ex, budget, slots=slots, max_batch=max_batch, on_complete=release,
                     max_batch_bytes=max_batch_bytes)
    done = srv.run_arrivals(reqs)
    torch.cuda.synchronize()
    measured = [r for r in done if r.rid >= warmup]
    for r in done:
        r.out = None
    out = summarize(measured)
    out.update({"rate": rate, "launches": srv.launches, "peak_budget_bytes": srv.peak_used,
                "mode": "one launch per request, FIFO, single stream" if baseline else
                f"continuous batching, {slots} slots, <= {max_batch} requests and "
                f"<= {max_batch_bytes / 1e6:g} MB per launch"})
    ex.close()
    return out


# -------------------------------------------------------------------- native
class NativeServer:
    """The C++ server of fdbb_server.h: its scheduler thread batches, launches
    and retires requests; outputs live in its HBM arena until released."""

    def __init__(self, budget_bytes: int, slots: int = 8, max_batch: int = 64,
                 max_batch_bytes: float = 64e6, mode: str = "batched"):
        import ctypes

        import torch

        from . import fdbb as F
        # the server's streams are not ordered after torch's: inputs written
        # so far must be complete before requests name them
        torch.cuda.synchronize()
        self.F = F
        self.ct = ctypes
        self._h = ctypes.c_void_p()
        code = 0 if mode == "batched" else 1
        F.check(F.library().fdbb_server_create(int(budget_bytes), slots, max_batch, float(max_batch_bytes),
                                               code, ctypes.byref(self._h)))
        self._buf = (F.Completion * 1024)()
        self._count = ctypes.c_int()

    def submit(self, task, tag: int):
        self.F.check(self.F.library().fdbb_server_submit(self._h, self.ct.byref(task), tag))

    def poll(self):
        lib = self.F.library()
        out = []
        while True:
            self.F.check(lib.fdbb_server_poll(self._h, self._buf, len(self._buf), self.ct.byref(self._count)))
            k = self._count.value
            out.extend(self._buf[i] for i in range(k))
            if k < len(self._buf):
                return out

    def release(self, tag: int):
        self.F.check(self.F.library().fdbb_server_release(self._h, tag))

    def stats(self) -> dict:
        st = self.F.ServerStats()
        self.F.check(self.F.library().fdbb_server_get_stats(self._h, self.ct.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if self._h and self._h.value:
            self.F.library().fdbb_server_destroy(self._h)
            self._h = self.ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Server-owned device memory described for torch.as_tensor (the array
    interface: pointer, shape, element type; C-contiguous)."""

    def __init__(self, ptr: int, shape, elem: int):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": tuple(int(x) for x in shape),
                                         "typestr": "<f8" if elem == 8 else "<f4", "version": 2,
                                         "strides": None}


def completion_outputs(c, op: str, dim: int, n: int, elem: int):
    """Zero-copy tensors over a native completion's outputs in the server's
    arena, in the layouts of the single-call entry points (fields (count, n),
    blocks (D, n, K, K); the fused op gives (F, A, R), eos (p, c)).  They are
    valid until the request is released."""
    import torch
    K = dim + 2
    ld = int(c.ld)

    def fields(ptr, count):
        return torch.as_tensor(_DeviceArray(ptr, (count, ld), elem), device="cuda")[:, :n]

    def blocks(ptr):
        return torch.as_tensor(_DeviceArray(ptr, (dim, ld, K, K), elem), device="cuda")[:, :n]

    def single(ptr):
        return torch.as_tensor(_DeviceArray(ptr, (ld,), elem), device="cuda")[:n]

    if op in ("cons2prim", "prim2cons", "cons2char", "char2cons", "adjoint", "roe_average", "flux_dir"):
        return (fields(c.out0, K),)
    if op == "flux":
        return (fields(c.out0, K * dim),)
    if op == "riemann_invariants":
        return (fields(c.out0, 2 * dim + 1),)
    if op == "flux_jacobian":
        return (blocks(c.out0),)
    if op == "v_mag2":
        return (single(c.out0),)
    if op == "eos":
        return (single(c.out0), single(c.out1))
    if op == "fused":
        return (fields(c.out0, K * dim), blocks(c.out1), fields(c.out2, 2 * dim + 1))
    raise ValueError(op)


def request_task(r: Request):
    """The fdbb_task of a request (outputs are placed by the server)."""
    from . import batch as B
    from . import fdbb as F
    op = r.op
    t = B._task(op, r.dim, F.dtype_code(r.U.dtype), r.gamma, r.n, -1 if op == "adjoint" else 0)
    B._set(t, "in0", r.U, r.dim + 2)
    if op == "adjoint":
        B._set(t, "in1", r.Fbar, (r.dim + 2) * r.dim)
    return t


def native_serve_benchmark(rate: float, count: int, warmup: int = 200, slots: int = 8, max_batch: int = 64,
                           budget: int = 200 * 10 ** 9, pools: StatePools | None = None, mode: str = "batched",
                           seed: int = 4, max_batch_bytes: float = 64e6):
    """Poisson arrivals at `rate` into the native server; latency runs from
    each request's scheduled arrival to its completion event (both on the
    monotonic clock).  The first `warmup` requests are not measured."""
    import numpy as np

    from . import inputs
    pools = pools or StatePools()
    specs = inputs.request_stream(rate, warmup + count, seed=seed, pool=pools.pool)
    reqs = [pools.request(s) for s in specs]
    tasks = [request_task(r) for r in reqs]
    srv = NativeServer(budget, slots=slots, max_batch=max_batch, max_batch_bytes=max_batch_bytes, mode=mode)
    t0 = time.monotonic_ns() + 2_000_000
    arrival = [t0 + int(r.t_arrival * 1e9) for r in reqs]
    done = {}
    k = 0
    while len(done) < len(reqs):
        now = time.monotonic_ns()
        while k < len(reqs) and arrival[k] <= now:
            srv.submit(tasks[k], k)
            k += 1
        for c in srv.poll():
            if c.status != 0:
                raise RuntimeError(f"request {c.tag} failed")
            done[c.tag] = c.t_done_ns
            srv.release(c.tag)
    st = srv.stats()
    srv.close()
    ids = range(warmup, warmup + count)
    lat = np.array([(done[i] - arrival[i]) * 1e-9 for i in ids])
    span = (max(done[i] for i in ids) - min(arrival[i] for i in ids)) * 1e-9
    pts = sum(reqs[i].n for i in ids)
    moved = sum(moved_bytes(reqs[i].op, reqs[i].dim, reqs[i].n, reqs[i].elem) for i in ids)
    return {"requests": count, "seconds": round(span, 4), "req_s": round(count / span, 1),
            "gpoints_s": round(pts / span / 1e9, 3), "gb_s": round(moved / span / 1e9, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4), "rate": rate,
            "launches": st["launches"], "peak_budget_bytes": st["peak_arena_bytes"],
            "mode": ("native server, continuous batching, " f"{slots} slots, <= {max_batch} requests and "
                     f"<= {max_batch_bytes / 1e6:g} MB per launch") if mode == "batched" else
                    "native server, one launch per request, FIFO, single stream"}


def native_serve_closed_loop(count: int, concurrency: int = 64, warmup: int = 200, slots: int = 8,
                             max_batch: int = 64, budget: int = 200 * 10 ** 9, pools: StatePools | None = None,
                             mode: str = "batched", seed: int = 4, max_batch_bytes: float = 64e6):
    """Saturating load: the serving workload's request mix with `concurrency`
    requests outstanding at all times (a new one is submitted as soon as one
    completes), so the device never waits for arrivals.  Throughput counts
    completions over the span from the first measured submission to the last
    measured completion; latency runs from submission to completion (the
    server's clock).  The first `warmup` requests are not measured."""
    import numpy as np

    from . import inputs
    pools = pools or StatePools()
    specs = inputs.request_stream(1.0, warmup + count, seed=seed, pool=pools.pool)
    reqs = [pools.request(s) for s in specs]
    tasks = [request_task(r) for r in reqs]
    srv = NativeServer(budget, slots=slots, max_batch=max_batch, max_batch_bytes=max_batch_bytes, mode=mode)
    sub, done = {}, {}
    k = 0
    while k < min(concurrency, len(reqs)):
        srv.submit(tasks[k], k)
        k += 1
    while len(done) < len(reqs):
        for c in srv.poll():
            if c.status != 0:
                raise RuntimeError(f"request {c.tag} failed")
            sub[c.tag] = c.t_submit_ns
            done[c.tag] = c.t_done_ns
            srv.release(c.tag)
            if k < len(reqs):
                srv.submit(tasks[k], k)
                k += 1
    st = srv.stats()
    srv.close()
    ids = range(warmup, warmup + count)
    lat = np.array([(done[i] - sub[i]) * 1e-9 for i in ids])
    span = (max(done[i] for i in ids) - min(sub[i] for i in ids)) * 1e-9
    pts = sum(reqs[i].n for i in ids)
    moved = sum(moved_bytes(reqs[i].op, reqs[i].dim, reqs[i].n, reqs[i].elem) for i in ids)
    return {"requests": count, "concurrency": concurrency, "seconds": round(span, 4),
            "req_s": round(count / span, 1), "gpoints_s": round(pts / span / 1e9, 3),
            "gb_s": round(moved / span / 1e9, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
            "launches": st["launches"], "peak_budget_bytes": st["peak_arena_bytes"],
            "mode": ("native server, continuous batching, " f"{slots} slots, <= {max_batch} requests and "
                     f"<= {max_batch_bytes / 1e6:g} MB per launch") if mode == "batched" else
                    "native server, one launch per request, FIFO, single stream"}
