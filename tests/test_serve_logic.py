"""Scheduler logic of the server on the CPU: a fake executor whose results
come from the oracle and whose launches take simulated time on a virtual
clock.  No GPU."""
import numpy as np
import pytest

import oracle
from paper_1809_09851_amd import inputs
from paper_1809_09851_amd.serve import Request, Server, moved_bytes

GAMMA = 1.4


class VirtualClock:
    def __init__(self, dt=1e-6):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


class FakeExecutor:
    """A launch of a batch takes overhead + moved bytes / bandwidth seconds."""

    def __init__(self, clock, bandwidth=5e12, overhead=5e-6):
        self.clock = clock
        self.bw = bandwidth
        self.overhead = overhead
        self.finish = {}
        self.in_flight_max = 0

    def launch(self, slot, batch):
        dur = self.overhead + sum(moved_bytes(r.op, r.dim, r.n, r.elem) for r in batch) / self.bw
        self.finish[slot] = self.clock.t + dur
        for r in batch:
            if r.op == "cons2prim":
                r.out = oracle.cons2prim(r.dim, r.gamma, r.U)
            elif r.op == "flux":
                r.out = oracle.flux(r.dim, r.gamma, r.U)
            elif r.op == "flux_jacobian":
                r.out = oracle.flux_jacobian(r.dim, r.gamma, r.U)
            else:
                r.out = oracle.flux_adjoint(r.dim, -1, r.gamma, r.U, r.Fbar)
        self.in_flight_max = max(self.in_flight_max, len(self.finish))

    def done(self, slot):
        if self.clock.t >= self.finish[slot]:
            return True
        return False

    def release(self, slot):
        self.finish.pop(slot)


def make_requests(count, seed, rate=1e4, nmax=5000):
    specs = inputs.request_stream(rate, count, seed=seed, pool=nmax, lo_exp=1.0, hi_exp=np.log10(nmax))
    reqs = []
    for k, s in enumerate(specs):
        dim, n = s["dim"], s["n"]
        V = inputs.gaussian(dim, n, seed=1000 + k)
        U = oracle.prim2cons(dim, GAMMA, V)
        Fb = inputs.cotangent(dim, n, 2000 + k) if s["op"] == "adjoint" else None
        reqs.append(Request(op=s["op"], dim=dim, n=n, elem=8 if s["dtype"] == "f64" else 4, U=U,
                            Fbar=Fb, t_arrival=s["t"]))
    return reqs


def test_budget_never_exceeded_and_everything_completes():
    clock = VirtualClock()
    reqs = make_requests(200, 1)
    budget = 3 * max(r.out_bytes for r in reqs)
    srv = Server(FakeExecutor(clock), budget, slots=3, max_batch=8, clock=clock)
    done = srv.run_arrivals(reqs)
    assert len(done) == 200
    assert srv.peak_used <= budget
    assert srv.used == 0
    assert all(r.t_done >= r.t_admit >= r.t_arrival for r in done)


def test_fifo_when_one_request_fits_at_a_time():
    clock = VirtualClock()
    reqs = make_requests(40, 2)
    budget = max(r.out_bytes for r in reqs)
    srv = Server(FakeExecutor(clock), budget, slots=4, max_batch=8, clock=clock)
    srv.run_arrivals(reqs)
    by_id = sorted(srv.completed, key=lambda r: r.rid)
    # admitted in arrival order
    assert all(a.t_admit <= b.t_admit for a, b in zip(by_id, by_id[1:]))
    # a request that does not fit next to the running ones waits for memory
    for a, b in zip(by_id, by_id[1:]):
        if a.out_bytes + b.out_bytes > budget:
            assert b.t_admit >= a.t_done


def test_slots_bound_batches_in_flight():
    clock = VirtualClock()
    reqs = make_requests(150, 3)
    ex = FakeExecutor(clock, bandwidth=1e11)
    srv = Server(ex, 10 ** 12, slots=2, max_batch=4, clock=clock)
    srv.run_arrivals(reqs)
    assert ex.in_flight_max <= 2
    assert len(srv.completed) == 150


def test_requests_arriving_during_a_batch_start_before_it_ends():
    """Continuous batching: with a free slot, a late arrival is started while
    an earlier batch is still on the device."""
    clock = VirtualClock()
    reqs = make_requests(2, 4)
    reqs[0].t_arrival, reqs[1].t_arrival = 0.0, 1e-6
    ex = FakeExecutor(clock, bandwidth=1e9)  # slow device: the first batch runs long
    srv = Server(ex, 10 ** 12, slots=2, max_batch=4, clock=clock)
    srv.run_arrivals(reqs)
    a, b = sorted(srv.completed, key=lambda r: r.rid)
    assert b.t_admit < a.t_done


def test_batches_respect_the_byte_cap():
    clock = VirtualClock()
    reqs = make_requests(120, 7)
    cap = 2e6
    seen = []

    class Recording(FakeExecutor):
        def launch(self, slot, batch):
            seen.append(batch)
            super().launch(slot, batch)

    srv = Server(Recording(clock), 10 ** 12, slots=3, max_batch=16, clock=clock, max_batch_bytes=cap)
    srv.run_arrivals(reqs)
    from paper_1809_09851_amd.serve import moved_bytes as mb
    for b in seen:
        if len(b) > 1:
            assert sum(mb(r.op, r.dim, r.n, r.elem) for r in b) <= cap
    assert len(srv.completed) == 120


def test_oversized_request_is_rejected():
    clock = VirtualClock()
    reqs = make_requests(1, 5)
    srv = Server(FakeExecutor(clock), reqs[0].out_bytes - 1, slots=1, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(reqs[0])


def test_result_alone_equals_result_in_the_mix():
    reqs = make_requests(60, 6)
    clock = VirtualClock()
    srv = Server(FakeExecutor(clock), 10 ** 12, slots=3, max_batch=16, clock=clock)
    srv.run_arrivals(reqs)
    mixed = {r.rid: r.out for r in srv.completed}
    for r in make_requests(60, 6)[:10]:
        c2 = VirtualClock()
        s2 = Server(FakeExecutor(c2), 10 ** 12, slots=1, clock=c2)
        (alone,) = s2.run_arrivals([r])
        idx = [q for q in srv.completed if q.n == r.n and q.op == r.op and q.dim == r.dim][0]
        assert np.array_equal(alone.out, mixed[idx.rid])
