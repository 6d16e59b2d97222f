"""Serving scheduler logic on the CPU: a fake backend that evaluates with the
FP64 oracle and finishes launches on a fake clock."""
import numpy as np

import oracle
from paper_1204_1121_amd.serve import (DONE, FAILED, REJECTED, TIMEOUT, Server,
                                       ServeRequest)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt


class FakeBackend:
    """Same interface as GpuBackend; a launch of n positions takes
    base + n * per_pos seconds of fake time; results come from the oracle."""

    def __init__(self, clock, systems, capacity=100, max_requests=8, slots=2,
                 base=1e-3, per_pos=1e-5, fail_on=()):
        self.clock = clock
        self.systems = systems          # list of (lattice, n, coef)
        self.nsystems = len(systems)
        self.slots_per_system = slots
        self._cap = capacity
        self._maxr = max_requests
        self.base = base
        self.per_pos = per_pos
        self.fail_on = set(fail_on)     # rids whose launch raises in done()
        self.launched = []              # (system, slot, [rids], t_start)
        self.results = {}
        self.bytes_per_pos = [100] * len(systems)

    def capacity(self, s):
        return self._cap

    def max_requests(self, s):
        return self._maxr

    def request_bytes(self, s, npos):
        # per-system bytes per position, indexed like the GPU backend's
        # tables, so a request for an unknown system must be rejected before
        # its size is asked for
        return npos * self.bytes_per_pos[s]

    def launch(self, s, slot, reqs):
        n = sum(r.npos for r in reqs)
        t_end = self.clock() + self.base + n * self.per_pos
        A, nn, c = self.systems[s]
        pos = np.concatenate([r.pos for r in reqs])
        self.results[(s, slot)] = oracle.evaluate(A, nn, c, pos)
        self.launched.append((s, slot, [r.rid for r in reqs], self.clock()))
        return (t_end, [r.rid for r in reqs])

    def done(self, h):
        t_end, rids = h
        if self.clock() >= t_end and self.fail_on.intersection(rids):
            raise RuntimeError("injected device error")
        return self.clock() >= t_end

    def fetch(self, s, slot, row0, npos):
        res = self.results[(s, slot)]
        return {k: v[row0:row0 + npos].copy() for k, v in res.items()}


def make_systems():
    rng = np.random.default_rng(0)
    out = []
    for n, L in (((6, 6, 6), 3), ((5, 7, 6), 2)):
        A = np.diag([4.0, 5.0, 4.5])
        out.append((A, n, rng.uniform(-1, 1, n + (L,))))
    return out


def req(rid, system, k, t=0.0, keep=False, seed=0):
    rng = np.random.default_rng(1000 + rid + seed)
    return ServeRequest(rid, system, rng.uniform(0, 5, (k, 3)), arrival=t, keep=keep)


def drain(server, clock, dt=1e-4, limit=100000):
    for _ in range(limit):
        server.pump()
        if server.idle():
            return
        clock.advance(dt)
    raise AssertionError("server did not drain")


def test_admission_respects_budget():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=100, max_requests=1, slots=8)
    sv = Server(be, budget_bytes=3 * 10 * 100, clock=clock)   # three 10-position requests
    for i in range(9):
        sv.offer(req(i, 0, 10))
    sv.pump()
    assert len(sv.running) == 3 and sv.inflight == 3000
    assert len(sv.queues[0]) == 6
    max_in = 0
    for _ in range(100000):
        sv.pump()
        max_in = max(max_in, sv.inflight)
        if sv.idle():
            break
        clock.advance(1e-4)
    assert max_in <= 3000
    assert all(r.status == DONE for r in sv.finished) and len(sv.finished) == 9


def test_fifo_within_a_system_and_batching():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=50, max_requests=4, slots=1)
    sv = Server(be, budget_bytes=10 ** 9, clock=clock)
    for i in range(12):
        sv.offer(req(i, 0, 10))
    drain(sv, clock)
    order = [rid for (_, _, rids, _) in be.launched for rid in rids]
    assert order == list(range(12))
    # capacity 50 positions / 4 requests per launch: launches of 4, 4, 4
    assert [len(r) for (_, _, r, _) in be.launched] == [4, 4, 4]
    done_t = [r.t_done for r in sorted(sv.finished, key=lambda r: r.rid)]
    assert done_t == sorted(done_t)


def test_slots_free_up_and_late_arrivals_join():
    """Continuous batching: requests arriving while a launch runs go into the
    next launch as soon as a slot frees."""
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=100, max_requests=8, slots=1,
                     base=1e-3, per_pos=0.0)
    sv = Server(be, budget_bytes=10 ** 9, clock=clock)
    sv.offer(req(0, 0, 5))
    sv.pump()
    assert len(be.launched) == 1
    clock.advance(2e-4)
    for i in (1, 2, 3):
        sv.offer(req(i, 0, 5))
    sv.pump()
    assert len(be.launched) == 1              # the only slot is busy
    clock.advance(1e-3)
    sv.pump()                                 # retires launch 0, launches 1..3 together
    assert len(be.launched) == 2 and be.launched[1][2] == [1, 2, 3]
    drain(sv, clock)
    assert all(r.status == DONE for r in sv.finished)


def test_two_systems_run_concurrently():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=100, max_requests=8, slots=1)
    sv = Server(be, budget_bytes=10 ** 9, clock=clock)
    sv.offer(req(0, 0, 5))
    sv.offer(req(1, 1, 5))
    sv.pump()
    assert {ln.system for ln in sv.running} == {0, 1}
    drain(sv, clock)


def test_rejections():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=20)
    sv = Server(be, budget_bytes=1500, clock=clock)
    sv.offer(req(0, 0, 16))      # 1600 bytes > budget
    sv.offer(ServeRequest(1, 0, np.zeros((0, 3))))   # empty
    sv.offer(req(2, 5, 3))       # unknown system
    sv.offer(req(4, -1, 3))      # unknown system
    big = FakeBackend(clock, make_systems(), capacity=20)
    sv2 = Server(big, budget_bytes=10 ** 9, clock=clock)
    sv2.offer(req(3, 0, 21))     # more positions than a launch holds
    st = {r.rid: r.status for r in sv.finished + sv2.finished}
    assert st == {0: REJECTED, 1: REJECTED, 2: REJECTED, 3: REJECTED, 4: REJECTED}
    assert "unknown system" in [r for r in sv.finished if r.rid == 2][0].error
    assert sv.idle() and sv2.idle()


def test_injected_failure_fails_only_its_launch():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=100, max_requests=1, slots=2, fail_on={3})
    sv = Server(be, budget_bytes=10 ** 9, clock=clock)
    for i in range(6):
        sv.offer(req(i, i % 2, 4, keep=True))
    drain(sv, clock)
    st = {r.rid: r.status for r in sv.finished}
    assert st[3] == FAILED and "injected" in [r for r in sv.finished if r.rid == 3][0].error
    assert all(st[i] == DONE for i in (0, 1, 2, 4, 5))
    assert sv.inflight == 0 and all(len(f) == 2 for f in sv.free_slots)


def test_timeouts():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=10, max_requests=1, slots=1,
                     base=5e-3, per_pos=0.0)
    sv = Server(be, budget_bytes=10 ** 9, timeout_s=8e-3, clock=clock)
    for i in range(4):
        sv.offer(req(i, 0, 2))
    drain(sv, clock)
    st = [r.status for r in sorted(sv.finished, key=lambda r: r.rid)]
    assert st[0] == DONE and st[1] == DONE and TIMEOUT in st[2:]


def test_result_alone_equals_result_in_the_mix():
    """Packing requests into a launch and unpacking them gives each request
    exactly what it gets alone (each position is independent)."""
    clock = FakeClock()
    systems = make_systems()
    be = FakeBackend(clock, systems, capacity=200, max_requests=16, slots=2)
    sv = Server(be, budget_bytes=10 ** 9, clock=clock)
    reqs = [req(i, i % 2, 1 + (7 * i) % 13, keep=True) for i in range(20)]
    for r in reqs:
        sv.offer(r)
    drain(sv, clock)
    assert max(len(x[2]) for x in be.launched) > 1      # really batched
    for r in reqs:
        A, n, c = systems[r.system]
        alone = oracle.evaluate(A, n, c, r.pos)
        for k in alone:
            np.testing.assert_array_equal(r.result[k], alone[k])


def test_open_loop_run_reports_latency():
    clock = FakeClock()
    be = FakeBackend(clock, make_systems(), capacity=100, max_requests=8, slots=2)
    sv = Server(be, budget_bytes=10 ** 9, clock=clock)
    reqs = [req(i, i % 2, 3, t=i * 1e-3) for i in range(30)]

    # the fake clock advances by itself each time the server reads it
    def tick():
        clock.advance(2e-5)
        return clock.t
    sv.clock = tick
    st = sv.run(reqs)
    assert st["done"] == 30 and st["p99_ms"] >= st["p50_ms"] > 0
    assert all(r.latency > 0 for r in reqs)
