"""Host logic of the continuous-batching request loop, on a recording
backend (no device): admission by memory, first come first served, whole
numbers of adaptation intervals per solve, and solves joining while others
are resident."""
import pytest

from paper_2310_07607_amd.serving import Request, Server


class FakeBackend:
    """Records what the loop asks of the device."""

    def __init__(self, footprints, intervals):
        self.fp = footprints        # rid -> bytes
        self.iv = intervals         # rid -> adaptation intervals
        self.opened = []            # rids in admission order
        self.open_now = set()
        self.advances = []          # [set of rids] per tick
        self.adapts = {}            # rid -> number of adaptations
        self.closed = []

    def footprint(self, spec):
        return self.fp[spec["rid"]]

    def intervals(self, spec, t_sim):
        return self.iv[spec["rid"]]

    def open(self, spec):
        rid = spec["rid"]
        self.opened.append(rid)
        self.open_now.add(rid)
        return rid

    def adapt(self, hs):
        for h in hs:
            self.adapts[h] = self.adapts.get(h, 0) + 1

    def advance(self, hs):
        assert set(hs) <= self.open_now
        self.advances.append(set(hs))

    def wait(self):
        pass

    def dof_updates(self, h):
        return 10 * self.adapts[h]

    def result(self, h):
        return {"rid": h, "intervals": sum(h in a for a in self.advances)}

    def close(self, h):
        self.open_now.discard(h)
        self.closed.append(h)


def make(reqs, budget):
    """reqs: [(rid, footprint, intervals, arrival_tick)]"""
    be = FakeBackend({r: f for r, f, _, _ in reqs}, {r: n for r, _, n, _ in reqs})
    srv = Server(be, budget)
    rs = [Request(r, {"rid": r}, 1.0, a) for r, _, _, a in reqs]
    return be, srv, rs


def test_every_request_runs_its_intervals_once_each():
    be, srv, rs = make([(0, 10, 3, 0), (1, 10, 1, 0), (2, 10, 5, 2), (3, 10, 2, 4)], budget=100)
    done = srv.run(rs, realtime=False)
    assert sorted(r.rid for r in done) == [0, 1, 2, 3]
    for r in done:
        assert r.result["intervals"] == be.iv[r.rid]
        assert be.adapts[r.rid] == be.iv[r.rid]  # one adaptation per interval
        assert r.dof_updates == 10 * be.iv[r.rid]
    assert sorted(be.closed) == [0, 1, 2, 3] and not be.open_now
    assert srv.reserved == 0


def test_late_arrivals_join_resident_solves():
    be, srv, rs = make([(0, 10, 6, 0), (1, 10, 2, 1), (2, 10, 2, 2)], budget=100)
    srv.run(rs, realtime=False)
    # request 0 is resident throughout and shares launches with 1 and 2
    assert any({0, 1} <= a for a in be.advances)
    assert any({0, 2} <= a for a in be.advances)
    assert all(0 in a for a in be.advances[:6])


def test_admission_by_memory_first_come_first_served():
    # budget fits two of the 40-byte solves at once; the 10-byte one that
    # arrives last must not overtake the queued 40-byte ones
    reqs = [(0, 40, 4, 0), (1, 40, 4, 0), (2, 40, 2, 0), (3, 10, 1, 0)]
    be, srv, rs = make(reqs, budget=80)
    srv.run(rs, realtime=False)
    assert be.opened == [0, 1, 2, 3]
    assert srv.peak_reserved <= 80
    for a in be.advances:
        assert sum(be.fp[h] for h in a) <= 80
    assert srv.peak_resident == 2


def test_request_above_budget_is_refused():
    be, srv, rs = make([(0, 200, 1, 0)], budget=100)
    with pytest.raises(ValueError):
        srv.run(rs, realtime=False)


def test_idle_gap_before_arrival():
    be, srv, rs = make([(0, 10, 1, 5)], budget=100)
    done = srv.run(rs, realtime=False)
    assert done[0].admitted >= 5
    assert done[0].latency >= 1


def test_realtime_clock_orders_latencies():
    t = [0.0]

    def clock():
        t[0] += 0.001
        return t[0]

    be = FakeBackend({0: 1, 1: 1}, {0: 1, 1: 3})
    srv = Server(be, 10, clock=clock)
    rs = [Request(0, {"rid": 0}, 1.0, 0.0), Request(1, {"rid": 1}, 1.0, 0.0)]
    done = srv.run(rs, realtime=True)
    lat = {r.rid: r.latency for r in done}
    assert 0 < lat[0] < lat[1]
