"""Serving policy on the CPU: the Server loop against a fake executor with a
fake clock and a small memory budget (no GPU)."""
import pytest

from paper_2012_11075_amd import inputs as I
from paper_2012_11075_amd.serve import Server, summarise


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeExecutor:
    """Slots with a byte budget; a request converges after `need` steps (its
    rid-derived property), diverges if its density ratio exceeds 500; running
    costs simulated time proportional to active node-steps."""

    def __init__(self, budget, clock, max_slots=8, rate=1e9):
        self.budget, self.clock, self.max_slots, self.rate = budget, clock, max_slots, rate
        self.used = 0
        self.slots = {}
        self.peak = 0
        self.admit_order = []

    def footprint(self, req):
        return req.problem.nx * req.problem.ny * 176

    def need(self, req):
        return 300 + 100 * (req.rid % 7)

    def admit(self, req):
        fp = self.footprint(req)
        if len(self.slots) >= self.max_slots or self.used + fp > self.budget:
            return None
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = [req, 0, "active"]
        self.used += fp
        self.peak = max(self.peak, self.used)
        self.admit_order.append(req.rid)
        return slot

    def run(self, k):
        nodes = 0
        for s in self.slots.values():
            if s[2] == "active":
                s[1] += k
                nodes += s[0].problem.nx * s[0].problem.ny
        self.clock.t += nodes * k / self.rate

    def poll(self):
        out = []
        for slot, s in self.slots.items():
            req, steps, st = s
            if st != "active":
                continue
            ratio = req.problem.physics.rho_l / req.problem.physics.rho_v
            if ratio > 500:
                s[2] = "diverged"
            elif steps >= self.need(req):
                s[2] = "converged"
            elif steps >= req.step_cap:
                s[2] = "capped"
            if s[2] != "active":
                out.append((slot, s[2], {"step": steps, "max_u": 0.0, "mass": 1.0}))
        return out

    def release(self, slot):
        req = self.slots.pop(slot)[0]
        self.used -= self.footprint(req)


def stream(n=30, rate=50.0, cap=50_000):
    return I.request_stream(n, rate, seed=9, side_lo=32, side_hi=256, step_cap=cap)


def test_all_requests_served_within_budget():
    clock = FakeClock()
    reqs = stream()
    budget = 3 * 256 * 256 * 176
    ex = FakeExecutor(budget, clock)
    srv = Server(ex, k=100, clock=clock, sleep=clock.sleep)
    out = srv.serve(reqs)
    assert sorted(o.rid for o in out) == sorted(r.rid for r in reqs)
    assert ex.peak <= budget and ex.used == 0
    assert ex.admit_order == sorted(ex.admit_order, key=lambda rid: reqs[rid].arrival)
    for o in out:
        assert o.latency >= 0 and o.retired >= o.admitted >= o.arrival - 1e-12
        ratio = reqs[o.rid].problem.physics.rho_l / reqs[o.rid].problem.physics.rho_v
        if ratio > 500:
            assert o.status == "diverged"
        else:
            assert o.status == "converged"
            need = ex.need(reqs[o.rid])
            assert need <= o.steps < need + 100
    s = summarise(out, clock.t)
    assert s["requests"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_step_cap_retires():
    clock = FakeClock()
    reqs = stream(10, cap=150)
    ex = FakeExecutor(1 << 40, clock)
    out = Server(ex, k=100, clock=clock, sleep=clock.sleep).serve(reqs)
    for o in out:
        assert o.status in ("capped", "diverged")
        if o.status == "capped":
            assert o.steps == 200


def test_continuous_batching_admits_while_running():
    """A request that arrives while others are on the device is admitted
    before they retire, when space allows."""
    clock = FakeClock()
    reqs = stream(12, rate=1000.0)
    ex = FakeExecutor(1 << 40, clock, max_slots=16, rate=1e7)
    srv = Server(ex, k=100, clock=clock, sleep=clock.sleep)
    srv.serve(reqs)
    first_retire = min(e[3] for e in srv.log if e[0] == "retire")
    admits_before = [e for e in srv.log if e[0] == "admit" and e[3] < first_retire]
    assert len(admits_before) > 1
    assert max(len([1 for e in srv.log[:i] if e[0] == "admit"]) -
               len([1 for e in srv.log[:i] if e[0] == "retire"]) for i in range(len(srv.log))) > 1


def test_oversized_request_is_reported():
    clock = FakeClock()
    reqs = stream(3)
    ex = FakeExecutor(10, clock)
    with pytest.raises(RuntimeError):
        Server(ex, k=100, clock=clock, sleep=clock.sleep).serve(reqs)
