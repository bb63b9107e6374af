"""Continuous-batching server for run-to-equilibrium requests.

Requests (``inputs.Request``: a lattice problem, a precision, a tolerance on
max|u| and a step cap) arrive over time.  The server keeps every admitted
lattice resident on the device as a batch slot, advances all active slots
together in rounds of ``k`` steps, observes them after each round, retires a
slot when max|u| falls below its tolerance, when it reaches its step cap or
when its state stops being finite, and admits waiting requests as soon as
the freed arena space and slots allow (admission by HBM footprint).

The policy lives in ``Server`` and talks to an executor: ``BatchExecutor``
drives ``lbm.Batch`` on the GPU; tests drive the same policy with a fake
executor and a fake clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: float
    retired: float
    steps: int
    status: str            # "converged", "capped" or "diverged"
    max_u: float
    mass: float
    nodes: int
    precision: str
    result: Optional[dict] = None   # final fields / populations when captured

    @property
    def latency(self) -> float:
        return self.retired - self.arrival


class BatchExecutor:
    """Executor over one ``lbm.Batch`` arena on the current device."""

    def __init__(self, arena_bytes: int, max_slots: int = 1024, graph_steps: int = 0,
                 tiles: Optional[Callable] = None, capture: bool = False):
        from . import lbm
        self.lbm = lbm
        self.capture = capture
        self.batch = lbm.Batch(arena_bytes, max_slots=max_slots)
        if graph_steps:
            self.batch.set_graph_steps(graph_steps)
        self.tiles = tiles

    def params(self, req):
        ph = req.problem.physics
        nz = getattr(req.problem, "nz", 0)
        return self.lbm.make_params(req.problem.nx, req.problem.ny, ph.tau, ph.beta, ph.kappa,
                                    ph.rho_l, ph.rho_v, ph.rho0, precision=req.precision,
                                    force_stencil=getattr(req, "force_stencil", 0), nz=nz,
                                    q3=getattr(req.problem, "q3", 19))

    def footprint(self, req) -> int:
        return self.lbm.Batch.slot_bytes(self.params(req))

    def admit(self, req):
        slot = self.batch.try_admit(self.params(req), req.problem.rho(),
                                    getattr(req, "scheme", "well_balanced"),
                                    tol=req.tol, step_cap=req.step_cap)
        if slot is not None and self.tiles is not None and not getattr(req.problem, "nz", 0):
            tile = self.tiles(req.problem.nx, req.problem.ny, req.precision)
            if tile and getattr(req, "force_stencil", 0):
                # the variant keeps its 256-wide blocks and one step per launch
                tile = (0, tile[1], min(tile[2], 3))
            if tile:
                self.batch.set_tile(slot, *tile)
        return slot

    def run(self, k: int):
        self.batch.run(k)

    def poll(self):
        """[(slot, status, observation)] of the slots retired by this poll."""
        out = []
        for s in self.batch.poll():
            st, ob = self.batch.info(s)
            out.append((s, st, ob))
        return out

    def result(self, slot) -> Optional[dict]:
        """Final fields and populations of a retired slot (when capturing)."""
        if not self.capture:
            return None
        r = self.batch.fetch(slot)
        r["populations"] = self.batch.get_populations(slot)
        return r

    def release(self, slot):
        self.batch.release(slot)

    def sync(self):
        import torch
        torch.cuda.synchronize()

    def close(self):
        self.batch.close()


def nodes_of(problem) -> int:
    """Lattice nodes of a 2-D or 3-D problem."""
    return problem.nx * problem.ny * max(1, getattr(problem, "nz", 0))


@dataclass
class Server:
    """Admission / advance / retirement loop (policy only)."""
    executor: object
    k: int = 200                        # steps per round
    clock: Callable[[], float] = time.perf_counter
    sleep: Callable[[float], None] = time.sleep
    log: list = field(default_factory=list)

    def serve(self, requests, horizon: Optional[float] = None) -> list:
        """Serve ``requests`` (sorted by arrival, seconds after start) until all
        have retired (or ``horizon`` seconds have passed); returns Outcomes."""
        ex = self.executor
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        active = {}            # slot -> (request, admitted time, steps)
        done = []
        t0 = self.clock()
        while pending or waiting or active:
            now = self.clock() - t0
            if horizon is not None and now > horizon:
                break
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admit in arrival order while slots and arena space allow
            while waiting:
                slot = ex.admit(waiting[0])
                if slot is None:
                    break
                req = waiting.popleft()
                active[slot] = [req, self.clock() - t0, 0]
                self.log.append(("admit", req.rid, slot, self.clock() - t0))
            if not active:
                if pending:
                    self.sleep(max(0.0, min(pending[0].arrival - (self.clock() - t0), 0.05)))
                    continue
                if waiting:
                    raise RuntimeError("request %d does not fit in an empty executor"
                                       % waiting[0].rid)
                break
            ex.run(self.k)
            for slot in active:
                active[slot][2] += self.k
            for slot, status, ob in ex.poll():
                req, adm, steps = active.pop(slot)
                res = ex.result(slot) if hasattr(ex, "result") else None
                t = self.clock() - t0
                done.append(Outcome(req.rid, req.arrival, adm, t, int(ob["step"]), status,
                                    float(ob["max_u"]), float(ob["mass"]),
                                    nodes_of(req.problem), req.precision, res))
                ex.release(slot)
                self.log.append(("retire", req.rid, slot, t, status))
        return done


def summarise(outcomes, wall_s: float) -> dict:
    """Latency percentiles over all requests and per outcome (converged,
    capped, diverged), the converged fraction, and the aggregate rate."""
    lat = np.array([o.latency for o in outcomes]) if outcomes else np.zeros(1)
    node_steps = sum(o.nodes * o.steps for o in outcomes)
    by = {}
    for o in outcomes:
        by.setdefault(o.status, []).append(o.latency)
    per = {st: {"count": len(v), "p50_latency_s": float(np.percentile(v, 50)),
                "p99_latency_s": float(np.percentile(v, 99)), "mean_latency_s": float(np.mean(v))}
           for st, v in sorted(by.items())}
    return {"requests": len(outcomes), "wall_s": wall_s,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "aggregate_mlups": node_steps / wall_s / 1e6 if wall_s > 0 else 0.0,
            "outcomes": {st: v["count"] for st, v in per.items()},
            "converged_fraction": (len(by.get("converged", [])) / len(outcomes)) if outcomes else 0.0,
            "by_outcome": per}
