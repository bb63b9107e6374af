"""Tile shapes for the step kernel.

``bench_tile`` is the launch configuration the benchmark and the full-size
parity test use; ``TUNED`` holds shapes picked by timing sweeps on the
device (``sweep``), keyed by (lattice-size bucket, precision).
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_tiles.json")


def _bucket(nx: int, ny: int) -> str:
    n = max(nx, ny)
    for b in (64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384):
        if n <= b:
            return str(b)
    return "huge"


def _table() -> dict:
    if os.path.exists(TABLE):
        with open(TABLE) as fh:
            return json.load(fh)
    return {}


def bench_tile(nx: int, ny: int, precision: str = "fp64"):
    """(block width, rows, depth) for a lattice; zeros keep the library default."""
    t = _table().get("%s/%s" % (_bucket(nx, ny), precision))
    return (int(t[0]), int(t[1]), int(t[2])) if t else (0, 0, 0)


def sweep(solver, scheme="well_balanced", blocks=(128, 192, 256, 320, 512),
          rows=(8, 16, 24, 32, 48, 64, 96, 128), depths=(1, 2, 3), steps=20):
    """Time each tile shape on an initialised solver; returns
    [(ms_per_step, block, rows, depth), ...] sorted fastest first."""
    import torch
    out = []
    for b in blocks:
      for r in rows:
        for d in depths:
            solver.set_tile(b, r, d)
            solver.step(2, scheme)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            solver.step(steps, scheme)
            e1.record()
            torch.cuda.synchronize()
            out.append((e0.elapsed_time(e1) / steps, b, r, d))
    out.sort()
    return out
