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


def two_step_tile(nx: int, ny: int, precision: str = "fp64", cus: int = 256, min_rows: int = 16,
                  max_rows: int = 512):
    """(block, rows, 4) for two steps per launch on an nx x ny lattice, or
    None where one step per launch is the better choice.  The two-step
    kernel runs 128-thread blocks in FP64 and 256-thread blocks in
    FP32-shifted storage (the faster of the two in each, measured at
    4096^2); either takes 66 KB of LDS, so two blocks are resident per
    compute unit, and the tile count should fill whole rounds of them:
    strips of block - 6 columns across x and, for the fewest rounds that
    keep chunks at most `max_rows` tall and the rounds at least 90% full,
    the most chunks whose tiles fit in them.  Chunks under `min_rows` rows
    (a lattice too small to fill the device) would spend most of each
    block in the 12 lead-in rows: None.  For 4096^2 this gives the
    measured best tiles, (128, 274, 4) in FP64 and (256, 137, 4) in
    FP32-shifted storage."""
    block = 256 if precision == "fp32s" else 128
    strips = -(-nx // (block - 6))
    resident = 2 * cus
    c_min = -(-ny // max_rows)
    first = -(-strips * c_min // resident)
    rows = None
    for rounds in range(first, first + 64):
        c = (rounds * resident) // strips
        if c < c_min:
            continue
        rows = -(-ny // c)
        chunks = -(-ny // rows)
        if strips * chunks >= 0.9 * rounds * resident:
            break
    if rows is None or rows < min_rows:
        return None
    return (block, rows, 4)


def batch_bucket(nx: int, ny: int) -> str:
    return _bucket(nx, ny)


def batch_tile(nx: int, ny: int, precision: str = "fp64"):
    """(block, rows, depth) for a lattice inside a batch, or None (library default)."""
    t = _table().get("batch/%s/%s" % (_bucket(nx, ny), precision))
    return (int(t[0]), int(t[1]), int(t[2])) if t else None


def stencil4_tile(nx: int, ny: int, precision: str = "fp64"):
    """(block, rows, depth) of the force-stencil variant's step (measured
    sweep at 4096^2), or None (library default)."""
    t = _table().get("stencil4/%s/%s" % (_bucket(nx, ny), precision))
    return (int(t[0]), int(t[1]), int(t[2])) if t else None


def serve_tile(nx: int, ny: int, precision: str = "fp64"):
    """(block, rows, depth) for a lattice of the served stream, or None.  A
    served batch holds a few tens of lattices at a time, not hundreds, so
    short chunks (more tiles per step) keep the device full: two-step
    tiles of 32 rows, 256-thread blocks in FP32 and 128-thread blocks in
    FP64 (two blocks per CU; p50 latency 3.98 s against 6.49 s for one-step
    tiles of 16 rows, at the same aggregate throughput).  The table covers
    every request size, so all requests of one precision share one launch
    group."""
    t = _table().get("serve/%s/%s" % (_bucket(nx, ny), precision))
    return (int(t[0]), int(t[1]), int(t[2])) if t else None


def tune_batch(problems, precision, blocks=(64, 128, 256), rows=(8, 16, 32, 64), depths=(1, 2, 3),
               steps=40, per_bucket=24):
    """Pick a tile per lattice-size bucket by timing batched launches of up to
    `per_bucket` lattices of that bucket under each candidate tile.
    Returns {bucket: (ms_per_step, block, rows, depth)}."""
    import torch
    from . import lbm
    buckets = {}
    for p in problems:
        buckets.setdefault(_bucket(p.nx, p.ny), []).append(p)
    best = {}
    for bk, probs in sorted(buckets.items(), key=lambda kv: int(kv[0]) if kv[0].isdigit() else 1 << 30):
        probs = probs[:per_bucket]
        prms = [lbm.make_params(p.nx, p.ny, p.physics.tau, p.physics.beta, p.physics.kappa,
                                p.physics.rho_l, p.physics.rho_v, precision=precision) for p in probs]
        need = sum(lbm.Batch.slot_bytes(q) for q in prms)
        arena = need + lbm.Batch.overhead_bytes(2 * need, len(probs)) + (1 << 22)
        b = lbm.Batch(arena, max_slots=len(probs))
        b.set_graph_steps(2)
        slots = [b.admit(q, p.rho(), "well_balanced") for q, p in zip(prms, probs)]
        res = []
        for bw in blocks:
            for r in rows:
                for d in depths:
                    for s in slots:
                        b.set_tile(s, bw, r, d)
                    b.run(4)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    e0.record()
                    b.run(steps)
                    e1.record()
                    torch.cuda.synchronize()
                    res.append((e0.elapsed_time(e1) / steps, bw, r, d))
        b.close()
        res.sort()
        best[bk] = res[0]
    return best


def tune_batch_full(problems, precision, blocks=(64, 128, 256), rows=(8, 16, 32, 64, 128),
                    depths=(1, 2, 3), two_step_rows=(32, 64, 128, 256), steps=20, passes=2):
    """Tile per size bucket on the whole batch; the candidates are the one-step
    tiles (blocks x rows x depths) and the two-step tiles (depth 4, block
    128 or 256, chunks of `two_step_rows`).  First every lattice gets the
    same candidate tile (one launch group) and the fastest is kept; then
    coordinate descent over the buckets: for each bucket in turn, time the
    full batch under every candidate for that bucket's lattices (the others
    fixed) and keep the fastest.  Starting from one shared tile matters: a
    bucket moved alone to another block width or depth forms a second group,
    launched after the first, so single-bucket moves are compared against a
    one-group start.  The shared tile is kept unless the per-bucket tiles
    beat it by more than 1%.  Returns {bucket: (block, rows, depth)}, the
    final ms per step and the uniform sweep [(ms, tile), ...]."""
    import torch
    from . import lbm
    prms = [lbm.make_params(p.nx, p.ny, p.physics.tau, p.physics.beta, p.physics.kappa,
                            p.physics.rho_l, p.physics.rho_v, precision=precision) for p in problems]
    need = sum(lbm.Batch.slot_bytes(q) for q in prms)
    b = lbm.Batch(need + lbm.Batch.overhead_bytes(2 * need, len(problems)) + (1 << 24),
                  max_slots=len(problems))
    b.set_graph_steps(10)
    slots = [b.admit(q, p.rho(), "well_balanced") for q, p in zip(prms, problems)]
    by = {}
    for s, p in zip(slots, problems):
        by.setdefault(_bucket(p.nx, p.ny), []).append(s)
    choice = {bk: (64, 32, 1) for bk in by}

    def timed():
        b.run(10)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        b.run(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    cands = [(bw, r, d) for bw in blocks for r in rows for d in depths]
    cands += [(bw, r, 4) for bw in (128, 256) for r in two_step_rows]
    uniform = []
    for cand in cands:
        for s in slots:
            b.set_tile(s, *cand)
        uniform.append((timed(), cand))
    uniform.sort()
    choice = {bk: uniform[0][1] for bk in by}
    for bk, ss in by.items():
        for s in ss:
            b.set_tile(s, *choice[bk])
    best_ms = timed()
    for _ in range(passes):
        for bk, ss in sorted(by.items()):
            for cand in cands:
                for s in ss:
                    b.set_tile(s, *cand)
                ms = timed()
                if ms < best_ms:
                    best_ms, choice[bk] = ms, cand
            for s in ss:
                b.set_tile(s, *choice[bk])
    b.close()
    # Per-bucket tiles that differ in block width or depth are separate launch
    # groups, each adding an end-of-launch tail when the batch is lightly
    # loaded: keep them only if they beat the best shared tile by over 1%.
    if best_ms > 0.99 * uniform[0][0]:
        choice = {bk: uniform[0][1] for bk in by}
        best_ms = uniform[0][0]
    return choice, best_ms, uniform


def main():
    import argparse
    ap = argparse.ArgumentParser(description="tile autotuning on the current device")
    ap.add_argument("--batch", action="store_true", help="tune batch tiles per size bucket")
    ap.add_argument("--single", action="store_true", help="tune the 4096^2 lattice tile")
    ap.add_argument("--two-step", action="store_true",
                    help="tune the 4096^2 tile of two steps per launch (the benchmark's)")
    ap.add_argument("--write", action="store_true", help="store the result in tuned_tiles.json")
    ap.add_argument("--out", default=None, help="write the table here instead of tuned_tiles.json")
    args = ap.parse_args()
    from . import inputs as I
    table = _table()
    if args.batch:
        probs = I.batch_instances(512)
        for prec in ("fp64", "fp32s"):
            choice, ms, uniform = tune_batch_full(probs, prec)
            for ums, cand in uniform:
                print("batch uniform", prec, cand, "%.4f ms/step" % ums, flush=True)
            for bk, (bw, r, d) in sorted(choice.items()):
                print("batch", bk, prec, bw, r, d, flush=True)
                table["batch/%s/%s" % (bk, prec)] = [bw, r, d]
            print("batch", prec, "%.4f ms/step for the 512-lattice batch" % ms, flush=True)
    if args.single:
        from . import lbm
        prob = I.DROPLET_4096
        for prec in ("fp64", "fp32s"):
            s = lbm.Solver.for_problem(prob, precision=prec)
            s.init(prob.rho(), scheme="well_balanced")
            res = sweep(s, blocks=(128, 256, 512), rows=(32, 64, 96, 128, 160, 192, 256),
                        depths=(1, 2, 3), steps=30)
            s.close()
            for ms, bw, r, d in res[:5]:
                print("single 4096", prec, bw, r, d, "%.4f ms/step" % ms, flush=True)
            table["4096/%s" % prec] = list(res[0][1:])
    if args.two_step:
        import torch
        from . import lbm
        prob = I.DROPLET_4096
        for prec in ("fp64", "fp32s"):
            block, base, _ = two_step_tile(prob.nx, prob.ny, prec)
            strips = -(-prob.nx // (block - 6))
            # resident blocks: two per CU
            per_round = max(1, 512 // strips)
            # chunk counts filling one round (and one less), two rounds, and
            # the one-step tile for comparison
            cands = sorted({-(-prob.ny // c) for c in (per_round, per_round - 1, 2 * per_round)})
            s = lbm.Solver.for_problem(prob, precision=prec)
            s.init(prob.rho(), scheme="well_balanced")
            res = []
            for tile in [(block, r, 4) for r in cands] + [(512, 128, 3)]:
                s.set_tile(*tile)
                s.step(50, "well_balanced")
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                s.step(200, "well_balanced")
                e1.record()
                torch.cuda.synchronize()
                res.append((e0.elapsed_time(e1) / 200, tile))
            s.close()
            res.sort()
            for ms, tile in res:
                print("two-step 4096", prec, tile, "%.4f ms/step" % ms, flush=True)
            table["4096/%s" % prec] = list(res[0][1])
    if args.write or args.out:
        with open(args.out or TABLE, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()
