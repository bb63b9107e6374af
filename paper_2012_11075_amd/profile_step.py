"""Workload driver for rocprofv3: a few step launches on the 4096^2
throughput lattice, followed by a plain elementwise kernel of known traffic
(reads and writes `--copy-mib` MiB each) that calibrates the HBM counters.

    rocprofv3 --kernel-trace --stats -d OUT -o run --output-format csv -- \
        python -m paper_2012_11075_amd.profile_step --precision fp64 --steps 20
    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch --output-format csv -- \
        python -m paper_2012_11075_amd.profile_step --precision fp64 --steps 20

Prints one line per phase so a long run shows progress.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32s"])
    ap.add_argument("--scheme", default="well_balanced")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--problem", default="droplet_4096")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--force-stencil", type=int, default=0,
                    help="1: the fourth-order force-stencil variant (one fused kernel per step)")
    ap.add_argument("--d3", type=int, default=0,
                    help="profile the 3-D step on an N^3 droplet instead")
    ap.add_argument("--q3", type=int, default=19, choices=[19, 27],
                    help="velocity set of the 3-D step: 19 (D3Q19) or 27 (D3Q27)")
    ap.add_argument("--batch", type=int, default=0,
                    help="profile the batched launch over this many uneven instances instead")
    ap.add_argument("--side", type=int, default=0,
                    help="profile an N x N lattice with a separable density and the Sec. IV "
                         "constants instead (the 4096^2 tile), e.g. 32768")
    args = ap.parse_args()
    import torch
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import lbm, tune
    if args.batch:
        run_batch(args, torch, I, lbm, tune)
        calibrate(args, torch)
        return
    if args.d3:
        n, ph = args.d3, I.PHYS3
        rho = I.droplet3_density(n, n, n, ph, I.DROPLET3_RADIUS * n / I.DROPLET3_SIDE,
                                 I.equilibrium_width(ph), 1e-3, seed=13)
        s = lbm.Solver(n, n, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, nz=n,
                       precision=args.precision, q3=args.q3)
        s.init(rho, scheme=args.scheme)
        print("profile_step: D3Q%d %d^3 %s %s tile=%s" % (args.q3, n, args.precision, args.scheme,
                                                          s.get_tile()), flush=True)
        s.step(args.steps, args.scheme)
        torch.cuda.synchronize()
        print("profile_step: %d steps done" % args.steps, flush=True)
        calibrate(args, torch)
        s.close()
        return
    if args.side:
        n, ph = args.side, I.PAPER_PHYS
        s = lbm.Solver(n, n, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                       precision=args.precision)
        # the benchmark's tile for this size (bench.py, largest lattice)
        s.set_tile(*(tune.two_step_tile(n, n, args.precision)
                     or tune.bench_tile(4096, 4096, args.precision)))
        s.init(I.separable_density(n, n, 17), scheme=args.scheme)
        print("profile_step: %d^2 separable density %s %s tile=%s" % (n, args.precision, args.scheme,
                                                                      s.get_tile()), flush=True)
        s.step(args.steps, args.scheme)
        torch.cuda.synchronize()
        print("profile_step: %d steps done" % args.steps, flush=True)
        calibrate(args, torch)
        s.close()
        return
    prob = I.PROBLEMS[args.problem]
    s = lbm.Solver.for_problem(prob, precision=args.precision, force_stencil=args.force_stencil)
    tile = (args.block, args.rows, args.depth) if (args.block or args.rows or args.depth) else \
        (tune.stencil4_tile if args.force_stencil else tune.bench_tile)(prob.nx, prob.ny,
                                                                         args.precision)
    s.set_tile(*tile)
    s.init(prob.rho(), scheme=args.scheme)
    print("profile_step: %s %s %s tile=%s" % (prob.name, args.precision, args.scheme,
                                               s.get_tile()), flush=True)
    s.step(args.steps, args.scheme)
    torch.cuda.synchronize()
    print("profile_step: %d steps done" % args.steps, flush=True)
    calibrate(args, torch)
    s.close()


def run_batch(args, torch, I, lbm, tune):
    """The batched workload: `args.batch` uneven instances (side 32..512)
    in one arena, tuned tiles, `args.steps` steps without graphs (one
    launch per group and step)."""
    probs = I.batch_instances(args.batch)
    prms = [lbm.make_params(p.nx, p.ny, p.physics.tau, p.physics.beta, p.physics.kappa,
                            p.physics.rho_l, p.physics.rho_v, precision=args.precision) for p in probs]
    need = sum(lbm.Batch.slot_bytes(q) for q in prms)
    b = lbm.Batch(need + lbm.Batch.overhead_bytes(2 * need, len(probs)) + (1 << 24),
                  max_slots=len(probs))
    for q, p in zip(prms, probs):
        sl = b.admit(q, p.rho(), args.scheme)
        t = tune.batch_tile(p.nx, p.ny, args.precision)
        if t:
            b.set_tile(sl, *t)
    nodes = sum(p.nx * p.ny for p in probs)
    print("profile_step: batch of %d instances, %d nodes, %s" % (len(probs), nodes, args.precision),
          flush=True)
    b.run(args.steps)
    torch.cuda.synchronize()
    print("profile_step: %d batched steps done" % args.steps, flush=True)
    b.close()


def calibrate(args, torch):
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print("profile_step: calibration kernel: 3 x (read %d MiB + write %d MiB)"
          % (args.copy_mib, args.copy_mib), flush=True)


if __name__ == "__main__":
    main()
