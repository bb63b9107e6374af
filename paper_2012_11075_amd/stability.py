"""Stability map of the two schemes over tau, density ratio and interface
width, run as one batch on the GPU.

The paper remarks (Sec. III, after Eq. 24) that the constant rho0 of the WB
equilibrium may affect stability, and its runs use one tau, one density
ratio and one interface width.  This module scans those three, the scheme,
and rho0 for the WB scheme: each cell is a droplet at rest (radius a
quarter of the side, the tanh profile of Eq. 38 at the equilibrium width,
multiplicative noise 1e-3) on a periodic lattice.  Every cell is one slot of
an ``lbm.Batch``; a cell is "diverged" at the first poll that finds a
non-finite value or rho <= 0, else it runs to the step cap and reports its
final max|u|.

The free-energy constants follow from the width: beta = 0.01 and
kappa = beta (W (rho_l - rho_v))^2 / 8, the inverse of
W = sqrt(8 kappa / beta) / (rho_l - rho_v) (Eq. 38 with the reading of the
interface width).

    python -m paper_2012_11075_amd.stability --side 128 --steps 20000 \
        --poll 500 --json out.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import time
from dataclasses import dataclass

from . import inputs as I

BETA = 0.01
TAUS = (0.55, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9, 1.0, 1.2)
RATIOS = (2, 5, 10, 100, 1000)
WIDTHS = (1.3, 2.0, 3.2, 5.0)


@dataclass(frozen=True)
class Cell:
    scheme: str
    tau: float
    ratio: float
    width: float
    rho0: float

    def physics(self) -> I.Physics:
        rho_v = 1.0 / self.ratio
        kappa = BETA * (self.width * (1.0 - rho_v)) ** 2 / 8.0
        return I.Physics(tau=self.tau, beta=BETA, kappa=kappa, rho_l=1.0, rho_v=rho_v,
                         rho0=self.rho0)

    def problem(self, side: int, seed: int) -> I.Problem:
        name = "stab_%s_t%g_r%g_w%g_z%g" % (self.scheme, self.tau, self.ratio, self.width,
                                            self.rho0)
        return I.Problem(name, side, side, self.physics(), "droplet", self.width, side / 4.0,
                         0.0, 1e-3, "mul", seed)


def cells(taus=TAUS, ratios=RATIOS, widths=WIDTHS, wb_rho0s=(0.0, 1.0)) -> list:
    out = []
    for tau, ratio, width in itertools.product(taus, ratios, widths):
        out.append(Cell("standard", tau, ratio, width, 0.0))
        for r0 in wb_rho0s:
            out.append(Cell("well_balanced", tau, ratio, width, r0))
    return out


def run_map(cell_list, side=128, steps=20_000, poll=500, seed=21, precision="fp64"):
    """Run every cell as one slot of a batch; returns one dict per cell with
    its outcome ("diverged" / "capped"), the step it retired at and the
    max|u| observed then."""
    from . import lbm
    probs = [c.problem(side, seed) for c in cell_list]
    prms = [lbm.make_params(p.nx, p.ny, p.physics.tau, p.physics.beta, p.physics.kappa,
                            p.physics.rho_l, p.physics.rho_v, p.physics.rho0,
                            precision=precision) for p in probs]
    need = sum(lbm.Batch.slot_bytes(q) for q in prms)
    arena = need + lbm.Batch.overhead_bytes(2 * need, len(prms)) + (1 << 20)
    b = lbm.Batch(arena, max_slots=len(prms))
    slot_of = {}
    for k, (c, p, q) in enumerate(zip(cell_list, probs, prms)):
        slot_of[b.admit(q, p.rho(), c.scheme, tol=0.0, step_cap=steps)] = k
    res = [None] * len(cell_list)
    done = 0
    while done < len(cell_list):
        b.run(poll)
        for s in b.poll():
            status, ob = b.info(s)
            k = slot_of[s]
            res[k] = dict(vars(cell_list[k]), outcome=status, step=ob["step"], max_u=ob["max_u"])
            b.release(s)
            done += 1
    b.close()
    return res


def table(results, scheme, rho0=0.0) -> str:
    """Markdown table for one scheme: rows tau, columns (ratio, width); a
    cell shows the divergence step ("d 1500") or the final max|u|."""
    rs = [r for r in results if r["scheme"] == scheme and r["rho0"] == rho0]
    cols = sorted({(r["ratio"], r["width"]) for r in rs})
    taus = sorted({r["tau"] for r in rs})
    by = {(r["tau"], r["ratio"], r["width"]): r for r in rs}
    head = "| tau | " + " | ".join("%g, W %g" % c for c in cols) + " |"
    lines = [head, "|---" * (len(cols) + 1) + "|"]
    for t in taus:
        row = []
        for c in cols:
            r = by[(t, c[0], c[1])]
            row.append("d %d" % r["step"] if r["outcome"] == "diverged" else "%.1e" % r["max_u"])
        lines.append("| %g | " % t + " | ".join(row) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--steps", type=int, default=20_000)
    ap.add_argument("--poll", type=int, default=500)
    ap.add_argument("--json", default="")
    args = ap.parse_args()
    cl = cells()
    t = time.time()
    res = run_map(cl, args.side, args.steps, args.poll)
    print("stability map: %d cells, %d^2, %d steps, %.1f s"
          % (len(cl), args.side, args.steps, time.time() - t), flush=True)
    for scheme, r0 in (("well_balanced", 0.0), ("well_balanced", 1.0), ("standard", 0.0)):
        print("\n%s, rho0 = %g (columns: density ratio, equilibrium width)\n" % (scheme, r0))
        print(table(res, scheme, r0))
    same = all(a["outcome"] == b["outcome"]
               for a in res if a["scheme"] == "well_balanced" and a["rho0"] == 0.0
               for b in res if b["scheme"] == "well_balanced" and b["rho0"] == 1.0
               and (a["tau"], a["ratio"], a["width"]) == (b["tau"], b["ratio"], b["width"]))
    print("\nWB outcome independent of rho0: %s" % same)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=0)


if __name__ == "__main__":
    main()
