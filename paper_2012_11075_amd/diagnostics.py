"""Steady-state reads of a droplet or slab (host-side analysis of fields the
GPU path returns).

Sec. IV.B of Guo (arXiv:2012.11075) reads the bulk liquid and vapour
densities of a droplet at rest and explains their shift from saturation by
the Laplace pressure; with the double well of Eq. (36) the thermodynamic
pressure is p0 = rho mu0 - psi0 (Eq. 37).
"""
from __future__ import annotations

import numpy as np


def pressure(rho, beta, rho_l, rho_v):
    """p0 = rho dpsi0/drho - psi0 for psi0 = beta (rho - rho_l)^2 (rho - rho_v)^2."""
    a, b = rho - rho_l, rho - rho_v
    mu0 = 2.0 * beta * a * b * (2.0 * rho - rho_l - rho_v)
    return rho * mu0 - beta * a * a * b * b


def droplet_reads(rho: np.ndarray, beta: float, rho_l: float, rho_v: float) -> dict:
    """Bulk density at the droplet centre (node (nx//2, ny//2)) and at the node
    farthest from it on the torus, and the pressure jump between them."""
    ny, nx = rho.shape
    cy, cx = ny // 2, nx // 2
    r_in = float(rho[cy, cx])
    r_out = float(rho[(cy + ny // 2) % ny, (cx + nx // 2) % nx])
    return {"rho_in": r_in, "rho_out": r_out,
            "laplace_dp": float(pressure(r_in, beta, rho_l, rho_v) - pressure(r_out, beta, rho_l, rho_v))}


def compare(a: dict, b: dict) -> dict:
    """Absolute and relative differences of matching scalar reads (b relative to a)."""
    out = {}
    for k, va in a.items():
        vb = b[k]
        out[k] = {"ref": va, "value": vb, "abs_err": abs(vb - va),
                  "rel_err": abs(vb - va) / abs(va) if va else None}
    return out
