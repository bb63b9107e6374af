"""Discrete 1-D equilibrium of the flat interface, by Newton's method (test
helper, independent of both the oracle and the GPU path)."""
import numpy as np


def flat_equilibrium(beta, kappa, rho_l, rho_v, n, mass, guess):
    """Solve mu0(rho_j) - kappa (rho_{j+1} - 2 rho_j + rho_{j-1}) = mu_b with
    sum rho = mass on a periodic 1-D lattice of n nodes; the profile is kept
    symmetric about the lattice centre (removes the nearly free translation)."""
    def mu0(r):
        return 2 * beta * (r - rho_l) * (r - rho_v) * (2 * r - rho_l - rho_v)

    def dmu0(r):
        a, b = r - rho_l, r - rho_v
        return 2 * beta * (b * (2 * r - rho_l - rho_v) + a * (2 * r - rho_l - rho_v) + 2 * a * b)

    z = np.concatenate([np.asarray(guess, dtype=float), [0.0]])
    L = -2 * np.eye(n) + np.roll(np.eye(n), 1, 1) + np.roll(np.eye(n), -1, 1)
    for _ in range(60):
        r, mb = z[:n], z[n]
        res = np.concatenate([mu0(r) - kappa * (L @ r) - mb, [r.sum() - mass]])
        J = np.zeros((n + 1, n + 1))
        J[:n, :n] = np.diag(dmu0(r)) - kappa * L
        J[:n, n] = -1.0
        J[n, :n] = 1.0
        dz = np.linalg.solve(J, -res)
        z = z + dz
        z[:n] = 0.5 * (z[:n] + z[:n][::-1])
        if np.abs(dz).max() < 1e-15:
            break
    return z[:n], z[n]
