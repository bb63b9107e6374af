"""FP64 CPU oracle of the two-phase LBE step -- TEST INFRASTRUCTURE.

This module wraps ``lbm_oracle.c`` (D2Q9) and ``lbm_oracle3d.c`` (the same
equations in 3-D, compiled for D3Q19 and, through ``lbm_oracle3d27.c``, for
D3Q27) -- plain C, double precision, scalar loops, array-of-structures
populations -- through ctypes, and adds the diagnostics the paper reads off a
steady state (bulk densities, Laplace pressure jump).
Only the test-suite, the smoke entry point and the CPU-baseline leg of the
benchmark use it; the product path never imports it.

Paper: Z. Guo, "Well-balanced lattice Boltzmann equation for two-phase
flows", arXiv:2012.11075.  Sec. II (standard LBE, Eqs. 2-6), Sec. III (WB
LBE, Eqs. 24-26), Sec. IV (double-well free energy, Eqs. 35-37).

Array conventions (numpy, float64, C-contiguous):
  f    : shape (ny, nx, 9), population i of node (x, y) at f[y, x, i]
  field: shape (ny, nx)
  3-D  : f (nz, ny, nx, q), fields (nz, ny, nx)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
SRC3 = os.path.join(HERE, "lbm_oracle3d.c")
SRC27 = os.path.join(HERE, "lbm_oracle3d27.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "liboracle.so")

STANDARD = 0
WELL_BALANCED = 1
STANDARD_EQF = 2  # standard LBE with F_i = (c_i - u).F feq_i / (cs2 rho)
SCHEMES = {"standard": STANDARD, "well_balanced": WELL_BALANCED, "wb": WELL_BALANCED,
           "standard_eq_forcing": STANDARD_EQF}

# D2Q9 in the paper's numbering (Sec. II): used by diagnostics that regroup
# populations, never by the step itself (which lives in C).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fused multiply-add, OpenMP rows)."""
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(x) for x in (SRC, SRC3, SRC27)):
        return LIB
    os.makedirs(BUILD_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, SRC, SRC3, SRC27, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("beta", ctypes.c_double),
                ("kappa", ctypes.c_double), ("rho_l", ctypes.c_double),
                ("rho_v", ctypes.c_double), ("rho0", ctypes.c_double),
                ("force_stencil", ctypes.c_int)]


@dataclass(frozen=True)
class Params:
    """Physical parameters in lattice units (Eq. 2 tau; Eq. 36 beta, rho_l,
    rho_v; kappa of mu = mu0 - kappa lap rho; rho0 of Eq. 24; force_stencil:
    0 the central gradients of Sec. II in the force, 1 the fourth-order ones
    of ``gradient4``)."""
    tau: float
    beta: float
    kappa: float
    rho_l: float
    rho_v: float
    rho0: float = 0.0
    force_stencil: int = 0

    def c(self) -> _Params:
        return _Params(self.tau, self.beta, self.kappa, self.rho_l, self.rho_v, self.rho0,
                       int(self.force_stencil))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER(_Params)
        i, d, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        sig = {
            "orc_mu0": (d, [P, d]),
            "orc_psi0": (d, [P, d]),
            "orc_p0": (d, [P, d]),
            "orc_feq": (None, [i, P, d, d, d, _D]),
            "orc_forcing": (None, [i, d, d, d, d, d, d, _D]),
            "orc_forcing_eq": (None, [_D, d, d, d, d, d, _D]),
            "orc_gradient": (None, [i, i, _D, _D, _D]),
            "orc_gradient4": (None, [i, i, _D, _D, _D]),
            "orc_laplacian": (None, [i, i, _D, _D]),
            "orc_macro": (None, [i, P, i, i, _D] + [_D] * 8),
            "orc_fields": (None, [i, P, i, i, _D, _D, _D, _D, _D]),
            "orc_init": (None, [i, P, i, i, _D, _D, _D, _D]),
            "orc_step": (None, [i, P, i, i, _D, i64]),
            "orc_observe": (None, [i, P, i, i, _D, _D]),
            "orc3_feq": (None, [i, P, d, d, d, d, _D]),
            "orc3_forcing": (None, [i] + [d] * 9 + [_D]),
            "orc3_forcing_eq": (None, [_D] + [d] * 7 + [_D]),
            "orc3_gradient": (None, [i, i, i, _D, _D, _D, _D]),
            "orc3_laplacian": (None, [i, i, i, _D, _D]),
            "orc3_macro": (None, [i, P, i, i, i, _D] + [_D] * 11),
            "orc3_init": (None, [i, P, i, i, i, _D, _D, _D, _D, _D]),
            "orc3_step": (None, [i, P, i, i, i, _D, i64]),
            "orc3_observe": (None, [i, P, i, i, i, _D, _D]),
            "orc27_feq": (None, [i, P, d, d, d, d, _D]),
            "orc27_forcing": (None, [i] + [d] * 9 + [_D]),
            "orc27_forcing_eq": (None, [_D] + [d] * 7 + [_D]),
            "orc27_gradient": (None, [i, i, i, _D, _D, _D, _D]),
            "orc27_laplacian": (None, [i, i, i, _D, _D]),
            "orc27_macro": (None, [i, P, i, i, i, _D] + [_D] * 11),
            "orc27_init": (None, [i, P, i, i, i, _D, _D, _D, _D, _D]),
            "orc27_step": (None, [i, P, i, i, i, _D, i64]),
            "orc27_observe": (None, [i, P, i, i, i, _D, _D]),
            "orc_set_threads": (None, [i]),
            "orc_get_threads": (i, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _scheme(s) -> int:
    return SCHEMES[s] if isinstance(s, str) else int(s)


def _scheme3(s) -> int:
    k = _scheme(s)
    if k not in (STANDARD, WELL_BALANCED, STANDARD_EQF):
        raise ValueError("unknown scheme %r" % (s,))
    return k


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


# ------------------------------------------------------------------ node level
def mu0(p: Params, rho: float) -> float:
    """Bulk chemical potential d psi0/d rho (Eq. 37)."""
    return _load().orc_mu0(ctypes.byref(p.c()), float(rho))


def psi0(p: Params, rho: float) -> float:
    """Double-well bulk free energy (Eq. 36)."""
    return _load().orc_psi0(ctypes.byref(p.c()), float(rho))


def p0(p: Params, rho: float) -> float:
    """Thermodynamic pressure rho mu0 - psi0 (Eq. 37)."""
    return _load().orc_p0(ctypes.byref(p.c()), float(rho))


def feq(scheme, p: Params, rho: float, ux: float, uy: float) -> np.ndarray:
    """Equilibrium populations: Eq. (3) standard, Eq. (24) well-balanced."""
    out = np.zeros(9)
    _load().orc_feq(_scheme(scheme), ctypes.byref(p.c()), rho, ux, uy, _ptr(out))
    return out


def forcing(scheme, ux, uy, Fx, Fy, grx=0.0, gry=0.0) -> np.ndarray:
    """Forcing term: Eq. (5) standard, Eq. (26) well-balanced (the
    equilibrium-proportional form is ``forcing_eq``)."""
    k = _scheme(scheme)
    if k not in (STANDARD, WELL_BALANCED):
        raise ValueError("forcing(): use forcing_eq for the standard_eq_forcing scheme")
    out = np.zeros(9)
    _load().orc_forcing(k, ux, uy, Fx, Fy, grx, gry, _ptr(out))
    return out


def forcing_eq(p: Params, rho, ux, uy, Fx, Fy) -> np.ndarray:
    """The other forcing term of the standard LBE named after Eq. (5):
    F_i = (c_i - u).F feq_i / (cs2 rho), feq of Eq. (3)."""
    fe = feq(STANDARD, p, rho, ux, uy)
    out = np.zeros(9)
    _load().orc_forcing_eq(_ptr(fe), rho, ux, uy, Fx, Fy, _ptr(out))
    return out


# ----------------------------------------------------------------- field level
def gradient(phi: np.ndarray):
    """Isotropic central gradient (1/cs2) sum_i w_i c_i phi(x+c_i), periodic."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    gx, gy = np.empty_like(phi), np.empty_like(phi)
    _load().orc_gradient(nx, ny, _ptr(phi), _ptr(gx), _ptr(gy))
    return gx, gy


def gradient4(phi: np.ndarray):
    """Fourth-order gradient: the central gradient of phi minus 1/6 of the
    central gradient of its isotropic Laplacian, periodic (the force-stencil
    variant; 1-D: (-phi_{j+2} + 8 phi_{j+1} - 8 phi_{j-1} + phi_{j-2})/12)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    gx, gy = np.empty_like(phi), np.empty_like(phi)
    _load().orc_gradient4(nx, ny, _ptr(phi), _ptr(gx), _ptr(gy))
    return gx, gy


def laplacian(phi: np.ndarray) -> np.ndarray:
    """Isotropic 9-point Laplacian (2/cs2) sum_i w_i [phi(x+c_i) - phi(x)]."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    out = np.empty_like(phi)
    _load().orc_laplacian(nx, ny, _ptr(phi), _ptr(out))
    return out


def macro(scheme, p: Params, f: np.ndarray) -> dict:
    """rho, u, mu, F and grad rho of the state f (Eq. 4, 6, 25)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    ny, nx, _ = f.shape
    names = ["rho", "ux", "uy", "mu", "Fx", "Fy", "grx", "gry"]
    out = {k: np.empty((ny, nx)) for k in names}
    _load().orc_macro(_scheme(scheme), ctypes.byref(p.c()), nx, ny, _ptr(f),
                      *[_ptr(out[k]) for k in names])
    return out


def fields(scheme, p: Params, f: np.ndarray):
    """(rho, ux, uy, mu) of the state f."""
    m = macro(scheme, p, f)
    return m["rho"], m["ux"], m["uy"], m["mu"]


def init(scheme, p: Params, rho: np.ndarray, ux=None, uy=None) -> np.ndarray:
    """f(0) = feq(rho, u) of the scheme (u = 0 when not given)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64)
    uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64)
    f = np.empty((ny, nx, 9))
    _load().orc_init(_scheme(scheme), ctypes.byref(p.c()), nx, ny, _ptr(rho),
                     _ptr(ux), _ptr(uy), _ptr(f))
    return f


def step(scheme, p: Params, f: np.ndarray, n: int = 1) -> np.ndarray:
    """Return the state after n steps of Eq. (2) (collide, then stream)."""
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    ny, nx, _ = g.shape
    _load().orc_step(_scheme(scheme), ctypes.byref(p.c()), nx, ny, _ptr(g), int(n))
    return g


def observe(scheme, p: Params, f: np.ndarray) -> dict:
    """max|u|, total mass, kinetic energy E (Sec. IV.A), a non-finite flag
    and the total momentum sum rho u (u the half-force velocity of Eq. 4)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    ny, nx, _ = f.shape
    out = np.zeros(6)
    _load().orc_observe(_scheme(scheme), ctypes.byref(p.c()), nx, ny, _ptr(f), _ptr(out))
    return {"max_u": out[0], "mass": out[1], "kinetic_energy": out[2], "nonfinite": bool(out[3]),
            "momentum": (out[4], out[5])}


# --------------------------------------------------------- steady-state reads
def surface_tension(p: Params) -> float:
    """sigma = (rho_l - rho_v)^3 sqrt(2 beta kappa) / 6 for the double well
    (Sec. IV.B, the Laplace-law passage)."""
    return (p.rho_l - p.rho_v) ** 3 * np.sqrt(2.0 * p.beta * p.kappa) / 6.0


def equilibrium_width(p: Params) -> float:
    """Width D of the tanh profile of Eq. (38), read as
    sqrt(8 kappa / beta) / (rho_l - rho_v): the first integral of
    kappa rho'' = mu0(rho) gives rho' = sqrt(2 beta/kappa)(rho_l-rho)(rho-rho_v)."""
    return np.sqrt(8.0 * p.kappa / p.beta) / (p.rho_l - p.rho_v)


def torus_distance(nx: int, ny: int, cx: float, cy: float) -> np.ndarray:
    x = np.arange(nx)[None, :] - cx
    y = np.arange(ny)[:, None] - cy
    x = np.minimum(np.abs(x), nx - np.abs(x))
    y = np.minimum(np.abs(y), ny - np.abs(y))
    return np.sqrt(x * x + y * y)


def droplet_diagnostics(p: Params, rho: np.ndarray, cx: float, cy: float) -> dict:
    """Bulk densities at the droplet centre and at the node farthest from it on
    the torus, the pressure jump p0(rho_in) - p0(rho_out) (Eq. 37), and the
    equivalent radius sqrt(A/pi), A = sum (rho - rho_out)/(rho_in - rho_out)."""
    ny, nx = rho.shape
    ic, jc = int(round(cy)) % ny, int(round(cx)) % nx
    jo, io = (jc + nx // 2) % nx, (ic + ny // 2) % ny
    rho_in = float(rho[ic, jc])
    rho_out = float(rho[io, jo])
    area = float(np.sum(rho - rho_out) / (rho_in - rho_out))
    return {
        "rho_in": rho_in,
        "rho_out": rho_out,
        "dp": p0(p, rho_in) - p0(p, rho_out),
        "r_eff": float(np.sqrt(max(area, 0.0) / np.pi)),
    }


# ------------------------------------------- three dimensions (D3Q19, D3Q27)
# Populations: shape (nz, ny, nx, q); fields: (nz, ny, nx).  q = 19: rest,
# the six axis directions, the twelve edge directions (order of C3); q = 27
# adds the eight corner directions (order of C27).  Every 3-D function takes
# q=19 (default) or q=27.
C3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
C27 = np.concatenate([C3, np.array([[1, 1, 1], [-1, -1, -1], [1, 1, -1], [-1, -1, 1],
                                    [1, -1, 1], [-1, 1, -1], [-1, 1, 1], [1, -1, -1]])])


def _fn3(name, q):
    if q not in (19, 27):
        raise ValueError("q must be 19 or 27")
    return getattr(_load(), ("orc3_" if q == 19 else "orc27_") + name)


def feq3(scheme, p: Params, rho, ux, uy, uz, q=19) -> np.ndarray:
    """3-D equilibrium: Eq. (3) standard, Eq. (24) well-balanced."""
    out = np.zeros(q)
    _fn3("feq", q)(_scheme3(scheme), ctypes.byref(p.c()), rho, ux, uy, uz, _ptr(out))
    return out


def forcing3(scheme, u, F, gr=(0.0, 0.0, 0.0), q=19) -> np.ndarray:
    """3-D forcing term: Eq. (5) standard, Eq. (26) with D = 3 (the
    equilibrium-proportional form is ``forcing_eq3``)."""
    k = _scheme3(scheme)
    if k == STANDARD_EQF:
        raise ValueError("forcing3(): use forcing_eq3 for the standard_eq_forcing scheme")
    out = np.zeros(q)
    _fn3("forcing", q)(k, *map(float, u), *map(float, F), *map(float, gr), _ptr(out))
    return out


def forcing_eq3(p: Params, rho, u, F, q=19) -> np.ndarray:
    """3-D form of the forcing term named after Eq. (5):
    F_i = (c_i - u).F feq_i / (cs2 rho), feq of Eq. (3)."""
    fe = feq3(STANDARD, p, rho, *map(float, u), q=q)
    out = np.zeros(q)
    _fn3("forcing_eq", q)(_ptr(fe), float(rho), *map(float, u), *map(float, F), _ptr(out))
    return out


def gradient3(phi: np.ndarray, q=19):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    g = [np.empty_like(phi) for _ in range(3)]
    _fn3("gradient", q)(nx, ny, nz, _ptr(phi), *[_ptr(a) for a in g])
    return tuple(g)


def laplacian3(phi: np.ndarray, q=19) -> np.ndarray:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    out = np.empty_like(phi)
    _fn3("laplacian", q)(nx, ny, nz, _ptr(phi), _ptr(out))
    return out


def macro3(scheme, p: Params, f: np.ndarray) -> dict:
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx, q = f.shape
    names = ["rho", "ux", "uy", "uz", "mu", "Fx", "Fy", "Fz", "grx", "gry", "grz"]
    out = {k: np.empty((nz, ny, nx)) for k in names}
    _fn3("macro", q)(_scheme3(scheme), ctypes.byref(p.c()), nx, ny, nz, _ptr(f),
                     *[_ptr(out[k]) for k in names])
    return out


def init3(scheme, p: Params, rho: np.ndarray, u=None, q=19) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nz, ny, nx = rho.shape
    comps = [None, None, None] if u is None else [np.ascontiguousarray(a, dtype=np.float64) for a in u]
    f = np.empty((nz, ny, nx, q))
    _fn3("init", q)(_scheme3(scheme), ctypes.byref(p.c()), nx, ny, nz, _ptr(rho),
                    *[_ptr(a) for a in comps], _ptr(f))
    return f


def step3(scheme, p: Params, f: np.ndarray, n: int = 1) -> np.ndarray:
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    nz, ny, nx, q = g.shape
    _fn3("step", q)(_scheme3(scheme), ctypes.byref(p.c()), nx, ny, nz, _ptr(g), int(n))
    return g


def observe3(scheme, p: Params, f: np.ndarray) -> dict:
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx, q = f.shape
    out = np.zeros(7)
    _fn3("observe", q)(_scheme3(scheme), ctypes.byref(p.c()), nx, ny, nz, _ptr(f), _ptr(out))
    return {"max_u": out[0], "mass": out[1], "kinetic_energy": out[2], "nonfinite": bool(out[3]),
            "momentum": (out[4], out[5], out[6])}
