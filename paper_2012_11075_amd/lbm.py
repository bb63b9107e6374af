"""Python binding of liblbm.so (argument marshalling only).

Every step of the computation runs in the HIP kernels behind the C ABI of
include/lbm.h.  PyTorch provides the device workspace and the HIP stream.
If the library has not been built, loading fails with an error: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "liblbm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "lbm.h")

STANDARD, WELL_BALANCED, STANDARD_EQ_FORCING = 0, 1, 2
FP64, FP32_SHIFTED = 0, 1
SCHEMES = {"standard": STANDARD, "well_balanced": WELL_BALANCED, "wb": WELL_BALANCED,
           "standard_eq_forcing": STANDARD_EQ_FORCING}
PRECISIONS = {"fp64": FP64, "fp32s": FP32_SHIFTED, "fp32_shifted": FP32_SHIFTED}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOSPACE", -3: "LBM_EHIP",
          -4: "LBM_ENONFINITE", -5: "LBM_ESTATE", -6: "LBM_EBUSY"}


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class NonFiniteState(LbmError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("beta", ctypes.c_double), ("kappa", ctypes.c_double), ("rho_l", ctypes.c_double),
                ("rho_v", ctypes.c_double), ("rho0", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("precision", ctypes.c_int32), ("shift_all", ctypes.c_int32),
                ("force_stencil", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lattice3", ctypes.c_int32)]


class Observation(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("max_u", ctypes.c_double), ("mass", ctypes.c_double),
                ("kinetic_energy", ctypes.c_double), ("nonfinite", ctypes.c_int32),
                ("momentum", ctypes.c_double * 3)]


_lib = None
_VP, _D = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)


def header_functions() -> list:
    """Names of the functions include/lbm.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def load():
    """Load liblbm.so (after torch, so that both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm.so is not built (%s); run python -m paper_2012_11075_amd.build"
                          % LIB_PATH)
    import torch  # noqa: F401  (loads the HIP runtime liblbm.so links against)
    lib = ctypes.CDLL(LIB_PATH)
    P, O = ctypes.POINTER(Params), ctypes.POINTER(Observation)
    i32, i64, st = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    sig = {
        "lbm_workspace_bytes": (ctypes.c_size_t, [P]),
        "lbm_create": (st, [P, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
        "lbm_init": (st, [_VP, _D, _D, _D, st]),
        "lbm_step": (st, [_VP, i64, st]),
        "lbm_observe": (st, [_VP, _D, _D, _D, _D, O]),
        "lbm_init3d": (st, [_VP, _D, _D, _D, _D, st]),
        "lbm_observe3d": (st, [_VP, _D, _D, _D, _D, _D, O]),
        "lbm_observe_noalloc": (st, [_VP, _VP]),
        "lbm_get_populations": (st, [_VP, _D]),
        "lbm_get_populations_window": (st, [_VP, i32, i32, i32, i32, _D]),
        "lbm_set_populations": (st, [_VP, _D, st, i64]),
        "lbm_set_tile": (st, [_VP, i32, i32, i32]),
        "lbm_get_tile": (st, [_VP, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "lbm_set_graph_steps": (st, [_VP, i32]),
        "lbm_destroy": (st, [_VP]),
        "lbm_status_string": (ctypes.c_char_p, [st]),
        "lbm_last_error": (ctypes.c_char_p, [_VP]),
        "lbm_kernels_per_step": (i32, [_VP]),
        "lbm_steps_per_launch": (i32, [_VP]),
        "lbm_batch_slot_bytes": (ctypes.c_size_t, [P]),
        "lbm_batch_overhead_bytes": (ctypes.c_size_t, [ctypes.c_size_t, i32]),
        "lbm_batch_create": (st, [_VP, ctypes.c_size_t, i32, _VP, ctypes.POINTER(_VP)]),
        "lbm_batch_admit": (st, [_VP, P, _D, st, ctypes.c_double, i64, ctypes.POINTER(i32)]),
        "lbm_batch_run": (st, [_VP, i32]),
        "lbm_batch_poll": (st, [_VP, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]),
        "lbm_batch_slot_info": (st, [_VP, i32, ctypes.POINTER(i32), O]),
        "lbm_batch_fetch": (st, [_VP, i32, _D, _D, _D, _D, O]),
        "lbm_batch_get_populations": (st, [_VP, i32, _D]),
        "lbm_batch_set_tile": (st, [_VP, i32, i32, i32, i32]),
        "lbm_batch_set_graph_steps": (st, [_VP, i32]),
        "lbm_batch_release": (st, [_VP, i32]),
        "lbm_batch_destroy": (st, [_VP]),
        "lbm_batch_last_error": (ctypes.c_char_p, [_VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _obs_dict(ob: Observation, nz: int) -> dict:
    """Scalars of an observation; momentum has two components in 2-D."""
    mom = tuple(ob.momentum[:3 if nz else 2])
    return {"step": ob.step, "max_u": ob.max_u, "mass": ob.mass,
            "kinetic_energy": ob.kinetic_energy, "nonfinite": bool(ob.nonfinite),
            "momentum": mom}


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _scheme(s) -> int:
    return SCHEMES[s] if isinstance(s, str) else int(s)


def make_params(nx, ny, tau, beta, kappa, rho_l, rho_v, rho0=0.0, precision="fp64",
                rho_ref=None, shift_all=False, force_stencil=0, nz=0, q3=19) -> Params:
    """force_stencil: 0 the central gradients of Sec. II in the force, 1 the
    fourth-order ones (single lattices only).  nz > 1: a 3-D lattice (single
    lattices) with q3 = 19 (D3Q19) or 27 (D3Q27) velocities.  All run in FP64
    or FP32-shifted storage."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if rho_ref is None:
        rho_ref = 0.5 * (rho_l + rho_v)
    return Params(int(nx), int(ny), float(tau), float(beta), float(kappa), float(rho_l),
                  float(rho_v), float(rho0), float(rho_ref), prec, int(bool(shift_all)),
                  int(force_stencil), int(nz), int(q3) if int(nz) > 1 else 0)


def stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Solver:
    """One periodic lattice on the current HIP device."""

    def __init__(self, nx, ny, tau, beta, kappa, rho_l, rho_v, rho0=0.0, precision="fp64",
                 rho_ref=None, shift_all=False, stream=None, force_stencil=0, nz=0, q3=19):
        import torch
        self.lib = load()
        self.params = make_params(nx, ny, tau, beta, kappa, rho_l, rho_v, rho0, precision,
                                  rho_ref, shift_all, force_stencil, nz, q3)
        self.nx, self.ny = int(nx), int(ny)
        self.nz = int(nz) if int(nz) > 1 else 0
        # field and population shapes: (ny, nx) and (9, ny, nx) in 2-D,
        # (nz, ny, nx) and (q3, nz, ny, nx) in 3-D
        self.shape = (self.nz, self.ny, self.nx) if self.nz else (self.ny, self.nx)
        self.q = int(q3) if self.nz else 9
        nbytes = self.lib.lbm_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise LbmError(-1, "invalid parameters")
        # torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        assert self.workspace.data_ptr() % 256 == 0
        self.stream = stream
        h = _VP()
        self._check(self.lib.lbm_create(ctypes.byref(self.params), self.workspace.data_ptr(),
                                        nbytes, stream_handle(stream), ctypes.byref(h)), None)
        self.ctx = h

    @classmethod
    def for_problem(cls, problem, precision="fp64", **kw):
        ph = problem.physics
        return cls(problem.nx, problem.ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                   precision=precision, **kw)

    def _check(self, status, ctx=-1):
        if status != 0:
            c = self.ctx if ctx == -1 else ctx
            msg = self.lib.lbm_last_error(c).decode()
            if status == -4:
                raise NonFiniteState(status, msg)
            raise LbmError(status, msg)

    def init(self, rho, ux=None, uy=None, scheme="well_balanced", uz=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        assert rho.shape == self.shape
        comps = [ux, uy, uz] if self.nz else [ux, uy]
        if ux is not None:
            comps = [np.ascontiguousarray(np.broadcast_to(a, rho.shape), dtype=np.float64)
                     for a in comps]
        else:
            comps = [None] * len(comps)
        if self.nz:
            self._check(self.lib.lbm_init3d(self.ctx, _dptr(rho), *[_dptr(a) for a in comps],
                                            _scheme(scheme)))
        else:
            self._check(self.lib.lbm_init(self.ctx, _dptr(rho), *[_dptr(a) for a in comps],
                                          _scheme(scheme)))
        return self

    def step(self, n=1, scheme="well_balanced"):
        self._check(self.lib.lbm_step(self.ctx, int(n), _scheme(scheme)))
        return self

    def observe(self, fields=("rho", "ux", "uy", "uz", "mu"), raise_nonfinite=True) -> dict:
        out = {k: np.empty(self.shape) for k in fields if k != "uz" or self.nz}
        obs = Observation()
        if self.nz:
            st = self.lib.lbm_observe3d(self.ctx, _dptr(out.get("rho")), _dptr(out.get("ux")),
                                        _dptr(out.get("uy")), _dptr(out.get("uz")),
                                        _dptr(out.get("mu")), ctypes.byref(obs))
        else:
            st = self.lib.lbm_observe(self.ctx, _dptr(out.get("rho")), _dptr(out.get("ux")),
                                      _dptr(out.get("uy")), _dptr(out.get("mu")), ctypes.byref(obs))
        if st != -4 or raise_nonfinite:
            self._check(st)
        out.update(_obs_dict(obs, self.nz))
        return out

    def observe_noalloc(self, out) -> None:
        """Enqueue lbm_observe_noalloc on the solver's stream: `out` is a CUDA
        float64 tensor of 8 elements (max|u|, mass, E, non-finite flag,
        momentum x, y, z, 0), valid once the stream has been synchronized."""
        import torch
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() >= 8
        assert out.is_contiguous()
        self._check(self.lib.lbm_observe_noalloc(self.ctx, ctypes.c_void_p(out.data_ptr())))

    def get_populations_window(self, x0, y0, w, h) -> np.ndarray:
        """Populations of the (periodic) window at columns x0.., rows y0.. as
        (9, h, w) doubles (2-D lattices)."""
        f = np.empty((9, int(h), int(w)))
        self._check(self.lib.lbm_get_populations_window(self.ctx, int(x0), int(y0), int(w),
                                                        int(h), _dptr(f)))
        return f

    def get_populations(self) -> np.ndarray:
        """Populations as (9, ny, nx) doubles (unshifted); 3-D: (q3, nz, ny, nx)."""
        f = np.empty((self.q,) + self.shape)
        self._check(self.lib.lbm_get_populations(self.ctx, _dptr(f)))
        return f

    def set_populations(self, f: np.ndarray, scheme="well_balanced", step=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (self.q,) + self.shape
        self._check(self.lib.lbm_set_populations(self.ctx, _dptr(f), _scheme(scheme), int(step)))
        return self

    def set_tile(self, block=0, rows=0, depth=0):
        self._check(self.lib.lbm_set_tile(self.ctx, int(block), int(rows), int(depth)))
        return self

    def get_tile(self):
        b, r, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.lbm_get_tile(self.ctx, ctypes.byref(b), ctypes.byref(r),
                                          ctypes.byref(d)))
        return b.value, r.value, d.value

    def set_graph_steps(self, k):
        self._check(self.lib.lbm_set_graph_steps(self.ctx, int(k)))
        return self

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SLOT_STATUS = {0: "free", 1: "active", 2: "converged", 3: "capped", 4: "diverged"}


class Batch:
    """Many independent lattices in one device arena, advanced together by
    batched launches, one per group of slots (see the lbm_batch_* calls of lbm.h)."""

    def __init__(self, arena_bytes: int, max_slots: int = 1024, stream=None):
        import torch
        self.lib = load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        assert self.arena.data_ptr() % 256 == 0
        h = _VP()
        st = self.lib.lbm_batch_create(self.arena.data_ptr(), int(arena_bytes), int(max_slots),
                                       stream_handle(stream), ctypes.byref(h))
        if st != 0:
            raise LbmError(st, self.lib.lbm_batch_last_error(None).decode())
        self.b = h
        self.shapes = {}   # slot -> field shape
        self.qs = {}       # slot -> populations per node

    def _check(self, st):
        if st != 0:
            msg = self.lib.lbm_batch_last_error(self.b).decode()
            if st == -4:
                raise NonFiniteState(st, msg)
            raise LbmError(st, msg)

    @staticmethod
    def slot_bytes(params: Params) -> int:
        return int(load().lbm_batch_slot_bytes(ctypes.byref(params)))

    @staticmethod
    def overhead_bytes(arena_bytes: int, max_slots: int) -> int:
        return int(load().lbm_batch_overhead_bytes(int(arena_bytes), int(max_slots)))

    def admit(self, params: Params, rho, scheme="well_balanced", tol=0.0, step_cap=0) -> int:
        """rho: (ny, nx), or (nz, ny, nx) for a 3-D lattice (params.nz > 1)."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        d3 = params.nz > 1
        shape = (params.nz, params.ny, params.nx) if d3 else (params.ny, params.nx)
        assert rho.shape == shape
        slot = ctypes.c_int32()
        self._check(self.lib.lbm_batch_admit(self.b, ctypes.byref(params), _dptr(rho), _scheme(scheme),
                                             float(tol), int(step_cap), ctypes.byref(slot)))
        self.shapes[slot.value] = shape
        self.qs[slot.value] = (params.lattice3 or 19) if d3 else 9
        return slot.value

    def try_admit(self, *a, **kw):
        """admit(), or None when no slot or arena range is free."""
        try:
            return self.admit(*a, **kw)
        except LbmError as e:
            if e.status == -6:
                return None
            raise

    def run(self, k: int):
        self._check(self.lib.lbm_batch_run(self.b, int(k)))

    def poll(self, cap: int = 65536) -> list:
        buf = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        self._check(self.lib.lbm_batch_poll(self.b, buf, cap, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def info(self, slot: int):
        st, ob = ctypes.c_int32(), Observation()
        self._check(self.lib.lbm_batch_slot_info(self.b, int(slot), ctypes.byref(st), ctypes.byref(ob)))
        return SLOT_STATUS[st.value], _obs_dict(ob, 0)

    def fetch(self, slot: int, fields=("rho", "ux", "uy", "mu")) -> dict:
        out = {k: np.empty(self.shapes[slot]) for k in fields}
        ob = Observation()
        st = self.lib.lbm_batch_fetch(self.b, int(slot), _dptr(out.get("rho")), _dptr(out.get("ux")),
                                      _dptr(out.get("uy")), _dptr(out.get("mu")), ctypes.byref(ob))
        if st not in (0, -4):
            self._check(st)
        out.update(_obs_dict(ob, 0))
        return out

    def get_populations(self, slot: int) -> np.ndarray:
        f = np.empty((self.qs[slot],) + self.shapes[slot])
        self._check(self.lib.lbm_batch_get_populations(self.b, int(slot), _dptr(f)))
        return f

    def set_tile(self, slot, block=0, rows=0, depth=0):
        self._check(self.lib.lbm_batch_set_tile(self.b, int(slot), int(block), int(rows), int(depth)))

    def set_graph_steps(self, k: int):
        self._check(self.lib.lbm_batch_set_graph_steps(self.b, int(k)))

    def release(self, slot: int):
        self._check(self.lib.lbm_batch_release(self.b, int(slot)))
        self.shapes.pop(slot, None)
        self.qs.pop(slot, None)

    def close(self):
        if getattr(self, "b", None):
            self.lib.lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
