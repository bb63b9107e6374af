"""lbm_observe_noalloc (the entry point that allocates nothing) against
lbm_observe, through the C ABI: two calls in a row, the second on a smaller
lattice, each bit-identical to lbm_observe's scalars on the same state."""
import ctypes

import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_11075_amd import lbm as L
    L.load()
    return L


def _run(L, prob, steps, tile=None):
    s = L.Solver.for_problem(prob)
    if tile:
        s.set_tile(*tile)
    s.init(prob.rho(), scheme="well_balanced")
    s.step(steps, "well_balanced")
    return s


def _noalloc(s):
    import torch
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    s.observe_noalloc(out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(v, ref):
    assert v[0] == ref["max_u"]
    assert v[1] == ref["mass"]
    assert v[2] == ref["kinetic_energy"]
    assert v[3] == (1.0 if ref["nonfinite"] else 0.0)
    assert v[4] == ref["momentum"][0] and v[5] == ref["momentum"][1]
    assert v[6] == 0.0 and v[7] == 0.0


def test_noalloc_matches_observe_two_calls(lbm):
    big = I.with_size(I.PAPER_DROPLET, 300, 211)
    small = I.with_size(I.PAPER_DROPLET, 70, 45)
    print("noalloc case", big.nx, big.ny, "then", small.nx, small.ny, flush=True)
    sa = _run(lbm, big, 200, tile=(64, 8, 2))     # 5 x 27 tiles, ragged in x and y
    va = _noalloc(sa)
    ra = sa.observe(fields=())
    _check(va, ra)
    sb = _run(lbm, small, 150)
    vb = _noalloc(sb)
    rb = sb.observe(fields=())
    _check(vb, rb)
    assert abs(vb[1] - va[1]) > 1.0       # the second call reports its own lattice
    # back on the first lattice after the smaller one used the shared array
    _check(_noalloc(sa), ra)
    sa.close()
    sb.close()


def test_noalloc_reports_nonfinite(lbm):
    prob = I.with_size(I.DROPLET_512_RATIO100, 96, 80)
    s = _run(lbm, prob, 200)        # density ratio 100 at width 1.3: diverges
    v = _noalloc(s)
    ref = s.observe(fields=(), raise_nonfinite=False)
    assert ref["nonfinite"] and v[3] == 1.0
    s.close()


def test_noalloc_argument_errors(lbm):
    prob = I.with_size(I.PAPER_DROPLET, 64, 48)
    s = lbm.Solver.for_problem(prob)
    import torch
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    assert s.lib.lbm_observe_noalloc(s.ctx, ctypes.c_void_p(out.data_ptr())) == -5  # before init
    s.init(prob.rho(), scheme="well_balanced")
    assert s.lib.lbm_observe_noalloc(s.ctx, None) == -1
    assert s.lib.lbm_observe_noalloc(None, ctypes.c_void_p(out.data_ptr())) == -1
    s.close()
    s4 = lbm.Solver.for_problem(prob, force_stencil=1)
    s4.init(prob.rho(), scheme="well_balanced")
    assert s4.lib.lbm_observe_noalloc(s4.ctx, ctypes.c_void_p(out.data_ptr())) == -1
    assert b"central force stencil" in s4.lib.lbm_last_error(s4.ctx)
    s4.close()
    # more tiles than the static array holds: 16384 x 2052 in 64 x 4 tiles is
    # 256 x 513 = 131328 tiles (the check comes before any device work)
    big = lbm.Solver(16384, 2052, 1.0, 0.01, 0.0128, 1.0, 0.2, precision="fp32s")
    big.set_tile(64, 4, 1)
    assert big.lib.lbm_observe_noalloc(big.ctx, ctypes.c_void_p(out.data_ptr())) == -1
    assert b"131072 tiles" in big.lib.lbm_last_error(big.ctx)
    big.close()
