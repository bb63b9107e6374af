"""The step at the largest lattices the library accepts (2^31 nodes) and
HBM holds: element offsets into one population copy far beyond 2^32.

No whole population array comes back to the host (it would be 77-155 GB):
windows of it do (lbm_get_populations_window).  The initial populations are
a local function of the initial density, so the oracle rebuilds any
window's state from the same density; after one GPU step, the populations
f, rho and u of sampled windows (the far corner, the periodic seams, the
middle, random places) are compared with the oracle's step on periodic
crops with a 3-node margin (5 for u).
"""
import ctypes
import gc

import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I

pytestmark = pytest.mark.gpu


def _run(orc, nx, ny, precision, scheme, tol, tol_u):
    import torch
    from paper_2012_11075_amd import lbm
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ph = I.PAPER_PHYS
    prm = lbm.make_params(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                          precision=precision)
    need = lbm.load().lbm_workspace_bytes(ctypes.byref(prm))
    assert need > 0
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need + (2 << 30):
        pytest.skip("needs %.0f GB of free device memory, %.0f GB free" % (need / 1e9, free / 1e9))
    print("max-size case", nx, ny, precision, scheme, "workspace %.1f GB" % (need / 1e9), flush=True)
    rho0 = I.separable_density(nx, ny, 17)
    s = lbm.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                   precision=precision)
    s.init(rho0, scheme=scheme)
    s.step(1, scheme)
    ob = s.observe(fields=("rho", "ux", "uy"))
    assert not ob["nonfinite"] and ob["step"] == 1
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    rng = np.random.default_rng(5)
    W, M = 22, 3
    corners = [(ny - W + M, nx - W + M), (ny - 1, nx - 1), (0, 0), (ny // 2, nx // 2),
               (ny - 2, 7), (5, nx - 3)]
    corners += [(int(rng.integers(0, ny)), int(rng.integers(0, nx))) for _ in range(6)]
    worst = {"f": 0.0, "rho": 0.0, "u": 0.0}
    for (y0, x0) in corners:
        ys = np.arange(y0 - M, y0 + W - M) % ny
        xs = np.arange(x0 - M, x0 + W - M) % nx
        crop = np.ascontiguousarray(rho0[ys][:, xs])
        fo = orc.step(scheme, p, orc.init(scheme, p, crop), 1)
        ro, uxo, uyo, _ = orc.fields(scheme, p, fo)
        inner = (slice(M, -M), slice(M, -M))
        # populations of the window whose origin is the crop's first interior node
        fw = s.get_populations_window(int(xs[M]), int(ys[M]), W - 2 * M, W - 2 * M)
        # u(t=1) needs f(t=1) up to two nodes away (the stencils of mu and of
        # its gradient), exact on the crop only 2 nodes further in
        U = M + 2
        uin = (slice(U, -U), slice(U, -U))
        err = {"f": np.abs(np.transpose(fw, (1, 2, 0)) - fo[inner]).max(),
               "rho": np.abs(ob["rho"][ys[M:-M]][:, xs[M:-M]] - ro[inner]).max(),
               "u": max(np.abs(ob["ux"][ys[U:-U]][:, xs[U:-U]] - uxo[uin]).max(),
                        np.abs(ob["uy"][ys[U:-U]][:, xs[U:-U]] - uyo[uin]).max())}
        for k, v in err.items():
            worst[k] = max(worst[k], v)
        assert err["f"] <= tol and err["rho"] <= tol and err["u"] <= tol_u, (y0, x0, err)
    s.close()
    del s, ob
    gc.collect()
    torch.cuda.empty_cache()
    print("max-size case", nx, ny, precision, "worst errors", worst, flush=True)


def test_fp64_32768_squared(orc):
    """FP64 at 32768^2 (1.07e9 nodes, 77 GB per population copy): f, rho and
    u to 1e-12."""
    _run(orc, 32768, 32768, "fp64", "well_balanced", 1e-12, 1e-12)


def test_fp32_at_the_node_limit(orc):
    """FP32-shifted at 46340^2 = 2,147,395,600 nodes, the largest square
    lattice within the 2^31-node limit (155 GB of populations): within the
    FP32 bound of one step: f and rho to 2e-6, u to 1e-6."""
    _run(orc, 46340, 46340, "fp32s", "standard", 2e-6, 1e-6)
