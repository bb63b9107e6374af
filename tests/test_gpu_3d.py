"""The 3-D (D3Q19) step on the GPU against the 3-D FP64 oracle, through the
C ABI: populations, fields and observables at 1e-11 after the stated steps
(both schemes; lattices with partial blocks in every direction and periodic
wrap over a few nodes), initial velocity, checkpoint/resume, graph replay and
the well-balanced fixed point of a flat interface along each axis."""
import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I
from equilibrium import flat_equilibrium

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_11075_amd import lbm as L
    L.load()
    return L


def solver(L, nx, ny, nz, ph):
    return L.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0, nz=nz)


def to_oracle(f):
    """(19, nz, ny, nx) -> (nz, ny, nx, 19)."""
    return np.ascontiguousarray(np.moveaxis(f, 0, -1))


CASES3 = [(16, 12, 10, 300), (33, 9, 5, 200), (1, 7, 3, 200), (5, 2, 6, 200), (40, 24, 16, 100)]


@pytest.mark.parametrize("scheme", ["well_balanced", "standard"])
@pytest.mark.parametrize("nx,ny,nz,steps", CASES3)
def test_parity_3d(orc, lbm, nx, ny, nz, steps, scheme):
    ph = I.PAPER_PHYS
    print("parity case 3-D", nx, ny, nz, scheme, steps, flush=True)
    rho0 = I.droplet3_density(nx, ny, nz, ph, 0.3 * min(nx, ny, nz) + 1.0, 4.0, 1e-2, seed=7)
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    fo = orc.step3(scheme, p, orc.init3(scheme, p, rho0), steps)
    m = orc.macro3(scheme, p, fo)
    oo = orc.observe3(scheme, p, fo)
    assert np.isfinite(fo).all() and m["rho"].min() > 0
    s = solver(lbm, nx, ny, nz, ph)
    assert s.lib.lbm_kernels_per_step(s.ctx) == 3
    s.init(rho0, scheme=scheme)
    s.step(steps, scheme)
    fg = to_oracle(s.get_populations())
    ob = s.observe()
    s.close()
    assert np.abs(fg - fo).max() <= TOL
    for k in ("rho", "ux", "uy", "uz"):
        assert np.abs(ob[k] - m[k]).max() <= TOL, k
    assert np.abs(ob["mu"] - m["mu"]).max() <= 1e-9 * max(1.0, np.abs(m["mu"]).max())
    assert abs(ob["max_u"] - oo["max_u"]) <= TOL
    assert abs(ob["mass"] - oo["mass"]) <= 1e-12 * oo["mass"]
    assert abs(ob["kinetic_energy"] - oo["kinetic_energy"]) <= 1e-9 * max(oo["kinetic_energy"], 1e-30)


def test_initial_velocity_3d(orc, lbm):
    ph = I.PAPER_PHYS
    nx, ny, nz = 12, 10, 8
    rng = np.random.default_rng(11)
    rho0 = 1.0 + 0.05 * rng.uniform(-1, 1, (nz, ny, nx))
    u = [0.02 * rng.uniform(-1, 1, (nz, ny, nx)) for _ in range(3)]
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v)
    fo = orc.step3("standard", p, orc.init3("standard", p, rho0, u), 50)
    s = solver(lbm, nx, ny, nz, ph)
    s.init(rho0, u[0], u[1], scheme="standard", uz=u[2])
    s.step(50, "standard")
    assert np.abs(to_oracle(s.get_populations()) - fo).max() <= TOL
    s.close()


def test_checkpoint_and_graph_replay_3d(lbm):
    ph = I.PAPER_PHYS
    nx, ny, nz = 20, 14, 9
    rho0 = I.droplet3_density(nx, ny, nz, ph, 4.0, 4.0, 1e-2, seed=3)
    s = solver(lbm, nx, ny, nz, ph)
    s.init(rho0, scheme="well_balanced")
    s.step(40, "well_balanced")
    ck = s.get_populations()
    s.step(26, "well_balanced")
    want = s.get_populations()
    s.set_populations(ck, "well_balanced", step=40)
    s.set_graph_steps(8)
    s.step(26, "well_balanced")
    assert np.array_equal(s.get_populations(), want)
    assert s.observe(fields=())["step"] == 66
    with pytest.raises(lbm.LbmError):
        s.set_tile(128, 32, 2)
    s.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_wb_flat_interface_fixed_point_3d(lbm, axis):
    """Sec. III in 3-D on the GPU: the discrete flat-interface equilibrium
    stays at rest to round-off under the WB step, along each axis."""
    ph = I.PAPER_PHYS
    n = 41
    W = np.sqrt(8 * ph.kappa / ph.beta) / (ph.rho_l - ph.rho_v)
    guess = I.tanh_slab(n, ph.rho_l, ph.rho_v, 10.5, 29.5, W)
    prof, _ = flat_equilibrium(ph.beta, ph.kappa, ph.rho_l, ph.rho_v, n, guess.sum(), guess)
    shape = [4, 4, 4]
    shape[axis] = n
    rho = np.broadcast_to(prof.reshape([-1 if a == axis else 1 for a in range(3)]), shape).copy()
    nz, ny, nx = rho.shape
    s = solver(lbm, nx, ny, nz, ph)
    s.init(rho, scheme="well_balanced")
    s.step(500, "well_balanced")
    ob = s.observe(fields=())
    s.close()
    assert ob["max_u"] < 1e-14
