"""The 3-D step on the D3Q27 lattice on the GPU against the D3Q27 FP64
oracle, through the C ABI: populations, fields and observables at 1e-11
after the stated steps (all three schemes; lattices with partial blocks in
every direction and periodic wrap over a few nodes), initial velocity,
checkpoint/resume, graph replay, the well-balanced fixed point of a flat
interface along each axis, every tiling bit for bit, FP32-shifted storage,
the degenerate cases and sampled nodes of a 256^3 lattice."""
import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I
from equilibrium import flat_equilibrium

pytestmark = pytest.mark.gpu
TOL = 1e-11
Q = 27


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_11075_amd import lbm as L
    L.load()
    return L


def solver(L, nx, ny, nz, ph, precision="fp64"):
    return L.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0, nz=nz,
                    precision=precision, q3=Q)


def to_oracle(f):
    """(27, nz, ny, nx) -> (nz, ny, nx, 27)."""
    assert f.shape[0] == Q
    return np.ascontiguousarray(np.moveaxis(f, 0, -1))


CASES = [(16, 12, 10, 300), (33, 9, 5, 200), (1, 7, 3, 200), (5, 2, 6, 200), (40, 24, 16, 100)]


@pytest.mark.parametrize("scheme", ["well_balanced", "standard", "standard_eq_forcing"])
@pytest.mark.parametrize("nx,ny,nz,steps", CASES)
def test_parity_d3q27(orc, lbm, nx, ny, nz, steps, scheme):
    ph = I.PAPER_PHYS
    print("parity case D3Q27", nx, ny, nz, scheme, steps, flush=True)
    rho0 = I.droplet3_density(nx, ny, nz, ph, 0.3 * min(nx, ny, nz) + 1.0, 4.0, 1e-2, seed=7)
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    fo = orc.step3(scheme, p, orc.init3(scheme, p, rho0, q=Q), steps)
    m = orc.macro3(scheme, p, fo)
    oo = orc.observe3(scheme, p, fo)
    assert np.isfinite(fo).all() and m["rho"].min() > 0
    s = solver(lbm, nx, ny, nz, ph)
    assert s.lib.lbm_kernels_per_step(s.ctx) == 1
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
    # |dE| <= TOL sqrt(2 mass E) + TOL^2 mass / 2 (Cauchy-Schwarz), plus rho's share
    E, M = oo["kinetic_energy"], oo["mass"]
    assert abs(ob["kinetic_energy"] - E) <= TOL * np.sqrt(2 * M * E) + 0.5 * TOL ** 2 * M + 1e-9 * E
    np.testing.assert_allclose(ob["momentum"], oo["momentum"], rtol=0, atol=TOL * M + 1e-12)


def test_d3q27_differs_from_d3q19(orc, lbm):
    """The two lattices give different results for the same droplet (the
    corner velocities take part): the GPU runs the lattice asked for."""
    ph = I.PAPER_PHYS
    nx, ny, nz = 14, 12, 10
    rho0 = I.droplet3_density(nx, ny, nz, ph, 4.0, 4.0, 1e-2, seed=9)
    out = {}
    for q in (19, 27):
        s = lbm.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, nz=nz, q3=q)
        s.init(rho0, scheme="well_balanced")
        s.step(50, "well_balanced")
        out[q] = s.observe(fields=("rho",))["rho"]
        s.close()
    assert np.abs(out[19] - out[27]).max() > 1e-8


def test_initial_velocity_d3q27(orc, lbm):
    ph = I.PAPER_PHYS
    nx, ny, nz = 12, 10, 8
    rng = np.random.default_rng(11)
    rho0 = 1.0 + 0.05 * rng.uniform(-1, 1, (nz, ny, nx))
    u = [0.02 * rng.uniform(-1, 1, (nz, ny, nx)) for _ in range(3)]
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v)
    fo = orc.step3("standard", p, orc.init3("standard", p, rho0, u, q=Q), 50)
    s = solver(lbm, nx, ny, nz, ph)
    s.init(rho0, u[0], u[1], scheme="standard", uz=u[2])
    s.step(50, "standard")
    assert np.abs(to_oracle(s.get_populations()) - fo).max() <= TOL
    s.close()


def test_checkpoint_and_graph_replay_d3q27(lbm):
    ph = I.PAPER_PHYS
    nx, ny, nz = 20, 14, 9
    rho0 = I.droplet3_density(nx, ny, nz, ph, 4.0, 4.0, 1e-2, seed=3)
    s = solver(lbm, nx, ny, nz, ph)
    s.init(rho0, scheme="well_balanced")
    s.step(40, "well_balanced")
    ck = s.get_populations()
    assert ck.shape == (Q, nz, ny, nx)
    s.step(26, "well_balanced")
    want = s.get_populations()
    s.set_populations(ck, "well_balanced", step=40)
    s.set_graph_steps(8)
    s.step(26, "well_balanced")
    assert np.array_equal(s.get_populations(), want)
    assert s.observe(fields=())["step"] == 66
    s.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_wb_flat_interface_fixed_point_d3q27(lbm, axis):
    """Sec. III in 3-D on the D3Q27 lattice: the discrete flat-interface
    equilibrium (the same profile as on D2Q9 and D3Q19: the stencils reduce
    to the central difference and the 3-point Laplacian along one axis)
    stays at rest to round-off under the WB step."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("scheme", ["well_balanced", "standard", "standard_eq_forcing"])
def test_tilings_bit_identical_d3q27(orc, lbm, scheme, prec):
    """Every D3Q27 tiling (32 x 8 tiles, ragged in x and y; chunks of 1 to 13
    planes, odd chunks marching towards -z; 1 or 2 planes in flight) gives
    the same populations bit for bit, and the oracle agrees (1e-11 in FP64,
    the FP32 bound in FP32-shifted storage)."""
    ph = I.PAPER_PHYS
    nx, ny, nz, steps = 37, 19, 13, 60
    print("tilings D3Q27", nx, ny, nz, scheme, prec, flush=True)
    rho0 = I.droplet3_density(nx, ny, nz, ph, 5.0, 4.0, 1e-2, seed=5)
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    fo = orc.step3(scheme, p, orc.init3(scheme, p, rho0, q=Q), steps)
    ref = None
    for block, rows, depth in [(256, 0, 1), (256, 1, 1), (256, 2, 2), (256, 5, 2), (256, 13, 1),
                               (256, 4, 1)]:
        s = solver(lbm, nx, ny, nz, ph, prec)
        s.set_tile(block, rows, depth)
        b, r, d = s.get_tile()
        assert b == block and d == depth and (rows == 0 or r == rows)
        s.init(rho0, scheme=scheme)
        s.step(steps, scheme)
        f = s.get_populations()
        s.close()
        if ref is None:
            ref = f
            assert np.abs(to_oracle(f) - fo).max() <= (TOL if prec == "fp64" else 5e-5)
        else:
            assert np.array_equal(f, ref), (block, rows, depth)


def test_tile_choice_errors_d3q27(lbm):
    """D3Q27 runs 32 x 8 tiles with 1 or 2 planes in flight only."""
    ph = I.PAPER_PHYS
    s = solver(lbm, 8, 8, 8, ph)
    for args in [(512, 4, 1), (512, 4, 2), (256, 4, 3), (128, 4, 1), (256, -1, 1)]:
        with pytest.raises(lbm.LbmError):
            s.set_tile(*args)
    assert s.get_tile()[0] == 256
    s.close()


@pytest.mark.parametrize("scheme", ["well_balanced", "standard"])
def test_fp32_d3q27_against_oracle(orc, lbm, scheme):
    """FP32-shifted storage against the FP64 oracle after 300 steps, with the
    FP32 bounds of the other lattices (rho, f < 5e-5, u < 1e-5); mass to
    1e-5."""
    ph = I.PAPER_PHYS
    nx, ny, nz, steps = 40, 24, 16, 300
    rho0 = I.droplet3_density(nx, ny, nz, ph, 0.3 * min(nx, ny, nz) + 1.0, 4.0, 1e-2, seed=7)
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    fo = orc.step3(scheme, p, orc.init3(scheme, p, rho0, q=Q), steps)
    m = orc.macro3(scheme, p, fo)
    s = solver(lbm, nx, ny, nz, ph, "fp32s")
    s.init(rho0, scheme=scheme)
    s.step(steps, scheme)
    f32 = to_oracle(s.get_populations())
    ob = s.observe()
    s.close()
    e_rho = np.abs(ob["rho"] - m["rho"]).max()
    e_u = max(np.abs(ob[k] - m[k]).max() for k in ("ux", "uy", "uz"))
    e_f = np.abs(f32 - fo).max()
    print("D3Q27 fp32 vs oracle, %s, %d steps: rho %.3e  u %.3e  f %.3e"
          % (scheme, steps, e_rho, e_u, e_f))
    assert e_rho < 5e-5 and e_u < 1e-5 and e_f < 5e-5
    assert abs(ob["mass"] - orc.observe3(scheme, p, fo)["mass"]) < 1e-5 * ob["mass"]


def test_fp32_d3q27_scheme_switch_keeps_populations(lbm):
    ph = I.PAPER_PHYS
    rho0 = I.droplet3_density(20, 16, 12, ph, 5.0, 4.0, 1e-2, seed=3)
    s = solver(lbm, 20, 16, 12, ph, "fp32s")
    s.init(rho0, scheme="well_balanced")
    s.step(30, "well_balanced")
    a = s.get_populations()
    s.step(0, "standard")
    b = s.get_populations()
    s.step(0, "well_balanced")
    c = s.get_populations()
    s.close()
    assert np.abs(b - a).max() <= 1.2e-7 and np.abs(c - a).max() <= 1.2e-7


@pytest.mark.parametrize("scheme", ["well_balanced", "standard", "standard_eq_forcing"])
def test_degenerate_cases_d3q27(orc, lbm, scheme):
    """The single-phase limit beta = kappa = 0 against the oracle to 1e-11
    and a uniform density at rest (unchanged bit for bit under WB, to
    round-off otherwise)."""
    nx, ny, nz = 21, 13, 11
    rng = np.random.default_rng(29)
    rho0 = 1.0 + 0.05 * rng.uniform(-1, 1, (nz, ny, nx))
    p = orc.Params(0.9, 0.0, 0.0, 1.0, 0.1)
    fo = orc.step3(scheme, p, orc.init3(scheme, p, rho0, q=Q), 150)
    s = lbm.Solver(nx, ny, 0.9, 0.0, 0.0, 1.0, 0.1, nz=nz, q3=Q)
    s.init(rho0, scheme=scheme)
    s.step(150, scheme)
    assert np.abs(to_oracle(s.get_populations()) - fo).max() <= TOL
    s.close()
    ph = I.PAPER_PHYS
    s = solver(lbm, nx, ny, nz, ph)
    s.init(np.full((nz, ny, nx), 0.7), scheme=scheme)
    f0 = s.get_populations()
    s.step(60, scheme)
    f1 = s.get_populations()
    s.close()
    if scheme == "well_balanced":
        assert np.array_equal(f0, f1)
    else:
        assert np.abs(f1 - f0).max() <= 1e-15


def test_full_grid_sampled_d3q27(orc, lbm):
    """The 256^3 droplet on D3Q27 in the default launch configuration: after
    20 steps, one more GPU step against the oracle's step on periodic crops
    around sampled windows, across tile, chunk and lattice seams."""
    n, ph = 256, I.PHYS3
    rho = I.droplet3_density(n, n, n, ph, I.DROPLET3_RADIUS * n / I.DROPLET3_SIDE,
                             I.equilibrium_width(ph), 1e-3, seed=13)
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    s = solver(lbm, n, n, n, ph)
    s.init(rho, scheme="well_balanced")
    del rho
    s.step(20, "well_balanced")
    f = s.get_populations()
    s.step(1, "well_balanced")
    g = s.get_populations()
    s.close()
    rng = np.random.default_rng(5)
    corners = [(0, 0, 0), (250, 250, 250), (62, 5, 30), (126, 100, 60), (190, 201, 222)]
    corners += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(4)]
    W, M = 14, 3
    for (z0, y0, x0) in corners:
        zs = np.arange(z0 - M, z0 + W - M) % n
        ys = np.arange(y0 - M, y0 + W - M) % n
        xs = np.arange(x0 - M, x0 + W - M) % n
        crop = to_oracle(f[:, zs][:, :, ys][:, :, :, xs])
        want = orc.step3("well_balanced", p, crop, 1)[M:-M, M:-M, M:-M]
        got = to_oracle(g[:, zs[M:-M]][:, :, ys[M:-M]][:, :, :, xs[M:-M]])
        assert np.abs(got - want).max() <= 1e-12, (z0, y0, x0)


@pytest.mark.parametrize("q", [19, 27])
def test_parity_wb_rho0_3d(orc, lbm, q):
    """Eq. (24) with rho0 != 0 in 3-D (reading 21): the WB step against the
    oracle to 1e-11 on both velocity sets, FP64, and the FP32-shifted form
    within its bound."""
    from dataclasses import replace
    ph = replace(I.PAPER_PHYS, rho0=0.5)
    nx, ny, nz, steps = 17, 11, 9, 150
    rho0 = I.droplet3_density(nx, ny, nz, ph, 4.0, 4.0, 1e-2, seed=19)
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    fo = orc.step3("well_balanced", p, orc.init3("well_balanced", p, rho0, q=q), steps)
    for prec, tol in (("fp64", TOL), ("fp32s", 5e-5)):
        s = lbm.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0, nz=nz,
                       q3=q, precision=prec)
        s.init(rho0, scheme="well_balanced")
        s.step(steps, "well_balanced")
        f = np.moveaxis(s.get_populations(), 0, -1)
        s.close()
        assert np.abs(f - fo).max() <= tol, (q, prec)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("nx,ny,nz", [(6, 1, 2), (1, 1, 3), (2, 3, 2), (1, 5, 2)])
def test_degenerate_shapes_3d(orc, lbm, q, nx, ny, nz):
    """The thinnest 3-D lattices the library accepts (nz = 2, a single row or
    column; every stencil and pull wraps onto the same few nodes) against the
    oracle, WB and standard, to 1e-11."""
    ph = I.PAPER_PHYS
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    rho0 = 0.5 + 0.3 * rng.uniform(-1, 1, (nz, ny, nx))
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    for scheme in ("well_balanced", "standard"):
        fo = orc.step3(scheme, p, orc.init3(scheme, p, rho0, q=q), 40)
        s = lbm.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, nz=nz, q3=q)
        s.init(rho0, scheme=scheme)
        s.step(40, scheme)
        f = np.moveaxis(s.get_populations(), 0, -1)
        s.close()
        assert np.isfinite(fo).all()
        assert np.abs(f - fo).max() <= TOL, (scheme, q, nx, ny, nz)
