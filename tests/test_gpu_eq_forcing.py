"""GPU step of the standard LBE with the forcing term named after Eq. (5),
F_i = (c_i - u).F feq_i / (cs2 rho), against the FP64 CPU oracle through
the C ABI (scheme LBM_STANDARD_EQ_FORCING; its 3-D form is covered by
tests/test_gpu_3d.py).

Same bar as the other parity tests: max abs difference <= 1e-11 on f, rho and
u after fixed step counts in FP64; the FP32-shifted bounds of the main step in
FP32.  Cases: the paper's workloads, ragged lattices with partial tiles and
wrapped halos, both force stencils, several tilings, scheme switches, and the
4096^2 grid in its benchmark launch configuration on sampled windows.
"""
import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-11
EQF = "standard_eq_forcing"


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_11075_amd import lbm as L
    L.load()
    return L


def oparams(orc, ph, stencil=0):
    return orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0, stencil)


def to_oracle(f9):
    """(9, ny, nx) -> (ny, nx, 9)."""
    return np.ascontiguousarray(np.transpose(f9, (1, 2, 0)))


def compare(orc, L, prob, steps, stencil=0, tile=None):
    print("parity case", EQF, prob.name, prob.nx, prob.ny, steps, "stencil", stencil, tile,
          flush=True)
    p = oparams(orc, prob.physics, stencil)
    rho0 = prob.rho()
    fo = orc.step(EQF, p, orc.init(EQF, p, rho0), steps)
    ro, uxo, uyo, muo = orc.fields(EQF, p, fo)
    oo = orc.observe(EQF, p, fo)
    assert np.isfinite(fo).all() and ro.min() > 0, "oracle state diverged: pick fewer steps"
    s = L.Solver.for_problem(prob, force_stencil=stencil)
    if tile:
        s.set_tile(*tile)
    s.init(rho0, scheme=EQF)
    s.step(steps, EQF)
    fg = to_oracle(s.get_populations())
    ob = s.observe()
    s.close()
    assert np.abs(fg - fo).max() <= TOL
    assert np.abs(ob["rho"] - ro).max() <= TOL
    assert np.abs(ob["ux"] - uxo).max() <= TOL
    assert np.abs(ob["uy"] - uyo).max() <= TOL
    assert np.abs(ob["mu"] - muo).max() <= 1e-9 * max(1.0, np.abs(muo).max())
    assert abs(ob["max_u"] - oo["max_u"]) <= TOL
    assert abs(ob["mass"] - oo["mass"]) <= 1e-12 * oo["mass"]


CASES = [("flat_200x4", 30), ("droplet_256", 30), ("paper_flat_21x101", 1000),
         ("paper_droplet_100", 1000), ("droplet_512_ratio100", 4)]


@pytest.mark.parametrize("name,steps", CASES)
def test_parity_eq_forcing_workloads(orc, lbm, name, steps):
    compare(orc, lbm, I.PROBLEMS[name], steps)


RAGGED = [(37, 53), (1, 7), (7, 1), (1, 1), (2, 2), (300, 5), (5, 300), (129, 130)]


@pytest.mark.parametrize("stencil", [0, 1])
@pytest.mark.parametrize("nx,ny", RAGGED)
def test_parity_eq_forcing_ragged(orc, lbm, nx, ny, stencil):
    compare(orc, lbm, I.with_size(I.PAPER_DROPLET, nx, ny), 200, stencil)


@pytest.mark.parametrize("stencil", [0, 1])
def test_eq_forcing_is_not_the_eq5_step(orc, lbm, stencil):
    """The two standard forcing terms give different trajectories, and the
    GPU's difference between them is the oracle's (so the scheme value
    really selects the other forcing term in the kernel)."""
    prob = I.with_size(I.PAPER_DROPLET, 64, 48)
    p = oparams(orc, prob.physics, stencil)
    out, ref = {}, {}
    for sch in ("standard", EQF):
        s = lbm.Solver.for_problem(prob, force_stencil=stencil)
        s.init(prob.rho(), scheme=sch)
        s.step(300, sch)
        out[sch] = to_oracle(s.get_populations())
        s.close()
        ref[sch] = orc.step(sch, p, orc.init(sch, p, prob.rho()), 300)
    d_gpu = out[EQF] - out["standard"]
    d_orc = ref[EQF] - ref["standard"]
    assert np.abs(d_orc).max() > 1e-8
    assert np.abs(d_gpu - d_orc).max() <= 2 * TOL


TILES = {0: [(128, 4, 1), (192, 7, 2), (256, 16, 3), (320, 33, 1), (512, 64, 2), (128, 5, 3)],
         1: [(256, 16, 2), (256, 4, 1), (256, 7, 3), (512, 45, 3), (512, 9, 2)]}


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
@pytest.mark.parametrize("stencil", [0, 1])
def test_eq_forcing_tilings_bit_identical(orc, lbm, stencil, prec):
    """Every tiling, and graph-captured steps, give the same populations bit
    for bit; the first agrees with the oracle (1e-11 FP64, 5e-5 FP32)."""
    prob = I.with_size(I.PAPER_DROPLET, 600, 45)
    steps = 100
    print("tilings", EQF, stencil, prec, flush=True)
    p = oparams(orc, prob.physics, stencil)
    fo = orc.step(EQF, p, orc.init(EQF, p, prob.rho()), steps)
    ref = None
    for k, tile in enumerate(TILES[stencil]):
        s = lbm.Solver.for_problem(prob, force_stencil=stencil, precision=prec)
        s.set_tile(*tile)
        if k == 1:
            s.set_graph_steps(16)
        s.init(prob.rho(), scheme=EQF)
        s.step(steps - 3, EQF)
        s.step(3, EQF)
        f = s.get_populations()
        s.close()
        if ref is None:
            ref = f
            assert np.abs(to_oracle(f) - fo).max() <= (TOL if prec == "fp64" else 5e-5)
        else:
            assert np.array_equal(f, ref), tile


@pytest.mark.parametrize("stencil", [0, 1])
def test_eq_forcing_fp32_against_oracle(orc, lbm, stencil):
    """FP32-shifted storage (the standard scheme's shift w_i rho_ref) against
    the FP64 oracle after 1000 steps, with the main step's FP32 bounds:
    rho, f < 5e-5, u < 1e-5; mass to 1e-5 relative."""
    prob = I.with_size(I.PAPER_DROPLET, 128, 96)
    steps = 1000
    p = oparams(orc, prob.physics, stencil)
    fo = orc.step(EQF, p, orc.init(EQF, p, prob.rho()), steps)
    ro, uxo, uyo, _ = orc.fields(EQF, p, fo)
    s = lbm.Solver.for_problem(prob, force_stencil=stencil, precision="fp32s")
    s.init(prob.rho(), scheme=EQF)
    s.step(steps, EQF)
    ob = s.observe()
    f32 = to_oracle(s.get_populations())
    s.close()
    e_rho = np.abs(ob["rho"] - ro).max()
    e_u = max(np.abs(ob["ux"] - uxo).max(), np.abs(ob["uy"] - uyo).max())
    e_f = np.abs(f32 - fo).max()
    print("eq forcing fp32 vs oracle, stencil %d, %d steps: rho %.3e  u %.3e  f %.3e"
          % (stencil, steps, e_rho, e_u, e_f))
    assert e_rho < 5e-5 and e_u < 1e-5 and e_f < 5e-5
    assert abs(ob["mass"] - orc.observe(EQF, p, fo)["mass"]) < 1e-5 * ob["mass"]


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_switching_between_forcing_terms(orc, lbm, prec):
    """Switching the scheme between steps keeps the populations (the two
    standard forms share the equilibrium and the FP32 shift), and the
    sequence standard -> eq forcing -> WB -> eq forcing matches the oracle."""
    prob = I.with_size(I.PAPER_DROPLET, 96, 64)
    p = oparams(orc, prob.physics)
    seq = [("standard", 40), (EQF, 60), ("well_balanced", 50), (EQF, 30)]
    fo = orc.init("standard", p, prob.rho())
    s = lbm.Solver.for_problem(prob, precision=prec)
    s.init(prob.rho(), scheme="standard")
    for sch, n in seq:
        fo = orc.step(sch, p, fo, n)
        s.step(n, sch)
    fg = to_oracle(s.get_populations())
    s.close()
    assert np.abs(fg - fo).max() <= (TOL if prec == "fp64" else 5e-5)


def test_eq_forcing_in_batches(orc, lbm):
    """Batch slots run the other forcing term too: slots of the three schemes
    in one batch (FP64 and FP32-shifted) give the populations of the same
    lattices run alone, bit for bit, and the FP64 ones match the oracle."""
    ph = I.PAPER_PHYS
    cases = [(I.with_size(I.PAPER_DROPLET, 48, 40), EQF, "fp64"),
             (I.with_size(I.PAPER_DROPLET, 70, 33), EQF, "fp32s"),
             (I.with_size(I.PAPER_DROPLET, 40, 40), "standard", "fp64"),
             (I.with_size(I.PAPER_DROPLET, 33, 50), "well_balanced", "fp64")]
    b = lbm.Batch(1 << 28, max_slots=8)
    b.set_graph_steps(10)
    slots = []
    for prob, sch, prec in cases:
        prm = lbm.make_params(prob.nx, prob.ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v,
                              precision=prec)
        slots.append(b.admit(prm, prob.rho(), sch))
    b.run(120)
    p = oparams(orc, ph, 0)
    for (prob, sch, prec), sl in zip(cases, slots):
        got = b.get_populations(sl)
        s = lbm.Solver.for_problem(prob, precision=prec)
        s.init(prob.rho(), scheme=sch)
        s.step(120, sch)
        assert np.array_equal(got, s.get_populations(), equal_nan=True), (sch, prec)
        s.close()
        if prec == "fp64":
            fo = orc.step(sch, p, orc.init(sch, p, prob.rho()), 120)
            assert np.abs(to_oracle(got) - fo).max() <= TOL, sch
    st, info = b.info(slots[0])
    b.poll()
    assert b.info(slots[0])[1]["step"] == 120
    b.close()


def test_full_grid_sampled_eq_forcing(orc, lbm):
    """The 4096^2 droplet with the Sec. IV.B constants (on which the standard
    LBE stays finite) in the benchmark's launch configuration: after 20
    steps, one more GPU step against the oracle's step on periodic crops
    around sampled windows, across strip, chunk and lattice seams (a node's
    update depends on f within 3 nodes)."""
    from paper_2012_11075_amd import tune
    prob = I.PAPER_DROPLET_4096
    p = oparams(orc, prob.physics)
    s = lbm.Solver.for_problem(prob)
    s.set_tile(*tune.bench_tile(prob.nx, prob.ny, "fp64"))
    s.init(prob.rho(), scheme=EQF)
    s.step(20, EQF)
    f = s.get_populations()
    s.step(1, EQF)
    g = s.get_populations()
    m = s.observe(fields=())
    s.close()
    assert not m["nonfinite"]
    rng = np.random.default_rng(13)
    corners = [(0, 0), (4090, 4090), (125, 509), (3071, 1021), (1023 + 1024, 2048)]
    corners += [tuple(int(v) for v in rng.integers(0, 4096, 2)) for _ in range(8)]
    W, M = 22, 3
    for (y0, x0) in corners:
        ys = np.arange(y0 - M, y0 + W - M) % 4096
        xs = np.arange(x0 - M, x0 + W - M) % 4096
        crop = to_oracle(f[:, ys][:, :, xs])
        out = orc.step(EQF, p, crop, 1)
        want = out[M:-M, M:-M]
        got = to_oracle(g[:, ys[M:-M]][:, :, xs[M:-M]])
        assert np.abs(got - want).max() <= 1e-12, (y0, x0)
