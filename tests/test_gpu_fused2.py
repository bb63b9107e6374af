"""Two steps per launch (tile depth 4: 2-D lattices, central force stencil,
128- or 256-thread blocks, in FP64 and FP32-shifted storage) through the C
ABI.  Each launch runs the first step into LDS and the second step from
there (temporal blocking), so the populations must equal those of one-step
launches bit for bit: for every scheme, ragged and tiny lattices, odd step
counts (which end with one one-step launch), graph replays whose launch
count flips the buffers, and the benchmark's 4096^2 launch configurations,
where one launch is also held against two steps of the FP64 oracle on
sampled crops."""
import numpy as np
import pytest

from paper_2012_11075_amd import inputs as I

pytestmark = pytest.mark.gpu
SCHEMES = ["well_balanced", "standard", "standard_eq_forcing"]


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_11075_amd import lbm as L
    L.load()
    return L


# the benchmark's block widths; the other one is covered by OTHER below
BLOCK = {"fp32s": 256, "fp64": 128}


def run(L, prob, scheme, tile, steps, graph_steps=0, split=3, precision="fp32s"):
    s = L.Solver.for_problem(prob, precision=precision)
    s.set_tile(*tile)
    if graph_steps:
        s.set_graph_steps(graph_steps)
    s.init(prob.rho(), scheme=scheme)
    s.step(steps - split, scheme)
    s.step(split, scheme)
    f = s.get_populations()
    ob = s.observe(fields=("rho", "ux", "uy", "mu"), raise_nonfinite=False)
    spl = s.lib.lbm_steps_per_launch(s.ctx)
    s.close()
    return f, ob, spl


# (precision, nx, ny, rows, steps, graph steps): one strip and several,
# strips that end ragged or exactly at the strip width (250 columns at 256
# threads, 122 at 128), lattices narrower than the first step's columns and
# shorter
# than a chunk, graphs of 4 (even launch count) and of 6 and 10 steps (odd
# launch count)
CASES = [("fp32s", 700, 300, 128, 40, 0), ("fp32s", 1100, 90, 32, 23, 0),
         ("fp32s", 249, 37, 16, 31, 0), ("fp32s", 250, 50, 8, 20, 0), ("fp32s", 251, 12, 4, 9, 0),
         ("fp32s", 501, 21, 8, 11, 0),
         ("fp32s", 5, 3, 4, 14, 0), ("fp32s", 33, 130, 64, 40, 10), ("fp32s", 600, 200, 96, 44, 4),
         ("fp32s", 250, 61, 20, 30, 6),
         ("fp64", 700, 300, 128, 40, 0), ("fp64", 1100, 90, 32, 23, 0), ("fp64", 249, 37, 16, 31, 0),
         ("fp64", 250, 50, 8, 20, 0), ("fp64", 251, 12, 4, 9, 0), ("fp64", 5, 3, 4, 14, 0),
         ("fp64", 121, 40, 16, 13, 0), ("fp64", 122, 33, 8, 10, 0), ("fp64", 123, 21, 4, 15, 0),
         ("fp64", 33, 130, 64, 40, 10), ("fp64", 600, 200, 96, 44, 6)]
# the other block width of each precision
OTHER = [("fp64", 700, 300, 128, 40, 0), ("fp64", 250, 50, 8, 20, 0), ("fp64", 600, 200, 96, 44, 6),
         ("fp32s", 700, 300, 128, 40, 0), ("fp32s", 122, 33, 8, 10, 0),
         ("fp32s", 600, 200, 96, 44, 4)]
ALL = [c[:1] + (BLOCK[c[0]],) + c[1:] for c in CASES] + \
      [c[:1] + (384 - BLOCK[c[0]],) + c[1:] for c in OTHER]


@pytest.mark.parametrize("case", ALL, ids=lambda c: "%s_b%d_%dx%d_r%d_n%d_g%d" % c)
def test_two_step_launch_bit_identical(lbm, case):
    prec, bw, nx, ny, rows, steps, gsteps = case
    prob = I.with_size(I.PAPER_DROPLET, nx, ny)
    for scheme in SCHEMES:
        print("two-step", case, scheme, flush=True)
        f1, o1, spl1 = run(lbm, prob, scheme, (256, rows, 3), steps, gsteps, precision=prec)
        f2, o2, spl2 = run(lbm, prob, scheme, (bw, rows, 4), steps, gsteps, precision=prec)
        assert (spl1, spl2) == (1, 2)
        assert np.array_equal(f1, f2, equal_nan=True), (case, scheme)
        for k in ("rho", "ux", "uy", "mu"):
            assert np.array_equal(o1[k], o2[k], equal_nan=True), (case, scheme, k)
        assert o1["step"] == o2["step"] == steps


@pytest.mark.parametrize("prec", ["fp32s", "fp64"])
def test_two_step_tile_rules(lbm, prec):
    """Depth 4 is accepted only for 2-D lattices with the central stencil
    and 128- or 256-thread blocks; the refused calls leave the tile as it
    was."""
    L = lbm
    prob = I.with_size(I.PAPER_DROPLET, 96, 64)
    ph = prob.physics
    bw = BLOCK[prec]
    s = L.Solver.for_problem(prob, precision=prec)
    s.set_tile(bw, 32, 4)
    assert s.get_tile() == (bw, 32, 4) and s.lib.lbm_steps_per_launch(s.ctx) == 2
    for bad in [(512, 32, 4), (64, 32, 4), (192, 32, 4), (bw, 32, 5)]:
        with pytest.raises(L.LbmError):
            s.set_tile(*bad)
    assert s.get_tile() == (bw, 32, 4)
    s.set_tile(bw, 32, 3)
    assert s.lib.lbm_steps_per_launch(s.ctx) == 1
    s.close()
    others = [L.Solver.for_problem(prob, precision=prec, force_stencil=1),
              L.Solver(24, 20, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                       precision=prec, nz=12)]
    for o in others:
        with pytest.raises(L.LbmError):
            o.set_tile(bw, 32, 4)
        assert o.lib.lbm_steps_per_launch(o.ctx) == 1
        o.close()


@pytest.mark.parametrize("prec", ["fp32s", "fp64"])
def test_two_step_checkpoint_resume(lbm, prec):
    """Populations saved after an odd number of steps and restored into a
    fresh context continue under two-step launches exactly as an
    uninterrupted run of one-step launches."""
    prob = I.with_size(I.PAPER_DROPLET, 640, 96)
    sch = "well_balanced"
    bw = BLOCK[prec]
    a = lbm.Solver.for_problem(prob, precision=prec)
    a.set_tile(bw, 24, 4)
    a.init(prob.rho(), scheme=sch)
    a.step(13, sch)
    f = a.get_populations()
    a.close()
    b = lbm.Solver.for_problem(prob, precision=prec)
    b.set_tile(bw, 24, 4)
    b.set_populations(f, scheme=sch, step=13)
    b.step(20, sch)
    got = b.get_populations()
    b.close()
    want, _, _ = run(lbm, prob, sch, (bw, 24, 3), 33, precision=prec)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("prec", ["fp32s", "fp64"])
def test_two_step_full_grid_sampled(orc, lbm, prec):
    """The benchmark's 4096^2 launch configurations (two steps per launch):
    after 20 steps, one more launch against two steps of the FP64 oracle
    from the same populations on periodic crops around sampled windows,
    including the seams of the strips (122 or 250 columns).
    FP64: 1e-11.  FP32: two steps add single-precision rounding of O(1)
    populations twice; the bound is 4e-6."""
    from paper_2012_11075_amd import tune
    prob = I.DROPLET_4096_FINITE
    ph = prob.physics
    p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    tile = tune.bench_tile(prob.nx, prob.ny, prec)
    assert tile[2] == 4, "the benchmark tile runs two steps per launch"
    s = lbm.Solver.for_problem(prob, precision=prec)
    s.set_tile(*tile)
    s.init(prob.rho(), scheme="well_balanced")
    s.step(20, "well_balanced")
    f = s.get_populations()
    s.step(2, "well_balanced")
    g = s.get_populations()
    s.close()
    rng = np.random.default_rng(5)
    corners = [(0, 0), (4090, 4090), (146, 503), (2050, 1009), (1000, 4045), (273, 248),
               (3836, 3998)]
    corners += [tuple(int(v) for v in rng.integers(0, 4096, 2)) for _ in range(5)]
    W, M = 28, 6
    worst = 0.0
    for (y0, x0) in corners:
        ys = np.arange(y0 - M, y0 + W - M) % 4096
        xs = np.arange(x0 - M, x0 + W - M) % 4096
        crop = np.ascontiguousarray(np.transpose(f[:, ys][:, :, xs], (1, 2, 0)))
        want = orc.step("well_balanced", p, crop, 2)[M:-M, M:-M]
        got = np.transpose(g[:, ys[M:-M]][:, :, xs[M:-M]], (1, 2, 0))
        worst = max(worst, np.abs(got - want).max())
    print("%s two-step error on 4096^2 crops: %.3e" % (prec, worst))
    assert worst < (4e-6 if prec == "fp32s" else 1e-11)


@pytest.mark.parametrize("prec", ["fp32s", "fp64"])
def test_two_step_degenerate_shapes(lbm, prec):
    """Lattices one node wide or tall and 2 x 2, where every pull and
    stencil wraps onto the node itself or its one neighbour: two-step
    launches equal one-step launches bit for bit."""
    ph = I.PAPER_PHYS
    rng = np.random.default_rng(17)
    bw = BLOCK[prec]
    for nx, ny in [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5)]:
        rho = 0.6 + 0.05 * rng.uniform(-1, 1, (ny, nx))
        out = []
        for depth in (3, 4):
            s = lbm.Solver(nx, ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                           precision=prec)
            s.set_tile(bw, 4, depth)
            s.init(rho, scheme="well_balanced")
            s.step(9, "well_balanced")
            out.append(s.get_populations())
            s.close()
        print("two-step degenerate", prec, nx, ny, flush=True)
        assert np.array_equal(out[0], out[1], equal_nan=True), (prec, nx, ny)
