"""Batched and served execution of the force-stencil variant (the
fourth-order gradients of the force discussed after Eq. 23) through the C
ABI.  A force-stencil slot runs the variant's own kernel code over the batch
table, so it gives the populations of the same lattice run alone, bit for
bit (FP64 and FP32-shifted, the three schemes, depths 1 to 3, mixed with
central-stencil slots, with and without graphs); its FP64 populations match
the oracle to 1e-11, and the poll observes it as lbm_observe does."""
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


def params_of(L, prob, precision, stencil):
    ph = prob.physics
    return L.make_params(prob.nx, prob.ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                         precision=precision, force_stencil=stencil)


def alone(L, prob, precision, scheme, steps, stencil, tile):
    s = L.Solver.for_problem(prob, precision=precision, force_stencil=stencil)
    s.set_tile(*tile)
    s.init(prob.rho(), scheme=scheme)
    s.step(steps, scheme)
    f = s.get_populations()
    ob = s.observe(fields=(), raise_nonfinite=False)
    s.close()
    return f, ob


# (problem, precision, scheme, force stencil, tile)
CASES = [
    (I.with_size(I.PAPER_DROPLET, 48, 40), "fp64", "well_balanced", 1, (256, 16, 1)),
    (I.with_size(I.PAPER_DROPLET, 70, 33), "fp32s", "well_balanced", 1, (256, 32, 2)),
    (I.with_size(I.PAPER_DROPLET, 300, 21), "fp64", "standard", 1, (256, 8, 3)),
    (I.with_size(I.PAPER_DROPLET, 40, 64), "fp64", EQF, 1, (256, 32, 2)),
    (I.with_size(I.PAPER_DROPLET, 5, 3), "fp64", "well_balanced", 1, (256, 4, 1)),
    (I.with_size(I.PAPER_DROPLET, 257, 19), "fp32s", "standard", 1, (256, 8, 1)),
    (I.with_size(I.PAPER_DROPLET, 64, 48), "fp64", "well_balanced", 0, (128, 32, 2)),
    (I.with_size(I.PAPER_DROPLET, 33, 50), "fp32s", EQF, 0, (64, 16, 3)),
]


@pytest.mark.parametrize("graph_steps", [0, 10])
def test_stencil4_slots_alone_vs_batch(orc, lbm, graph_steps):
    steps = 120
    b = lbm.Batch(1 << 28, max_slots=16)
    b.set_graph_steps(graph_steps)
    slots = []
    for prob, prec, sch, st, tile in CASES:
        sl = b.admit(params_of(lbm, prob, prec, st), prob.rho(), sch)
        b.set_tile(sl, *tile)
        slots.append(sl)
    b.run(steps - 7)
    b.run(7)
    b.poll()
    for (prob, prec, sch, st, tile), sl in zip(CASES, slots):
        print("force stencil %d slot" % st, prob.nx, prob.ny, prec, sch, tile, flush=True)
        got = b.get_populations(sl)
        want, ob = alone(lbm, prob, prec, sch, steps, st, tile)
        assert np.array_equal(got, want, equal_nan=True), (prob.nx, prob.ny, prec, sch, st)
        info = b.info(sl)[1]
        assert info["step"] == steps
        assert np.array_equal([info["max_u"], info["mass"], info["kinetic_energy"]],
                              [ob["max_u"], ob["mass"], ob["kinetic_energy"]], equal_nan=True)
        if prec == "fp64" and st == 1:
            ph = prob.physics
            p = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0, 1)
            fo = orc.step(sch, p, orc.init(sch, p, prob.rho()), steps)
            assert np.abs(np.transpose(got, (1, 2, 0)) - fo).max() <= TOL, (prob.nx, sch)
    b.close()


def test_stencil4_slot_tile_width(lbm):
    """Force-stencil slots run 256-wide blocks; other widths are refused
    and the slot keeps running."""
    prob = I.with_size(I.PAPER_DROPLET, 40, 30)
    b = lbm.Batch(1 << 26, max_slots=4)
    sl = b.admit(params_of(lbm, prob, "fp64", 1), prob.rho(), "well_balanced")
    for bad in [(64, 16, 1), (128, 16, 1), (512, 16, 1)]:
        with pytest.raises(lbm.LbmError):
            b.set_tile(sl, *bad)
    b.set_tile(sl, 256, 16, 3)
    b.run(20)
    want, _ = alone(lbm, prob, "fp64", "well_balanced", 20, 1, (256, 16, 3))
    assert np.array_equal(b.get_populations(sl), want)
    b.close()


@pytest.mark.parametrize("tuned", [False, True])
def test_served_stencil4_requests_equal_alone(lbm, tuned):
    """A served stream in which every third request uses the fourth-order
    force stencil: each result equals the same request run alone, with the
    default tiles and with the served stream's table (whose two-step FP32
    tiles the variant's requests take at one step per launch)."""
    from dataclasses import replace
    from paper_2012_11075_amd import tune
    from paper_2012_11075_amd.serve import BatchExecutor, Server
    reqs = I.request_stream(9, rate_hz=400.0, seed=41, side_lo=32, side_hi=200, step_cap=400,
                            fp64_fraction=0.5)
    reqs = [replace(r, force_stencil=1) if r.rid % 3 == 1 else r for r in reqs]
    ex = BatchExecutor(int(2e9), max_slots=16, graph_steps=10, capture=True,
                       tiles=(lambda nx, ny, prec: tune.serve_tile(nx, ny, prec)) if tuned else None)
    srv = Server(ex, k=100)
    out = srv.serve(reqs)
    ex.close()
    assert sorted(o.rid for o in out) == list(range(len(reqs)))
    for o in out:
        req = reqs[o.rid]
        ph = req.problem.physics
        s = lbm.Solver(req.problem.nx, req.problem.ny, ph.tau, ph.beta, ph.kappa, ph.rho_l,
                       ph.rho_v, ph.rho0, precision=req.precision, force_stencil=req.force_stencil)
        s.set_tile(256 if req.force_stencil else 0, 0, 0)
        s.init(req.problem.rho(), scheme=req.scheme)
        s.step(o.steps, req.scheme)
        f = s.get_populations()
        s.close()
        assert np.array_equal(f, o.result["populations"], equal_nan=True), (o.rid, o.status)
