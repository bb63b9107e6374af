"""3-D lattices (D3Q19 and D3Q27) in batches, through the C ABI.  A 3-D slot
runs the fused 3-D step over the batch's table, so it gives the populations
of the same lattice run alone, bit for bit (FP64 and FP32-shifted, the three
schemes, depths 1 and 2, mixed with 2-D slots, with and without graphs);
FP64 slots match the oracle to 1e-11; the poll observes a 3-D slot as
lbm_observe does and retires it by its criterion; a served stream of 3-D and
2-D requests gives each request the result of running it alone."""
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


PH = I.PAPER_PHYS


def rho3(nx, ny, nz, seed):
    return I.droplet3_density(nx, ny, nz, PH, 0.3 * min(nx, ny, nz) + 1.0, 4.0, 1e-2, seed=seed)


def params3(L, nx, ny, nz, prec, q):
    return L.make_params(nx, ny, PH.tau, PH.beta, PH.kappa, PH.rho_l, PH.rho_v, PH.rho0,
                         precision=prec, nz=nz, q3=q)


def alone3(L, nx, ny, nz, prec, q, scheme, steps, tile, rho):
    s = L.Solver(nx, ny, PH.tau, PH.beta, PH.kappa, PH.rho_l, PH.rho_v, PH.rho0, precision=prec,
                 nz=nz, q3=q)
    s.set_tile(*tile)
    s.init(rho, scheme=scheme)
    s.step(steps, scheme)
    f = s.get_populations()
    ob = s.observe(fields=(), raise_nonfinite=False)
    s.close()
    return f, ob


# (nx, ny, nz, precision, q, scheme, tile)
CASES = [(16, 12, 10, "fp64", 19, "well_balanced", (256, 4, 1)),
         (33, 9, 5, "fp32s", 19, "standard", (256, 3, 2)),
         (20, 14, 9, "fp64", 27, "well_balanced", (256, 0, 2)),
         (5, 2, 6, "fp64", 27, EQF, (256, 2, 1)),
         (40, 24, 16, "fp32s", 27, "well_balanced", (256, 5, 1)),
         (12, 10, 8, "fp64", 19, EQF, (256, 8, 2))]


@pytest.mark.parametrize("graph_steps", [0, 10])
def test_3d_slots_alone_vs_batch(orc, lbm, graph_steps):
    steps = 60
    b = lbm.Batch(1 << 28, max_slots=16)
    b.set_graph_steps(graph_steps)
    slots, rhos = [], []
    for k, (nx, ny, nz, prec, q, sch, tile) in enumerate(CASES):
        rho = rho3(nx, ny, nz, seed=k + 3)
        sl = b.admit(params3(lbm, nx, ny, nz, prec, q), rho, sch)
        b.set_tile(sl, *tile)
        slots.append(sl)
        rhos.append(rho)
    # a 2-D slot in the same batch
    p2 = I.with_size(I.PAPER_DROPLET, 48, 40)
    s2 = b.admit(lbm.make_params(48, 40, PH.tau, PH.beta, PH.kappa, PH.rho_l, PH.rho_v, PH.rho0),
                 p2.rho(), "well_balanced")
    b.run(steps - 7)
    b.run(7)
    b.poll()
    for (nx, ny, nz, prec, q, sch, tile), sl, rho in zip(CASES, slots, rhos):
        print("3-D slot", nx, ny, nz, prec, q, sch, tile, flush=True)
        got = b.get_populations(sl)
        assert got.shape == (q, nz, ny, nx)
        want, ob = alone3(lbm, nx, ny, nz, prec, q, sch, steps, tile, rho)
        assert np.array_equal(got, want, equal_nan=True), (nx, ny, nz, prec, q, sch)
        st, info = b.info(sl)
        assert st == "active" and info["step"] == steps
        assert np.array_equal([info["max_u"], info["mass"], info["kinetic_energy"]],
                              [ob["max_u"], ob["mass"], ob["kinetic_energy"]], equal_nan=True)
        if prec == "fp64":
            p = orc.Params(PH.tau, PH.beta, PH.kappa, PH.rho_l, PH.rho_v, PH.rho0)
            fo = orc.step3(sch, p, orc.init3(sch, p, rho, q=q), steps)
            assert np.abs(np.moveaxis(got, 0, -1) - fo).max() <= TOL, (nx, ny, nz, q, sch)
    s = lbm.Solver.for_problem(p2)
    s.init(p2.rho(), scheme="well_balanced")
    s.step(steps, "well_balanced")
    assert np.array_equal(b.get_populations(s2), s.get_populations())
    s.close()
    b.close()


def test_3d_slot_tiles_and_retirement(lbm):
    """3-D slots take 256-thread tiles with depth 1 or 2 only; a 3-D slot
    with a loose tolerance retires at the first poll and a capped one at its
    cap, while another keeps running."""
    b = lbm.Batch(1 << 27, max_slots=4)
    a = b.admit(params3(lbm, 16, 12, 10, "fp64", 19), rho3(16, 12, 10, 1), "well_balanced",
                tol=1.0)
    c = b.admit(params3(lbm, 16, 12, 10, "fp64", 27), rho3(16, 12, 10, 2), "well_balanced",
                step_cap=20)
    d = b.admit(params3(lbm, 12, 10, 8, "fp32s", 19), rho3(12, 10, 8, 3), "standard")
    for bad in [(512, 4, 1), (256, 4, 3), (128, 4, 1)]:
        with pytest.raises(lbm.LbmError):
            b.set_tile(c, *bad)
    b.run(20)
    retired = sorted(b.poll())
    assert retired == sorted([a, c])
    assert b.info(a)[0] == "converged" and b.info(c)[0] == "capped"
    assert b.info(d)[0] == "active"
    b.run(10)
    assert b.poll() == [] and b.info(d)[1]["step"] == 30
    b.close()


def test_served_3d_requests_equal_alone(lbm):
    """A served stream of 3-D requests (D3Q19 and D3Q27, FP64 and
    FP32-shifted) mixed with 2-D ones: every result equals the same request
    run alone for the same number of steps, bit for bit."""
    from dataclasses import replace
    from paper_2012_11075_amd.serve import BatchExecutor, Server
    reqs = I.request_stream3(6, rate_hz=400.0, seed=9, side_lo=12, side_hi=48, step_cap=300)
    reqs += [replace(r, rid=r.rid + 6) for r in
             I.request_stream(3, rate_hz=400.0, seed=10, side_lo=32, side_hi=96, step_cap=300)]
    assert {r.problem.q3 for r in reqs[:6]} == {19, 27}
    ex = BatchExecutor(int(2e9), max_slots=16, graph_steps=10, capture=True)
    srv = Server(ex, k=100)
    out = srv.serve(reqs)
    ex.close()
    assert sorted(o.rid for o in out) == list(range(len(reqs)))
    for o in out:
        req = reqs[o.rid]
        ph, pr = req.problem.physics, req.problem
        print("served", o.rid, type(pr).__name__, pr.nx, getattr(pr, "q3", 9), req.precision,
              o.status, o.steps, flush=True)
        if hasattr(pr, "nz"):
            s = lbm.Solver(pr.nx, pr.ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                           precision=req.precision, nz=pr.nz, q3=pr.q3)
            assert o.nodes == pr.nx * pr.ny * pr.nz
        else:
            s = lbm.Solver.for_problem(pr, precision=req.precision)
        s.init(pr.rho(), scheme=req.scheme)
        s.step(o.steps, req.scheme)
        f = s.get_populations()
        s.close()
        assert np.array_equal(f, o.result["populations"], equal_nan=True), (o.rid, o.status)
