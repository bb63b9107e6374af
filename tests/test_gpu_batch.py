"""Batched execution of many uneven lattices (lbm_batch_* through the C ABI).

Every slot runs the same kernel code as a single lattice, so a lattice must
give bit-identical populations alone and inside a batch (NaN-for-NaN where a
configuration diverges); FP64 slots must match the oracle to 1e-11.
"""
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


def params_of(L, prob, precision):
    ph = prob.physics
    return L.make_params(prob.nx, prob.ny, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                         precision=precision)


def alone(L, prob, precision, scheme, steps):
    s = L.Solver.for_problem(prob, precision=precision)
    s.init(prob.rho(), scheme=scheme)
    s.step(steps, scheme)
    f = s.get_populations()
    s.close()
    return f


def mix_cases():
    probs = [p for p in I.batch_instances(64, seed=4, side_lo=16, side_hi=300)][:14]
    probs.append(I.with_size(I.PAPER_DROPLET, 7, 5))
    probs.append(I.with_size(I.PAPER_DROPLET, 129, 3))
    out = []
    for k, p in enumerate(probs):
        out.append((p, "fp64" if k % 2 == 0 else "fp32s",
                    "standard" if k % 5 == 3 else "well_balanced"))
    return out


@pytest.mark.parametrize("graph_steps", [0, 16])
def test_alone_vs_mix_bit_exact(lbm, graph_steps):
    cases = mix_cases()
    steps = 150
    need = sum(lbm.Batch.slot_bytes(params_of(lbm, p, prec)) for p, prec, _ in cases)
    arena = need + lbm.Batch.overhead_bytes(need * 2, 64) + (1 << 20)
    b = lbm.Batch(arena, max_slots=64)
    b.set_graph_steps(graph_steps)
    slots = [b.admit(params_of(lbm, p, prec), p.rho(), scheme) for p, prec, scheme in cases]
    b.run(steps - 7)
    b.run(7)
    for (p, prec, scheme), sl in zip(cases, slots):
        print("batch slot", sl, p.name, p.nx, p.ny, prec, scheme, flush=True)
        got = b.get_populations(sl)
        want = alone(lbm, p, prec, scheme, steps)
        assert np.array_equal(got, want, equal_nan=True), (p.name, prec, scheme)
    b.close()


BATCH_TILES = [(64, 8, 1), (128, 16, 2), (256, 32, 3), (64, 33, 3), (128, 5, 1), (256, 64, 2),
               (64, 128, 2), (128, 32, 3)]


def test_batch_tiles_bit_exact(lbm):
    """Slots of one batch on every batched block width and depth (several
    launch groups at once) give the populations of
    the lattice run alone."""
    cases = mix_cases()
    steps = 40
    need = sum(lbm.Batch.slot_bytes(params_of(lbm, p, prec)) for p, prec, _ in cases)
    b = lbm.Batch(need + lbm.Batch.overhead_bytes(need * 2, 64) + (1 << 20), max_slots=64)
    b.set_graph_steps(10)
    slots = []
    for k, (p, prec, scheme) in enumerate(cases):
        sl = b.admit(params_of(lbm, p, prec), p.rho(), scheme)
        b.set_tile(sl, *BATCH_TILES[k % len(BATCH_TILES)])
        slots.append(sl)
    b.run(steps - 5)
    b.run(5)
    for k, ((p, prec, scheme), sl) in enumerate(zip(cases, slots)):
        print("batch tile", BATCH_TILES[k % len(BATCH_TILES)], p.name, p.nx, p.ny, prec, scheme,
              flush=True)
        assert np.array_equal(b.get_populations(sl), alone(lbm, p, prec, scheme, steps),
                              equal_nan=True), (p.name, prec, scheme)
    b.close()


def test_batch_fp64_slots_match_oracle(orc, lbm):
    probs = [I.with_size(I.PAPER_DROPLET, 64, 48), I.with_size(I.PAPER_DROPLET, 33, 70),
             I.PAPER_FLAT]
    b = lbm.Batch(1 << 28, max_slots=8)
    slots = [b.admit(params_of(lbm, p, "fp64"), p.rho(), s)
             for p, s in zip(probs, ["well_balanced", "standard", "well_balanced"])]
    b.run(300)
    for p, s, sl in zip(probs, ["well_balanced", "standard", "well_balanced"], slots):
        ph = p.physics
        op = orc.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
        fo = orc.step(s, op, orc.init(s, op, p.rho()), 300)
        fg = np.ascontiguousarray(np.transpose(b.get_populations(sl), (1, 2, 0)))
        assert np.abs(fg - fo).max() <= 1e-11
        ob = b.fetch(sl)
        assert ob["step"] == 300
        oo = orc.observe(s, op, fo)
        np.testing.assert_allclose(ob["momentum"], oo["momentum"], rtol=0, atol=1e-11 * oo["mass"])
    # the poll's per-slot scalars come from the batched observe launch and its
    # fixed-order finish; they agree with the single-lattice observe of fetch
    b.poll()
    for sl in slots:
        st, info = b.info(sl)
        ob = b.fetch(sl, fields=())
        assert info["step"] == ob["step"] == 300
        for k in ("max_u", "mass", "kinetic_energy"):
            assert abs(info[k] - ob[k]) <= 1e-12 * max(1.0, abs(ob[k])), (k, info[k], ob[k])
        np.testing.assert_allclose(info["momentum"], ob["momentum"], rtol=0, atol=1e-12 * ob["mass"])
    b.close()


def test_admission_retirement_and_reuse(lbm):
    flat = I.with_size(I.PAPER_DROPLET, 40, 40)
    pr = params_of(lbm, flat, "fp64")
    one = lbm.Batch.slot_bytes(pr)
    arena = 2 * one + lbm.Batch.overhead_bytes(4 * one, 4) + 4096
    b = lbm.Batch(arena, max_slots=4)
    uniform = np.full((40, 40), 0.6)
    s_conv = b.admit(pr, uniform, "well_balanced", tol=1e-12)       # at rest: converges at once
    s_cap = b.admit(pr, flat.rho(), "well_balanced", tol=1e-30, step_cap=20)
    assert b.try_admit(pr, flat.rho()) is None                       # arena full
    b.run(10)
    retired = b.poll()
    assert retired == [s_conv]
    assert b.info(s_conv)[0] == "converged"
    b.run(10)                                                        # only s_cap advances
    assert b.poll() == [s_cap]
    st, ob = b.info(s_cap)
    assert st == "capped" and ob["step"] == 20
    assert b.fetch(s_conv)["step"] == 10
    b.release(s_conv)
    bad = I.with_size(I.DROPLET_512_RATIO100, 40, 40)
    s_div = b.admit(params_of(lbm, bad, "fp64"), bad.rho(), "standard")
    b.run(60)
    assert b.poll() == [s_div]
    assert b.info(s_div)[0] == "diverged"
    b.release(s_div)
    b.release(s_cap)
    s2 = b.admit(pr, flat.rho(), "well_balanced")
    b.run(33)
    assert np.array_equal(b.get_populations(s2), alone(lbm, flat, "fp64", "well_balanced", 33))
    b.close()


def test_lanes_with_graphs_release_and_admit(lbm):
    """One launch group with slots in both lanes (even and odd slot index),
    captured graphs of 8 steps and odd step counts: releasing a slot of one
    lane and admitting another (that lane's table and graph change, the
    other's do not) leaves every lattice bit-identical to its run alone."""
    probs = [I.with_size(I.PAPER_DROPLET, n, n + 3) for n in (40, 57, 33, 64, 29, 48)]
    extra = I.with_size(I.PAPER_DROPLET, 51, 38)
    prec, scheme = "fp32s", "well_balanced"
    need = sum(lbm.Batch.slot_bytes(params_of(lbm, p, prec)) for p in probs + [extra])
    b = lbm.Batch(need + lbm.Batch.overhead_bytes(need * 2, 16) + (1 << 20), max_slots=16)
    b.set_graph_steps(8)
    slots = [b.admit(params_of(lbm, p, prec), p.rho(), scheme) for p in probs]
    b.run(21)
    b.release(slots[3])
    s_new = b.admit(params_of(lbm, extra, prec), extra.rho(), scheme)
    b.run(13)
    for k, (p, sl) in enumerate(zip(probs, slots)):
        if k == 3:
            continue
        print("lane test slot", sl, p.nx, p.ny, flush=True)
        assert np.array_equal(b.get_populations(sl), alone(lbm, p, prec, scheme, 34)), p.name
    assert np.array_equal(b.get_populations(s_new), alone(lbm, extra, prec, scheme, 13))
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_full_batch_sampled(lbm, prec):
    """The benchmark's batched configuration (the 512 uneven lattices, tuned
    tiles, two lanes, graphs of 50 steps): after 60 steps, sampled slots of
    both lanes and all size ranges hold the populations of the same lattice
    run alone, bit for bit (NaN for NaN where a lattice diverges)."""
    from paper_2012_11075_amd import tune
    probs = I.batch_instances(512)
    prms = [params_of(lbm, p, prec) for p in probs]
    need = sum(lbm.Batch.slot_bytes(q) for q in prms)
    b = lbm.Batch(need + lbm.Batch.overhead_bytes(2 * need, len(probs)) + (1 << 24),
                  max_slots=len(probs))
    b.set_graph_steps(50)
    slots = []
    for q, p in zip(prms, probs):
        sl = b.admit(q, p.rho(), "well_balanced")
        t = tune.batch_tile(p.nx, p.ny, prec)
        if t:
            b.set_tile(sl, *t)
        slots.append(sl)
    b.run(60)
    order = sorted(range(len(probs)), key=lambda k: probs[k].nx)
    picks = sorted(set([order[0], order[1], order[len(order) // 2], order[-2], order[-1], 7, 300]))
    for k in picks:
        p = probs[k]
        print("full batch slot", k, p.nx, p.ny, prec, flush=True)
        assert np.array_equal(b.get_populations(slots[k]), alone(lbm, p, prec, "well_balanced", 60),
                              equal_nan=True), (k, p.nx)
    b.close()
