"""Two steps per launch inside batches (slot tile depth 4 through
lbm_batch_set_tile, the C ABI): a slot's populations equal those of the
lattice run alone with one-step launches, bit for bit (NaN for NaN where a
configuration diverges), for both precisions and every scheme, next to
slots of one-step tiles in the same batch, with odd step counts (which end
with one one-step launch), and with captured graphs whose two-step launch
count per replay is even (4 steps) or odd (6 and 10 steps, where
consecutive replays alternate in parity)."""
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


def cases():
    """(problem, precision, scheme, tile): uneven lattices from 1 node to
    several strips wide, most on two-step tiles of both block widths and
    several chunk heights, every fourth on a one-step tile."""
    probs = I.batch_instances(64, seed=9, side_lo=8, side_hi=600)[:12]
    probs += [I.with_size(I.PAPER_DROPLET, nx, ny) for nx, ny in
              [(1, 7), (7, 1), (507, 12), (251, 40), (2, 2), (300, 251)]]
    rows = [4, 16, 37, 64, 9]
    out = []
    for k, p in enumerate(probs):
        prec = "fp64" if k % 2 == 0 else "fp32s"
        bw = 128 if k % 3 else 256
        tile = (bw, rows[k % len(rows)], 4) if k % 4 != 3 else (128, 16, 2)
        out.append((p, prec, SCHEMES[k % 3], tile))
    return out


def make_batch(L, cs, graph_steps):
    need = sum(L.Batch.slot_bytes(params_of(L, p, prec)) for p, prec, _, _ in cs)
    b = L.Batch(need + L.Batch.overhead_bytes(need * 2, 64) + (1 << 20), max_slots=64)
    b.set_graph_steps(graph_steps)
    slots = []
    for p, prec, scheme, tile in cs:
        sl = b.admit(params_of(L, p, prec), p.rho(), scheme)
        b.set_tile(sl, *tile)
        slots.append(sl)
    return b, slots


@pytest.mark.parametrize("graph_steps", [0, 4, 6, 10])
def test_batch_two_step_bit_exact(lbm, graph_steps):
    cs = cases()
    b, slots = make_batch(lbm, cs, graph_steps)
    runs = [13, 6, 1, 22]
    for k in runs:
        b.run(k)
    steps = sum(runs)
    for (p, prec, scheme, tile), sl in zip(cs, slots):
        print("batch two-step slot", sl, p.nx, p.ny, prec, scheme, tile, graph_steps, flush=True)
        got = b.get_populations(sl)
        assert np.array_equal(got, alone(lbm, p, prec, scheme, steps), equal_nan=True), \
            (p.nx, p.ny, prec, scheme, tile)
    b.close()


def test_batch_two_step_poll_observations(lbm):
    """The poll observes slots of two-step tiles with the one-step table's
    batched observe launch: its per-slot scalars agree with the
    single-lattice observe of fetch."""
    cs = cases()
    b, slots = make_batch(lbm, cs, 8)
    b.run(35)
    retired = set(b.poll())
    checked = 0
    for (p, prec, scheme, tile), sl in zip(cs, slots):
        st, info = b.info(sl)
        if st == "diverged":
            assert sl in retired
            continue
        ob = b.fetch(sl, fields=())
        assert info["step"] == ob["step"] == 35
        for k in ("max_u", "mass", "kinetic_energy"):
            assert abs(info[k] - ob[k]) <= 1e-12 * max(1.0, abs(ob[k])), (sl, k, info[k], ob[k])
        checked += 1
    assert checked >= len(cs) // 2
    b.close()


def test_batch_two_step_tile_rules_and_switch(lbm):
    """Depth 4 needs a 2-D central-stencil slot and block 128 or 256; block
    512 is refused for batched tiles of any depth.  A slot switched
    between two-step and one-step tiles between runs stays bit-identical
    to its run alone."""
    L = lbm
    p = I.with_size(I.PAPER_DROPLET, 300, 70)
    q = I.with_size(I.PAPER_DROPLET, 90, 41)
    need = 4 * L.Batch.slot_bytes(params_of(L, p, "fp64"))
    b = L.Batch(need + L.Batch.overhead_bytes(need * 2, 8) + (1 << 20), max_slots=8)
    s64 = b.admit(params_of(L, p, "fp64"), p.rho(), "well_balanced")
    s32 = b.admit(params_of(L, q, "fp32s"), q.rho(), "standard")
    ph = p.physics
    s4 = b.admit(L.make_params(64, 40, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0,
                               force_stencil=1), I.with_size(I.PAPER_DROPLET, 64, 40).rho())
    for sl, bad in [(s64, (512, 16, 4)), (s64, (64, 16, 4)), (s32, (512, 16, 4)),
                    (s32, (512, 16, 3)), (s32, (192, 16, 4)), (s4, (256, 16, 4)),
                    (s4, (128, 16, 4))]:
        with pytest.raises(L.LbmError):
            b.set_tile(sl, *bad)
    b.release(s4)
    b.set_graph_steps(6)
    b.set_tile(s64, 128, 24, 4)
    b.set_tile(s32, 256, 8, 4)
    b.run(17)
    b.set_tile(s64, 256, 16, 3)
    b.run(9)
    b.set_tile(s64, 256, 40, 4)
    b.set_tile(s32, 128, 20, 4)
    b.run(7)
    b.set_tile(s64, 128, 40, 4)
    b.set_tile(s32, 128, 16, 2)
    b.run(12)
    assert np.array_equal(b.get_populations(s64), alone(L, p, "fp64", "well_balanced", 45))
    assert np.array_equal(b.get_populations(s32), alone(L, q, "fp32s", "standard", 45))
    b.close()
