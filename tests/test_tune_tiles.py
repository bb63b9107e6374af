"""Tile tables and the two-step tile helper (paper_2012_11075_amd/tune.py),
on the CPU: the benchmark's 4096^2 tiles run two steps per launch and fill
one round of blocks (two per compute unit: 128-thread blocks in FP64,
256-thread blocks in FP32-shifted storage); the helper reproduces them,
fills whole rounds of
blocks on other sizes and leaves lattices too small for the device to one
step per launch."""
import math

from paper_2012_11075_amd import tune


def tiles_of(nx, ny, tile):
    block, rows, depth = tile
    assert depth == 4
    return math.ceil(nx / (block - 6)) * math.ceil(ny / rows)


RESIDENT = {"fp64": 512, "fp32s": 512}
BLOCK = {"fp64": 128, "fp32s": 256}


def test_bench_tiles_two_steps_per_launch():
    assert tune.bench_tile(4096, 4096, "fp64") == (128, 274, 4)
    assert tune.bench_tile(4096, 4096, "fp32s") == (256, 137, 4)
    for prec in ("fp64", "fp32s"):
        r = RESIDENT[prec]
        assert 0.93 * r <= tiles_of(4096, 4096, tune.bench_tile(4096, 4096, prec)) <= r


def test_two_step_helper_matches_the_measured_tiles():
    for prec in ("fp64", "fp32s"):
        assert tune.two_step_tile(4096, 4096, prec) == tune.bench_tile(4096, 4096, prec)


def test_two_step_helper_rounds_and_limits():
    for n in (2048, 8192, 32768):
        for prec in ("fp64", "fp32s"):
            t = tune.two_step_tile(n, n, prec)
            assert t is not None and t[0] == BLOCK[prec]
            assert 16 <= t[1] <= 512
            k = tiles_of(n, n, t)
            r = RESIDENT[prec]
            rounds = math.ceil(k / r)
            # no round is less than about half full
            assert k > (rounds - 1) * r + r // 2 or rounds == 1, (n, prec, t, k)
    assert tune.two_step_tile(512, 512, "fp64") is None
    assert tune.two_step_tile(1024, 1024, "fp32s") is None
    assert tune.two_step_tile(1024, 1024, "fp64") == (128, 19, 4)
