"""Throughput benchmark of the D2Q9 two-phase LBE step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 4096 x 4096 periodic droplet (radius 1024, density ratio 100,
beta = 0.1, kappa = 0.02, tau = 0.8), well-balanced scheme, populations in
FP64 (the headline line) and in the shifted FP32 form (reported beside it).
These constants make the interface 1.3 nodes wide and the state diverges
within ~100 steps (in the CPU oracle as well); the step kernel's work does not
depend on the values, and the same grid with the free-energy constants of
Sec. IV, whose state stays finite, is timed beside it (finite_state) with the
FP32 errors against FP64 at full size.
A step is one launch of the fused step kernel over the whole lattice; the
populations stay in HBM for the whole timed region.  Beside it: 512 batched
uneven lattices (5,000 steps, FP32-shifted and FP64), a served stream of
run-to-equilibrium requests (p50/p99 latency, aggregate MLUPS) and the FP64
CPU oracle on a bounded sample.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BYTES_PER_UPDATE = {"fp64": 144, "fp32s": 72}   # 9 populations read + written
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ["lbm_kernels.hip", "lbm_kernels.h"]:
        with open(os.path.join(ROOT, "paper_2012_11075_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(PROFILE_DIR, "step_droplet_4096.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    e = d.get(precision)
    return None if e is None else round(e.get("bytes_per_launch"))


def time_gpu(prob, precision, steps, warmup, scheme="well_balanced", fields=False):
    import torch
    from paper_2012_11075_amd import lbm, tune
    s = lbm.Solver.for_problem(prob, precision=precision)
    s.set_tile(*tune.bench_tile(prob.nx, prob.ny, precision))
    rho0 = prob.rho()
    torch.cuda.synchronize()
    t_init = time.perf_counter()
    s.init(rho0, scheme=scheme)          # host density -> device populations
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    s.step(warmup, scheme)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps, scheme)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    t_obs = time.perf_counter()
    ob = s.observe(fields=("rho", "ux", "uy", "mu"), raise_nonfinite=False)   # device -> host fields
    t_obs = time.perf_counter() - t_obs
    tile = s.get_tile()
    kps = s.lib.lbm_kernels_per_step(s.ctx)
    spl = s.lib.lbm_steps_per_launch(s.ctx)
    s.close()
    del s
    torch.cuda.empty_cache()
    nodes = prob.nx * prob.ny
    ms_step = ms / steps
    mlups = nodes * steps / (ms / 1e3) / 1e6
    # a launch reads and writes every population once and advances the state
    # `spl` steps (2 with two steps per launch): its algorithmic bytes are
    # BYTES_PER_UPDATE x nodes over spl steps' time
    bpu = BYTES_PER_UPDATE[precision]
    per_launch = bpu * nodes
    launch_ms = ms_step * spl / kps
    achieved = per_launch / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(precision)
    return {
        "mlups": mlups,
        "ms_per_step": ms_step,
        "wall_s": wall,
        "tile": list(tile),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_update": bpu / spl, "steps_per_launch": spl,
                     # the HBM rate a kernel moving every population once per step
                     # would need for the same step rate (above `peak` when spl = 2)
                     "one_step_traffic_gbs": round(bpu * nodes / (ms_step / 1e3) / 1e9, 1)},
        "state_after": {"step": ob["step"], "max_u": ob["max_u"], "nonfinite": ob["nonfinite"]},
        "observation": ob if fields else None,
        # the whole job through the host boundary: density in over PCIe, the
        # timed steps, and rho, u, mu back (context only, never the value)
        "host_io": {"init_s": round(t_init, 4), "observe_fields_s": round(t_obs, 4),
                    "pcie_inclusive_mlups": round(nodes * steps / (t_init + ms / 1e3 + t_obs) / 1e6, 1)},
    }


def time_batch(precision, steps, warmup, count=512, graph_steps=50):
    """Batched uneven instances: `count` lattices (side log-uniform 32..512,
    droplet or slab, density ratio 10 or 100, tau in [0.6, 1.2]) advanced
    together for `steps` steps of the WB scheme.  Slots retire only at the
    poll after the timed region, so every lattice is advanced every step;
    the poll's count of diverged lattices is split at tau = 0.8, below which
    the WB step has a growing mode in bulk liquid.  Slots on two-step tiles
    (depth 4 in the tuned table) advance two steps per launch; the rate
    counts the algorithmic bytes of one step per node and step."""
    import torch
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import lbm, tune
    probs = I.batch_instances(count)
    prms = [lbm.make_params(p.nx, p.ny, p.physics.tau, p.physics.beta, p.physics.kappa,
                            p.physics.rho_l, p.physics.rho_v, precision=precision) for p in probs]
    need = sum(lbm.Batch.slot_bytes(q) for q in prms)
    arena = need + lbm.Batch.overhead_bytes(2 * need, count) + (1 << 24)
    b = lbm.Batch(arena, max_slots=count)
    b.set_graph_steps(graph_steps)
    tau_of = {}
    two_step = 0
    for q, p in zip(prms, probs):
        sl = b.admit(q, p.rho(), "well_balanced")
        tau_of[sl] = p.physics.tau
        t = tune.batch_tile(p.nx, p.ny, precision)
        if t:
            b.set_tile(sl, *t)
            two_step += t[2] == 4
    b.run(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    retired = b.poll()
    status = {}
    for sl in retired:
        st = b.info(sl)[0]
        if st == "diverged":
            st = "diverged_tau_lt_0.8" if tau_of[sl] < 0.8 else "diverged_tau_ge_0.8"
        status[st] = status.get(st, 0) + 1
    b.close()
    del b
    torch.cuda.empty_cache()
    nodes = sum(p.nx * p.ny for p in probs)
    bpu = BYTES_PER_UPDATE[precision]
    gbs = bpu * nodes * steps / (ms / 1e3) / 1e9
    return {"value": round(nodes * steps / (ms / 1e3) / 1e6, 1), "unit": "MLUPS",
            "instances": count, "total_nodes": nodes, "steps": steps,
            "ms_per_step": round(ms / steps, 5), "hbm_gbs_algorithmic": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_update": bpu,
            "graph_steps": graph_steps, "two_step_slots": two_step,
            "retired_at_end": status,
            "active_at_end": count - len(retired)}


def serve_stream(n_requests=100, rate_hz=None, arena_gb=8.0, k=250):
    """Served stream: Poisson arrivals of run-to-equilibrium requests (side
    log-uniform 64..2048, density ratio 10..1000, FP32-shifted by default and
    FP64 for one request in ten), continuous batching over one arena."""
    import torch
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import tune
    from paper_2012_11075_amd.serve import BatchExecutor, Server, summarise
    if rate_hz is None:
        # offered load ~0.7 of a ~60 GLUPS device at the mean request size and cap
        mean_nodes = (2048 ** 2 - 64 ** 2) / (2 * math.log(2048 / 64))
        rate_hz = 0.7 * 60e9 / (mean_nodes * 50_000)
    reqs = I.request_stream(n_requests, rate_hz)
    ex = BatchExecutor(int(arena_gb * 1e9), max_slots=256, graph_steps=50,
                       tiles=lambda nx, ny, prec: tune.serve_tile(nx, ny, prec))
    srv = Server(ex, k=k)
    t0 = time.perf_counter()
    out = srv.serve(reqs)
    wall = time.perf_counter() - t0
    ex.close()
    torch.cuda.empty_cache()
    s = summarise(out, wall)
    s.update(rate_hz=round(rate_hz, 4), steps_per_round=k, arena_bytes=int(arena_gb * 1e9),
             max_concurrent=max(sum(1 for e in srv.log[:i + 1] if e[0] == "admit") -
                                sum(1 for e in srv.log[:i + 1] if e[0] == "retire")
                                for i in range(len(srv.log))))
    for key in ("p50_latency_s", "p99_latency_s", "mean_latency_s", "aggregate_mlups", "wall_s",
                "converged_fraction"):
        s[key] = round(s[key], 4)
    for v in s["by_outcome"].values():
        for key in ("p50_latency_s", "p99_latency_s", "mean_latency_s"):
            v[key] = round(v[key], 4)
    return s


def fp32_errors(steps=20_000):
    """FP32-shifted against FP64 on the 256^2 droplet (ratio 10, tau 1, WB,
    20,000 steps): max|u|, bulk densities and the Laplace pressure jump
    (the FP64 path matches the CPU oracle to 1e-11 in the parity tests)."""
    import numpy as np
    from paper_2012_11075_amd import diagnostics as D
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import lbm
    prob = I.DROPLET_256
    ph = prob.physics
    reads = {}
    for prec in ("fp64", "fp32s"):
        s = lbm.Solver.for_problem(prob, precision=prec)
        s.set_graph_steps(100)
        s.init(prob.rho(), scheme="well_balanced")
        s.step(steps, "well_balanced")
        ob = s.observe(fields=("rho", "ux", "uy"))
        s.close()
        r = D.droplet_reads(ob["rho"], ph.beta, ph.rho_l, ph.rho_v)
        r["max_u"] = ob["max_u"]
        r["mass"] = ob["mass"]
        reads[prec] = (r, ob)
    cmp_ = D.compare(reads["fp64"][0], reads["fp32s"][0])
    drho = float(np.abs(reads["fp32s"][1]["rho"] - reads["fp64"][1]["rho"]).max())
    return {"workload": "droplet_256 (256x256, R=64, ratio 10, tau 1), WB, %d steps" % steps,
            "reads": {k: {kk: (float("%.6g" % vv) if isinstance(vv, float) and vv is not None else vv)
                          for kk, vv in v.items()} for k, v in cmp_.items()},
            "max_abs_rho_field_err": drho}


def finite_state(steps, warmup):
    """The same 4096^2 droplet with the free-energy constants of Sec. IV
    (interface 3.2 nodes wide), whose state stays finite: the FP64 and
    FP32-shifted rates on a finite state, and the FP32 errors at full size
    against the FP64 path (max|u|, bulk densities, Laplace pressure jump)."""
    import numpy as np
    from paper_2012_11075_amd import diagnostics as D
    from paper_2012_11075_amd import inputs as I
    prob = I.DROPLET_4096_FINITE
    ph = prob.physics
    res, reads = {}, {}
    for prec in ("fp64", "fp32s"):
        r = time_gpu(prob, prec, steps, warmup, fields=True)
        ob = r.pop("observation")
        rd = D.droplet_reads(ob["rho"], ph.beta, ph.rho_l, ph.rho_v)
        rd["max_u"], rd["mass"] = ob["max_u"], ob["mass"]
        reads[prec] = (rd, ob["rho"])
        res[prec] = {"value": round(r["mlups"], 1), "unit": "MLUPS",
                     "ms_per_step": round(r["ms_per_step"], 5), "hbm_frac": r["roofline"]["frac"],
                     "state_after": r["state_after"]}
    cmp_ = D.compare(reads["fp64"][0], reads["fp32s"][0])
    res["fp32_error_vs_fp64"] = {
        "reads": {k: {kk: (float("%.6g" % vv) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in cmp_.items()},
        "max_abs_rho_field_err": float(np.abs(reads["fp32s"][1] - reads["fp64"][1]).max())}
    res["workload"] = ("droplet_4096_finite: 4096x4096, R=1024, rho_l=1, rho_v=0.01, beta=0.01, "
                       "kappa=0.0128, tau=0.8, tanh width %.3f, WB, %d steps after %d warm-up"
                       % (prob.width, steps, warmup))
    return res


STENCIL4_BYTES = 144   # FP64 bytes per node of the variant step: 9 populations read and written


def time_stencil4(prob, steps, warmup, scheme="standard", tile=None, precision="fp64",
                  force_stencil=1):
    """A variant of the 2-D step: by default the force-stencil variant
    (fourth-order gradients in the force); with force_stencil=0 the main
    step, e.g. under the standard_eq_forcing scheme.  One fused pass per
    step, 9 populations read and written = 144 (FP64) or 72 (FP32-shifted)
    algorithmic bytes per node.  `tile` (block, rows, depth) overrides the
    default."""
    import torch
    from paper_2012_11075_amd import lbm
    s = lbm.Solver.for_problem(prob, force_stencil=force_stencil, precision=precision)
    if tile:
        s.set_tile(*tile)
    s.init(prob.rho(), scheme=scheme)
    s.step(warmup, scheme)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps, scheme)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kps = s.lib.lbm_kernels_per_step(s.ctx)
    spl = s.lib.lbm_steps_per_launch(s.ctx)
    used = s.get_tile()
    ob = s.observe(fields=(), raise_nonfinite=False)
    s.close()
    del s
    torch.cuda.empty_cache()
    nodes = prob.nx * prob.ny
    # HBM bytes per node update: one read and one write of every population
    # per launch, a launch advancing spl steps
    bpu = (STENCIL4_BYTES // 2 if precision == "fp32s" else STENCIL4_BYTES) // spl
    gbs = bpu * nodes / (ms / 1e3) / 1e9
    return {"value": round(nodes / (ms / 1e3) / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(ms, 5),
            "scheme": scheme, "precision": precision, "kernels_per_step": kps, "tile": list(used),
            "bytes_per_update": bpu, "steps_per_launch": spl,
            "state_after": {"step": ob["step"], "max_u": ob["max_u"], "nonfinite": ob["nonfinite"]},
            "hbm_gbs_algorithmic": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "workload": "%s, %s scheme, %s force stencil, %s, %d steps"
                        % (prob.name, scheme, "fourth-order" if force_stencil else "central",
                           precision.upper(), steps)}


def time_largest(steps, warmup, n=32768):
    """The FP64 WB step on the largest square lattice HBM holds in FP64
    (32768^2, a 189 GB workspace), with the two-step tile that
    tune.two_step_tile picks for its size, on a separable density (Sec. IV
    constants, density ratio 5): the rate at 64x the headline's node
    count."""
    import ctypes
    import gc
    import torch
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import lbm, tune
    ph = I.PAPER_PHYS
    prm = lbm.make_params(n, n, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    need = lbm.load().lbm_workspace_bytes(ctypes.byref(prm))
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need + (2 << 30):
        return {"skipped": "needs %.0f GB of free device memory, %.0f GB free"
                           % (need / 1e9, free / 1e9)}
    rho = I.separable_density(n, n, 17)
    s = lbm.Solver(n, n, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    s.set_tile(*(tune.two_step_tile(n, n, "fp64") or tune.bench_tile(4096, 4096, "fp64")))
    s.init(rho, scheme="well_balanced")
    del rho
    s.step(warmup, "well_balanced")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps, "well_balanced")
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ob = s.observe(fields=(), raise_nonfinite=False)
    used = s.get_tile()
    spl = s.lib.lbm_steps_per_launch(s.ctx)
    s.close()
    del s
    gc.collect()
    torch.cuda.empty_cache()
    nodes = n * n
    # one read and one write of every population per launch of spl steps
    bpu = 144 // spl
    gbs = bpu * nodes / (ms / 1e3) / 1e9
    return {"value": round(nodes / (ms / 1e3) / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(ms, 4),
            "nx": n, "ny": n, "workspace_gb": round(need / 1e9, 1), "tile": list(used),
            "bytes_per_update": bpu, "steps_per_launch": spl, "hbm_gbs_algorithmic": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "state_after": {"step": ob["step"], "max_u": ob["max_u"], "nonfinite": ob["nonfinite"]},
            "workload": "%d^2 separable density, Sec. IV constants (ratio 5), WB, FP64, %d steps "
                        "after %d" % (n, steps, warmup)}


def time_d3(steps, warmup, side=None, tile=None, precision="fp64", q=19):
    """The 3-D WB step on a side^3 droplet on the D3Q19 (q = 19) or D3Q27
    (q = 27) lattice: one fused pass per step, q populations read and written
    = 16 q algorithmic bytes per node in FP64 (304 for D3Q19, 432 for D3Q27),
    8 q in FP32-shifted storage.  `tile` (block threads, planes per chunk)
    overrides the default."""
    import torch
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import lbm
    n = side or I.DROPLET3_SIDE
    ph = I.PHYS3
    rho = I.droplet3_density(n, n, n, ph, I.DROPLET3_RADIUS * n / I.DROPLET3_SIDE,
                             I.equilibrium_width(ph), 1e-3, seed=13)
    s = lbm.Solver(n, n, ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, nz=n, precision=precision,
                   q3=q)
    if tile:
        s.set_tile(*tile)
    s.init(rho, scheme="well_balanced")
    del rho
    s.step(warmup, "well_balanced")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps, "well_balanced")
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ob = s.observe(fields=(), raise_nonfinite=False)
    kps = s.lib.lbm_kernels_per_step(s.ctx)
    used = s.get_tile()
    s.close()
    del s
    torch.cuda.empty_cache()
    nodes = n ** 3
    bpu = (8 if precision == "fp32s" else 16) * q
    gbs = bpu * nodes / (ms / 1e3) / 1e9
    return {"value": round(nodes / (ms / 1e3) / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(ms, 5),
            "precision": precision, "kernels_per_step": kps, "bytes_per_update": bpu,
            "tile": list(used),
            "hbm_gbs_algorithmic": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "state_after": {"step": ob["step"], "max_u": ob["max_u"], "nonfinite": ob["nonfinite"]},
            "workload": "D3Q%d droplet %d^3, R=%g, rho_l=1, rho_v=0.1, beta=0.01, kappa=0.0128, "
                        "tau=1, WB, %s, %d steps" % (q, n, I.DROPLET3_RADIUS * n / I.DROPLET3_SIDE,
                                                     precision.upper(), steps)}


def copy_reference(nx, ny):
    """The step's traffic without its arithmetic: `hbm_ceiling` (built next to
    the library) streams the nine population rows of every lattice row from
    one buffer to another in the same layout, FP64 and FP32, and times a
    plain vectorised copy.  Run as a child process before this process uses
    the GPU."""
    exe = os.path.join(ROOT, "paper_2012_11075_amd", "_lib", "hbm_ceiling")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe, str(nx), str(ny), "20"], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return {"error": (r.stderr or r.stdout).strip()[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, budget_s=15.0):
    """The FP64 oracle on the same lattice for a bounded number of steps, on
    up to 16 host threads (OpenMP over rows) and on one thread."""
    import oracle
    oracle.build()
    ph = prob.physics
    p = oracle.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
    threads = min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    f = oracle.init("well_balanced", p, prob.rho())
    t0 = time.perf_counter()
    f = oracle.step("well_balanced", p, f, 1)
    t1 = time.perf_counter() - t0
    k = max(1, min(30, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    f = oracle.step("well_balanced", p, f, k)
    dt = time.perf_counter() - t0
    nodes = prob.nx * prob.ny
    used = oracle.get_threads()
    oracle.set_threads(1)
    t0 = time.perf_counter()
    f = oracle.step("well_balanced", p, f, 1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": round(nodes * k / dt / 1e6, 3), "unit": "MLUPS", "cores": used,
            "kind": "oracle",
            "sample": "%dx%d %s lattice, %d WB steps after one warm-up step, FP64, %d threads"
                      % (prob.nx, prob.ny, prob.name, k, used),
            "single_thread_mlups": round(nodes / dt1 / 1e6, 3),
            "single_thread_sample": "1 WB step of the same lattice on one thread",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def full_runs():
    """The 200x4 flat interface (10,000 steps) and the 256^2 droplet (20,000
    steps) in full with the WB scheme: wall time on the GPU (HIP-graph
    captured steps, 100 per graph, after 100 warm-up steps) and of the FP64
    oracle on up to 16 host threads, from the same initial state."""
    import torch
    import oracle
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import lbm
    out = {}
    for prob in (I.FLAT_200x4, I.DROPLET_256):
        rho = prob.rho()
        s = lbm.Solver.for_problem(prob)
        s.set_graph_steps(100)
        s.init(rho, scheme="well_balanced")
        s.step(100, "well_balanced")
        s.init(rho, scheme="well_balanced")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(prob.steps, "well_balanced")
        torch.cuda.synchronize()
        gpu_s = time.perf_counter() - t0
        g = s.observe(fields=(), raise_nonfinite=False)
        s.close()
        ph = prob.physics
        p = oracle.Params(ph.tau, ph.beta, ph.kappa, ph.rho_l, ph.rho_v, ph.rho0)
        oracle.set_threads(min(16, os.cpu_count() or 1))
        f = oracle.init("well_balanced", p, rho)
        t0 = time.perf_counter()
        f = oracle.step("well_balanced", p, f, prob.steps)
        cpu_s = time.perf_counter() - t0
        o = oracle.observe("well_balanced", p, f)
        upd = prob.nx * prob.ny * prob.steps
        out[prob.name] = {"steps": prob.steps, "gpu_s": round(gpu_s, 4),
                          "gpu_mlups": round(upd / gpu_s / 1e6, 1),
                          "oracle_s": round(cpu_s, 3), "oracle_mlups": round(upd / cpu_s / 1e6, 2),
                          "oracle_threads": oracle.get_threads(),
                          "max_u": {"gpu": g["max_u"], "oracle": o["max_u"]}}
    return out


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-finite", action="store_true")
    ap.add_argument("--no-stencil4", action="store_true")
    ap.add_argument("--no-eq-forcing", action="store_true")
    ap.add_argument("--no-largest", action="store_true")
    ap.add_argument("--no-d3", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--serve-requests", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the step runs on a single device "
              "(multi-GPU decomposition is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    from paper_2012_11075_amd import inputs as I
    from paper_2012_11075_amd import tune
    prob = I.DROPLET_4096
    ref = copy_reference(prob.nx, prob.ny)
    progress("copy reference %s" % ref)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    r64 = time_gpu(prob, "fp64", args.steps, args.warmup)
    progress("fp64 headline %.4f ms/step" % r64["ms_per_step"])
    out = {
        "metric": "MLUPS (million lattice-node updates per second), FP64 well-balanced step",
        "value": round(r64["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "droplet_4096: 4096x4096 periodic D2Q9 lattice, droplet R=1024, "
                               "rho_l=1, rho_v=0.01, beta=0.1, kappa=0.02, tau=0.8, "
                               "well-balanced scheme",
                   "nx": prob.nx, "ny": prob.ny, "scheme": "well_balanced",
                   "tile": r64["tile"], "kernels_per_step": 1},
        "roofline": r64["roofline"],
        "state_after": r64["state_after"],
        "host_io": r64["host_io"],
        # the same bytes moved with no arithmetic: the practical ceiling for
        # this traffic (frac_* = the step's algorithmic GB/s over it)
        "copy_reference": None if not ref or "error" in ref else dict(
            ref, frac_fp64=round(r64["roofline"]["achieved"] / ref["rows_copy_fp64_gbs"], 4)),
        "note": "with these constants the interface is 1.3 nodes wide and the step (the FP64 "
                "CPU oracle too) diverges within ~100 steps; the kernel does the same work "
                "on any values, and finite_state times the same grid on a finite state",
    }
    if not args.no_fp32:
        r32 = time_gpu(prob, "fp32s", args.steps, args.warmup)
        progress("fp32s %.4f ms/step" % r32["ms_per_step"])
        if out["copy_reference"]:
            out["copy_reference"]["frac_fp32"] = round(
                r32["roofline"]["achieved"] / out["copy_reference"]["rows_copy_fp32_gbs"], 4)
        out["fp32_shifted"] = {"value": round(r32["mlups"], 1), "unit": "MLUPS",
                               "ms_per_step": round(r32["ms_per_step"], 5),
                               "tile": r32["tile"], "roofline": r32["roofline"],
                               "state_after": r32["state_after"]}
    if not args.no_fp32:
        out["fp32_shifted"]["error_vs_fp64"] = fp32_errors()
        progress("fp32 errors on droplet_256 done")
    if not args.no_finite:
        out["finite_state"] = finite_state(args.steps, args.warmup)
        progress("finite-state companion done")
    # A freshly started process runs its first launches into a dip of the core
    # clock (power management after an idle device: 2.27 -> 1.8 GHz over
    # launches 4-25 at 4096^2), 10-25% slower than the steady rate; each
    # entry below warms up 150 steps past it (the headline takes --warmup
    # steps and times --steps).
    if not args.no_stencil4:
        # on the finite-state droplet: at density ratio 100 the standard
        # scheme diverges within a few steps, so the WB step is timed
        out["force_stencil4"] = time_stencil4(I.DROPLET_4096_FINITE, 500, 150, "well_balanced",
                                              tile=tune.stencil4_tile(prob.nx, prob.ny, "fp64"))
        out["force_stencil4"]["fp32_shifted"] = time_stencil4(
            I.DROPLET_4096_FINITE, 500, 150, "well_balanced",
            tile=tune.stencil4_tile(prob.nx, prob.ny, "fp32s"), precision="fp32s")
        progress("force-stencil variant %.4f ms/step" % out["force_stencil4"]["ms_per_step"])
    if not args.no_eq_forcing:
        # the standard LBE with the forcing term named after Eq. (5), on the
        # 4096^2 droplet with the Sec. IV.B constants (the standard LBE goes
        # to negative densities within a few steps at density ratio 100)
        pd = I.PAPER_DROPLET_4096
        out["standard_eq_forcing"] = time_stencil4(
            pd, 400, 150, "standard_eq_forcing", tile=tune.bench_tile(pd.nx, pd.ny, "fp64"),
            force_stencil=0)
        out["standard_eq_forcing"]["fp32_shifted"] = time_stencil4(
            pd, 400, 150, "standard_eq_forcing", tile=tune.bench_tile(pd.nx, pd.ny, "fp32s"),
            precision="fp32s", force_stencil=0)
        out["standard_eq_forcing"]["eq5_same_grid"] = time_stencil4(
            pd, 400, 150, "standard", tile=tune.bench_tile(pd.nx, pd.ny, "fp64"), force_stencil=0)
        progress("standard LBE, eq-proportional forcing %.4f ms/step"
                 % out["standard_eq_forcing"]["ms_per_step"])
    if not args.no_largest:
        out["largest_lattice"] = time_largest(100, 100)
        progress("largest lattice %s" % out["largest_lattice"].get("ms_per_step",
                                                                   out["largest_lattice"]))
    if not args.no_d3:
        for q in (19, 27):
            key = "d3q%d" % q
            out[key] = time_d3(100, 50, q=q)
            out[key]["fp32_shifted"] = time_d3(100, 50, precision="fp32s", q=q)
            progress("D3Q%d %.4f ms/step (FP32 %.4f)" % (q, out[key]["ms_per_step"],
                                                         out[key]["fp32_shifted"]["ms_per_step"]))
    if not args.no_batch:
        out["batched"] = {}
        for prec in ("fp32s", "fp64"):
            out["batched"][prec] = time_batch(prec, args.batch_steps, 200)
            progress("batched %s %.4f ms/step" % (prec, out["batched"][prec]["ms_per_step"]))
    if not args.no_serve:
        out["served"] = serve_stream(args.serve_requests)
        progress("served stream done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
        progress("cpu baseline done")
        out["cpu_baseline"]["full_runs"] = full_runs()
        progress("full 200x4 and 256^2 runs done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
