#!/usr/bin/env python3
"""Throughput of the nested-grid PM step on one MI355X.

Workload (the one the metric is quoted on): the disc-bulge-halo galaxy on
3 nested 128^3 grids (half-extents 1, 4, 20; inner two flattened to q = 1/4),
8.5M particles (2M disc, 0.5M bulge, 6M halo), FP32 with FP64 diagnostics
every 10 steps, dt = 0.01.  One step = loss test and centre of mass, mass
assignment, the 5 isolated 128^3 solves, Eq. 8 forces with the
grid-selection rule, kick and drift.

Prints one JSON line: particle-steps/s of the FP32 form (value), the FP64 form
on the same workload, standalone batched 128^3 solves/s in both precisions,
per-phase GPU times from HIP events recorded on the library's stream during
the timed region, the roofline of the dominant kernel, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FFT_PASSES = ("fwd_x", "fwd_y", "zpass", "inv_y", "inv_x")


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def phase_bytes(phase, N, nsolves, n_live, esz, form=5):
    """Algorithmic HBM bytes of one launch of a phase (the data it must read
    and write once): FFT passes per the pruned layout, particle kernels per
    the SoA fields they touch.  form 3 (plane-fused solves): the plane
    forward pass is timed as fwd_x, the plane inverse as inv_y, and the
    x-transformed planes never reach memory."""
    cplx = 2 * esz
    cells = N ** 3
    X = (N + 1) * N * N * cplx       # half spectrum after the x pass
    Cb = (N + 1) * 2 * N * N * cplx  # after the y pass (z < N kept)
    H = (N + 1) ** 3 * esz
    if form == 3:
        per_solve = {"fwd_x": cells * esz + Cb, "fwd_y": 0, "zpass": 2 * Cb + H,
                     "inv_y": Cb + cells * esz, "inv_x": 0}
    else:
        per_solve = {
            "fwd_x": cells * esz + X,
            "fwd_y": X + Cb,
            "zpass": 2 * Cb + H,
            "inv_y": Cb + X,
            "inv_x": X + cells * esz,
        }
    if phase in per_solve:
        return per_solve[phase] * nsolves
    grids = nsolves * cells * esz
    if phase == "zero":
        return grids
    if phase == "pre":      # x, m, gal, lost
        return n_live * (4 * esz + 2)
    if phase == "deposit":  # x, m, gal, lost read; grids written once
        return n_live * (4 * esz + 2) + grids
    if phase == "force":    # x, v, gal, lost read; x, v written; fields read once
        return n_live * (12 * esz + 2) + grids
    return 0


def fft_form(report, esz, N, count):
    """The form (3 or 5) the tuner chose for count solves of N^3 grids, from
    the tuning report of the library (5 when the mix was never planned)."""
    tag = f"{'fp64' if esz == 8 else 'fp32'} N={N} x{count} form="
    for line in report.splitlines():
        if line.startswith(tag):
            return int(line[len(tag):].split()[0])
    return 5


KERNEL_SOURCES = ["paper_1210_1736_amd/csrc/particles.hip", "paper_1210_1736_amd/csrc/particles.h",
                  "paper_1210_1736_amd/csrc/common.h", "paper_1210_1736_amd/csrc/fft.hip",
                  "paper_1210_1736_amd/csrc/fft.h"]
PROFILE = "profiles/step_kernels_disc_galaxy_3x128_fp32.md"
PHASE_KERNEL = {"deposit": "k_deposit<float, false>", "force": "k_force<float, 1>", "pre": "k_pre<float>"}


def measured_traffic(phase):
    """HBM bytes per launch of the phase's kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        text = open(os.path.join(ROOT, PROFILE)).read()
    except OSError:
        return None
    if f"Kernel-source hash: {h.hexdigest()[:16]}" not in text or phase not in PHASE_KERNEL:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip("|").split("|")]
        if len(cells) == 5 and cells[0] == PHASE_KERNEL[phase]:
            return float(cells[4]) * 1e6
    return None


def time_solves(sbx, torch, N, R, q, prec, batch, iters):
    dt = torch.float64 if prec == sbx.SBX_FP64 else torch.float32
    g = torch.Generator(device="cuda").manual_seed(1736)
    rho = torch.rand((batch, N, N, N), dtype=dt, device="cuda", generator=g)
    phi = torch.empty_like(rho)
    stream = torch.cuda.current_stream()
    p = sbx.Poisson(N, R, q, prec=prec, stream=stream.cuda_stream)
    for _ in range(3):
        p.sbx_poisson_solve(batch, rho.data_ptr(), phi.data_ptr())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(iters):
        p.sbx_poisson_solve(batch, rho.data_ptr(), phi.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    p.close()
    del rho, phi
    return batch / (ms * 1e-3), ms


def make_ctx(sbx, w, prec, merge=False):
    from paper_1210_1736_amd import sbx as S
    cent = {"com": S.SBX_CENTRE_COM, "fixed": S.SBX_CENTRE_FIXED, "density": S.SBX_CENTRE_DENSITY}
    hs = [S.make_hierarchy([(L.N, L.R, L.q) for L in h.levels], cent[h.centring], h.centre,
                           h.outer_centre) for h in w.hier]
    ctx = S.Context(prec=prec, G=w.G)
    if merge:
        ctx.sbx_set_outer_merge(1)
    ctx.sbx_build_grids(hs)
    ctx.sbx_load_particles(w.x, w.v, w.m, w.comp, w.gal)
    return ctx


def timed_steps(sbx, torch, w, prec, steps, warmup, diag_every, profile=True, sort_every=None,
                merge=False, fixed=False):
    ctx = make_ctx(sbx, w, prec, merge)
    if sort_every is not None:
        ctx.sbx_set_sort_interval(sort_every)
    if fixed:
        ctx.sbx_set_deterministic_deposit(1)
    ctx.sbx_step(w.dt, warmup, diag_every)
    ctx.sbx_sync()
    live0 = ctx.sbx_count_live()
    torch.cuda.synchronize()
    ctx.sbx_sync()
    t0 = time.perf_counter()
    ctx.sbx_step(w.dt, steps, diag_every)
    ctx.sbx_sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    live1 = ctx.sbx_count_live()
    phases = {}
    if profile:
        # phase times from a second pass of the same length with an event
        # after every phase (the events themselves cost time, so the timed
        # pass above runs without them)
        ctx.sbx_profile_begin(64 * (steps + 2))
        ctx.sbx_step(w.dt, steps, diag_every)
        phases = ctx.sbx_profile_end()
    ctx.close()
    return t1 - t0, 0.5 * (live0 + live1), phases


def precision_errors(sbx, w):
    """Force and potential error of the FP32 form at the initial state of the
    workload, against the FP64 form (which the parity tests hold within 1e-9
    of the FP64 oracle): per-particle |a32 - a64| over rms|a64|, and
    max|phi32 - phi64| over max|phi64|."""
    import dataclasses
    out = {}
    res = {}
    # both forms start from the same (FP32-representable) inputs, so that
    # cells and classes agree and only the arithmetic differs
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    w = dataclasses.replace(w, x=f32(w.x), v=f32(w.v), m=f32(w.m))
    for name, prec in (("fp64", sbx.SBX_FP64), ("fp32", sbx.SBX_FP32)):
        ctx = make_ctx(sbx, w, prec)
        res[name] = ctx.sbx_compute_forces()
        ctx.close()
    a64, p64 = res["fp64"]
    a32, p32 = res["fp32"]
    rms = float(np.sqrt(np.mean(np.sum(a64 * a64, axis=1))))
    e = np.linalg.norm(a32 - a64, axis=1) / rms
    out["reference"] = ("FP64 GPU form on the same FP32-rounded inputs (transitive: the parity "
                        "tests hold the FP64 form within 1e-9 of the FP64 oracle's forces, and the "
                        "FP32 form against the oracle directly at the FP32 bars)")
    out["force_rel_p99"] = float(np.percentile(e, 99))
    out["force_rel_max"] = float(e.max())
    out["pot_rel_max"] = float(np.abs(p32 - p64).max() / np.abs(p64).max())
    return out


def galaxy_satellite_rate(sbx, torch, steps, warmup):
    """Galaxy plus satellite: two 3-level hierarchies, 10 solves per step, and
    9 with the two grids 5 merged into one solve."""
    import synth
    w = synth.galaxy_satellite()
    t, live, _ = timed_steps(sbx, torch, w, sbx.SBX_FP32, steps, warmup, 10, profile=False)
    tm, livem, _ = timed_steps(sbx, torch, w, sbx.SBX_FP32, steps, warmup, 10, profile=False,
                               merge=True)
    return {"workload": "disc galaxy + Plummer satellite (200k, M 0.1), two 3-level 128^3 "
                        "hierarchies, FP32, diagnostics every 10 steps",
            "particles_live": live, "solves_per_step": 10, "steps": steps,
            "particle_steps_per_s": live * steps / t, "ms_per_step": 1e3 * t / steps,
            "merged_grid5": {"solves_per_step": 9, "ms_per_step": 1e3 * tm / steps,
                             "particle_steps_per_s": livem * steps / tm}}


def density_centring_rate(sbx, torch, w, steps, warmup, diag_every):
    """The main workload with the inner and middle grids on the galaxy's
    density maximum instead of its centre of mass."""
    import copy
    wd = copy.deepcopy(w)
    wd.hier[0].centring = "density"
    t, live, ph = timed_steps(sbx, torch, wd, sbx.SBX_FP32, steps, warmup, diag_every)
    return {"workload": "the FP32 disc-galaxy step with density-maximum centring",
            "steps": steps, "particles_live": live, "ms_per_step": 1e3 * t / steps,
            "particle_steps_per_s": live * steps / t,
            "centring_ms_per_step": ph["pre"][0] / steps if "pre" in ph else None}


def fixed_point_rate(sbx, torch, w, steps, warmup, diag_every):
    """The main workload with the fixed-point (bit-reproducible) mass
    assignment: exact 64-bit integer cell sums and one conversion pass."""
    t, live, ph = timed_steps(sbx, torch, w, sbx.SBX_FP32, steps, warmup, diag_every, fixed=True)
    return {"workload": "the FP32 disc-galaxy step with the fixed-point mass assignment",
            "steps": steps, "particles_live": live, "ms_per_step": 1e3 * t / steps,
            "particle_steps_per_s": live * steps / t,
            "deposit_ms_per_step": ph["deposit"][0] / steps if "deposit" in ph else None}


def heating_experiment(sbx, torch, w, steps=400, every=100):
    """The reduced isolated-disc heating sweep (N in {64, 128}, q in {1,
    0.5, 0.25}) on the benchmark galaxy, FP32, diagnostics every `every`
    steps."""
    from paper_1210_1736_amd import heating
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = heating.sweep(w.x, w.v, w.m, w.comp, w.gal, steps=steps, every=every, dt=w.dt, G=w.G)
    t1 = time.perf_counter()
    rows = []
    for r in runs:
        if "skipped" in r:
            rows.append({"N": r["N"], "q": r["q"], "skipped": r["skipped"]})
            continue
        rows.append({"N": r["N"], "q": r["q"], "ms_per_step": 1e3 * r["steps_s"] / r["steps"],
                     "e_heat": [r["e_heat"][0], r["e_heat"][-1]],
                     "heating_rate_rel": r["heating_rate_rel"],
                     "sig_z": [r["sig_z"][0], r["sig_z"][-1]],
                     "rms_z": [r["rms_z"][0], r["rms_z"][-1]]})
    return {"workload": f"disc galaxy in isolation, {steps} steps of dt {w.dt} per configuration, "
                        "grids (N, 1, q), (N, 4, q), (N, 20, 1)",
            "configs": rows, "wall_s": t1 - t0}


def ensemble_rate(sbx, torch, steps, warmup):
    """16 independent galaxy + satellite instances of uneven size stepped as
    one batch (one graph replay per step)."""
    import synth
    ws = synth.ensemble()
    ctxs = [make_ctx(sbx, w, sbx.SBX_FP32) for w in ws]
    b = sbx.Batch(ctxs)
    b.sbx_batch_step(0.01, warmup)
    b.sbx_batch_sync()
    live0 = sum(c.sbx_count_live() for c in ctxs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sbx_batch_step(0.01, steps)
    b.sbx_batch_sync()
    t1 = time.perf_counter()
    live1 = sum(c.sbx_count_live() for c in ctxs)
    sizes = [w.hier[0].levels[0].N for w in ws]
    b.close()
    for c in ctxs:
        c.close()
    live = 0.5 * (live0 + live1)
    return {"workload": "16 galaxy + satellite instances, grids " +
                        ", ".join(f"{sizes.count(N)} x {N}^3" for N in sorted(set(sizes))) +
                        f", {sum(w.n for w in ws)} particles, FP32",
            "instances": len(ws), "solves_per_step": 10 * len(ws), "steps": steps,
            "particles_live": live, "particle_steps_per_s": live * steps / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / steps}


def adjoint_rate(sbx, torch):
    """Differentiable segment: 10 steps forward and the reverse mode with
    checkpoints every 2 steps, gradients for every particle."""
    import synth
    w = synth.adjoint_segment()
    ctx = make_ctx(sbx, w, sbx.SBX_FP32)
    ctx.sbx_step(w.dt, 1)
    ctx.sbx_sync()
    t0 = time.perf_counter()
    ctx.sbx_step(w.dt, w.steps)
    ctx.sbx_sync()
    t1 = time.perf_counter()
    ctx.sbx_adjoint_segment(w.dt, w.steps, 2, synth.DISC, 0)   # allocations, first use
    # gradients into device memory (the inputs are resident, so are the outputs)
    gm = torch.empty(w.n, dtype=torch.float64, device="cuda")
    gx = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
    gv = torch.empty_like(gx)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    loss = ctx.sbx_adjoint_segment_device(w.dt, w.steps, 2, synth.DISC, 0, gm.data_ptr(),
                                          gx.data_ptr(), gv.data_ptr())
    t3 = time.perf_counter()
    _, hm, hx, hv = ctx.sbx_adjoint_segment(w.dt, w.steps, 2, synth.DISC, 0)
    t4 = time.perf_counter()
    ctx.close()
    return {"workload": "one 256^3 grid, 1M disc + 1M halo + 50k satellite, FP32, 10 steps, "
                        "checkpoints every 2 steps, loss = disc vertical kinetic energy",
            "particles": w.n, "forward_s": t1 - t0, "segment_s": t3 - t2,
            "segment_over_forward": (t3 - t2) / (t1 - t0),
            "includes": "forward with checkpoints, recomputation, reverse cycles; gradients "
                        "left in device memory",
            "segment_with_host_copies_s": t4 - t3,
            "loss": loss, "grad_finite": bool(torch.isfinite(gm).all() and torch.isfinite(gx).all())}


def disc_analysis_rate(sbx, torch, w):
    """The paper's disc diagnostics on the benchmark galaxy (2M disc
    particles): 100 equal-number radial bins, heat, dispersions and the
    vertical profile near R = 3.2."""
    ctx = make_ctx(sbx, w, sbx.SBX_FP32)
    ctx.sbx_step(w.dt, 1)
    ctx.sbx_disc_analysis(100, (3.0, 3.4), 40, 1.0)
    ctx.sbx_sync()
    t0 = time.perf_counter()
    out = ctx.sbx_disc_analysis(100, (3.0, 3.4), 40, 1.0)
    t1 = time.perf_counter()
    ctx.close()
    return {"ms": 1e3 * (t1 - t0), "n_disc": out["n_disc"], "e_heat": out["e_heat"],
            "sig_z_over_sig_R": out["sig_z"] / out["sig_R"] if out["sig_R"] > 0 else None,
            "includes": "selection, stable radix sort of the radii, bins, heat, annulus, "
                        "allocations and host copies"}


def cpu_threads():
    """Threads the CPU baseline may use: the process's thread budget
    (OMP_NUM_THREADS) when set, else the usable cores, at most 16 (a
    one-GPU host's share of the CPU)."""
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return env or min(aff, 16)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_CPU_STATE = {}   # inherited by the forked workers of the CPU baseline


def _eq8_chunk(bounds):
    a, b = bounds
    st = _CPU_STATE
    return st["sysm"].field_at(st["x"][a:b], st["centres"], st["pots"])[0]


def oracle_parallel_step(sysm, x, v, m, gal, lost, dt, cores):
    """One integration cycle of the oracle, as System.step computes it and in
    its order (loss test, centres, the five solves per galaxy with the FFT on
    `cores` threads, Eq. 8 with the selection rule, leapfrog, loss test), the
    per-particle Eq. 8 phase split over `cores` forked processes (each
    particle's force depends only on its position and the fields).  Returns
    new (x, v, lost, acc)."""
    import multiprocessing as mp
    from oracle import pm_oracle as O
    x = x.copy(); v = v.copy(); lost = lost.copy()
    lost |= sysm.lost_now(x)
    centres = sysm.centres(x, m, gal, lost)
    pots = sysm.potentials(x, m, gal, lost, centres)
    live = np.flatnonzero(~lost)
    _CPU_STATE.update(sysm=sysm, x=x[live], centres=centres, pots=pots)
    cuts = np.linspace(0, live.size, 4 * cores + 1).astype(int)
    with mp.get_context("fork").Pool(cores) as pool:
        parts = pool.map(_eq8_chunk, list(zip(cuts[:-1], cuts[1:])))
    _CPU_STATE.clear()
    acc = np.zeros_like(x)
    acc[live] = np.concatenate(parts) if parts else np.zeros((0, 3))
    x[live], v[live] = O.leapfrog_kd(x[live], v[live], acc[live], dt)
    was_live = ~lost
    lost |= was_live & sysm.lost_now(x)
    return x, v, lost, acc


def cpu_baseline_worker(npz, frac):
    """The CPU-baseline leg proper, in a process that never touches the GPU:
    the oracle, as it stands, on a bounded sample of the benchmark workload
    (one step of the same galaxy and grids with a random `frac` of its
    particles), on the host's cores; then standalone 128^3 solves."""
    from oracle import pm_oracle as O
    import synth
    cores = cpu_threads()
    O.set_fft_workers(cores)
    d = np.load(npz)
    w = synth.disc_galaxy(scale=1e-4)            # the grid set-up; particles from the file
    rng = np.random.default_rng(1736)
    n_all = d["x"].shape[0]
    n = int(n_all * frac)
    s = np.sort(rng.choice(n_all, n, replace=False))
    hs = []
    for h in w.hier:
        lv = [O.Level(L.N, L.R, L.q) for L in h.levels[:2]]
        lv.append(O.Level(h.levels[2].N, h.levels[2].R, h.levels[2].q, centre=h.outer_centre))
        hs.append(O.Hierarchy(lv, h.centring, h.centre))
    sysm = O.System(hs, G=w.G)
    x, v, m, gal = d["x"][s], d["v"][s], d["m"][s], d["gal"][s]
    lost = np.zeros(n, bool)
    t0 = time.perf_counter()
    oracle_parallel_step(sysm, x, v, m, gal, lost, w.dt, cores)
    dt = time.perf_counter() - t0
    L = hs[0].levels[1]
    rho = np.random.default_rng(1737).random((L.N, L.N, L.N))
    ts = []
    for _ in range(3):
        t1 = time.perf_counter()
        sysm.solve(rho, L)
        ts.append(time.perf_counter() - t1)
    ts.sort()
    return {"value": n / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "solves_per_s": 1.0 / ts[1],
            "step_s": dt,
            "sample": f"1 step of the same galaxy and grids with {n} of its {n_all} particles "
                      f"(random {frac:.0%}): the FP64 numpy oracle's step with its FFTs on "
                      f"{cores} threads and its per-particle Eq. 8 phase over {cores} processes, "
                      f"{dt:.1f} s; solves/s: median of 3 standalone {L.N}^3 solves on "
                      f"{cores} threads"}


def cpu_baseline(w, frac):
    """Run the CPU-baseline leg in a child process (it forks workers, which a
    process holding the GPU should not do) on the workload's particles."""
    import subprocess
    import tempfile
    tmp = tempfile.mkdtemp(prefix="sbx_cpu_")
    npz = os.path.join(tmp, "w.npz")
    try:
        np.savez(npz, x=w.x, v=w.v, m=w.m, gal=w.gal)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", npz,
                            "--cpu-frac", str(frac)], capture_output=True, text=True)
        if r.returncode != 0:
            _log(f"CPU baseline failed: {r.stderr[-2000:]}")
            return None
        return json.loads(r.stdout.strip().splitlines()[-1])
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--solve-iters", type=int, default=20)
    ap.add_argument("--diag-every", type=int, default=10)
    ap.add_argument("--cpu-frac", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--step-only", action="store_true",
                    help="only the FP32 step loop (for profiler runs)")
    ap.add_argument("--sort-every", type=int, default=None)
    ap.add_argument("--extra-steps", type=int, default=20,
                    help="timed steps of the galaxy + satellite and ensemble workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a buffer of this many MiB three times (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the precision, satellite, ensemble and adjoint measurements")
    ap.add_argument("--cpu-baseline-worker", metavar="NPZ", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        print(json.dumps(cpu_baseline_worker(args.cpu_baseline_worker, args.cpu_frac)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1210_1736_amd import sbx

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    _log("generating the 3 x 128^3 disc-galaxy workload (8.5M particles)")
    w = synth.disc_galaxy(scale=1.0)
    N = w.hier[0].levels[0].N
    nsolves = 5

    _log(f"FP32: {args.warmup} warmup + {args.steps} timed steps")
    t32, live32, ph32 = timed_steps(sbx, torch, w, sbx.SBX_FP32, args.steps, args.warmup,
                                    args.diag_every, sort_every=args.sort_every)
    value = live32 * args.steps / t32
    _log(f"FP32 {value:.4g} particle-steps/s ({1e3 * t32 / args.steps:.3f} ms/step)")

    if args.step_only:
        args.no_fp64 = True
        args.no_cpu_baseline = True
        args.no_extra = True
    fp64 = None
    if not args.no_fp64:
        _log(f"FP64: {args.fp64_steps} timed steps")
        t64, live64, ph64 = timed_steps(sbx, torch, w, sbx.SBX_FP64, args.fp64_steps, 2,
                                        args.diag_every, sort_every=args.sort_every)
        fp64 = {"particle_steps_per_s": live64 * args.fp64_steps / t64,
                "ms_per_step": 1e3 * t64 / args.fp64_steps,
                "phases_ms_per_step": {k: v[0] / args.fp64_steps for k, v in ph64.items() if v[1]}}

    _log("standalone 128^3 solves")
    solves = {}
    for name, prec in (() if args.step_only else (("fp32", sbx.SBX_FP32), ("fp64", sbx.SBX_FP64))):
        for batch in (5, 20):
            rate, ms = time_solves(sbx, torch, 128, 4.0, 0.25, prec, batch, args.solve_iters)
            esz = 8 if prec == sbx.SBX_FP64 else 4
            form = fft_form(sbx.sbx_fft_tuning_report(), esz, 128, batch)
            model = sum(phase_bytes(ph, 128, 1, 0, esz, form) for ph in FFT_PASSES)
            solves[f"{name}_batch{batch}"] = {"solves_per_s": rate, "ms_per_batch": ms, "form": form,
                                             "model_bytes_per_solve": model,
                                             "frac_of_hbm_peak": rate * model / 1e9 / HBM_PEAK_GBS}
    torch.cuda.synchronize()

    extra = {}
    if not args.no_extra:
        _log("FP32 force and potential error against the FP64 form")
        extra["precision"] = precision_errors(sbx, w)
        _log("density-maximum centring")
        extra["density_centring"] = density_centring_rate(sbx, torch, w, args.extra_steps, 2,
                                                          args.diag_every)
        _log("fixed-point mass assignment")
        extra["fixed_point_deposit"] = fixed_point_rate(sbx, torch, w, args.extra_steps, 2, args.diag_every)
        _log("galaxy + satellite")
        extra["galaxy_satellite"] = galaxy_satellite_rate(sbx, torch, args.extra_steps, 2)
        _log("ensemble of 16 instances")
        extra["ensemble"] = ensemble_rate(sbx, torch, args.extra_steps, 2)
        _log("differentiable segment")
        extra["adjoint"] = adjoint_rate(sbx, torch)
        _log("disc diagnostics")
        extra["disc_analysis"] = disc_analysis_rate(sbx, torch, w)
        _log("heating sweep")
        extra["heating"] = heating_experiment(sbx, torch, w)

    # roofline of the dominant kernel of the FP32 step
    steps = args.steps
    per_step = {k: v[0] / steps for k, v in ph32.items() if v[1]}
    dom = max(per_step, key=per_step.get)
    launches = ph32[dom][1]
    avg_ms = ph32[dom][0] / launches
    step_form = fft_form(sbx.sbx_fft_tuning_report(), 4, N, nsolves)
    by = phase_bytes(dom, N, nsolves, live32, 4, step_form)
    achieved = by / (avg_ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
            "bytes_per_launch": by, "avg_launch_ms": avg_ms}
    step_bytes = sum(phase_bytes(k, N, nsolves, live32, 4, step_form) for k in per_step)
    step_roof = step_bytes / (t32 / steps) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        _log("oracle CPU baseline")
        cpu = cpu_baseline(w, args.cpu_frac)

    out = {
        "metric": "particle-steps/s and 3D-FFT Poisson solves/s (128^3 grids), FP32 vs FP64",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "disc-bulge-halo galaxy, 3 nested 128^3 grids (R = 1, 4, 20; "
                               "q = 1/4, 1/4, 1), 8.5M particles, dt 0.01, FP64 diagnostics "
                               "every 10 steps",
                   "particles_live": live32, "solves_per_step": nsolves},
        "fp64": fp64,
        "solves": solves,
        "phases_ms_per_step": per_step,
        "phases_note": "HIP events after every phase, from a second pass of the same steps "
                       "(the timed pass runs without events)",
        "solves_in_step_per_s": nsolves / (1e-3 * sum(per_step.get(k, 0.0) for k in FFT_PASSES)),
        **extra,
        "step_effective_GBs": step_roof,
        "step_frac_of_hbm_peak": step_roof / HBM_PEAK_GBS,
        "solves_in_step_frac_of_hbm_peak": sum(phase_bytes(k, N, nsolves, live32, 4, step_form)
                                               for k in FFT_PASSES)
        / (1e-3 * sum(per_step.get(k, 0.0) for k in FFT_PASSES)) / 1e9 / HBM_PEAK_GBS,
        "roofline": roof,
        "cpu_baseline": cpu,
        # the form and launch shapes the tuner chose for the step's five
        # 128^3 solves (block size, persistent grid, values per thread)
        "fft_tuning": [l for l in sbx.sbx_fft_tuning_report().splitlines()
                       if " N=128 x5 " in l],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
