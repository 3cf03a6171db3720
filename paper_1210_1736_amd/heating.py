"""Reduced isolated-disc heating experiment (Sec. 4, Table 3; diagnostics of
Sec. 4.2 and 5.2-5.4): one disc galaxy evolved in isolation on three nested grids of
N^3 cells whose inner two levels are flattened to q, with the disc's heat,
velocity dispersions and thickness recorded along the way.  The paper runs
this sweep over N and q on its relaxed model for a gigayear; here it runs on
the seeded synthetic galaxy for a few hundred steps, so the numbers show the
trend with resolution, not the paper's values.

Everything goes through the library's C ABI (sbx.py); nothing here computes
the method.
"""
from __future__ import annotations

import time

import numpy as np

from . import sbx


def run(x, v, m, comp, gal, N, q, steps, every, dt, G=1.0, prec=sbx.SBX_FP32,
        radii=(1.0, 4.0, 20.0), annulus=(3.0, 3.4), n_bins=100, n_z=40, z_max=1.0,
        centring=sbx.SBX_CENTRE_COM):
    """Evolve one configuration; diagnostics at t = 0, every, 2 every, ...

    Returns a dict with the time series (t, e_heat, sig_R, sig_z, rms_z: the
    mean over the equal-number bins of the RMS height) and the wall time of
    the steps alone.
    """
    ctx = sbx.Context(prec=prec, G=G)
    try:
        h = sbx.make_hierarchy([(N, radii[0], q), (N, radii[1], q), (N, radii[2], 1.0)], centring)
        ctx.sbx_build_grids([h])
        ctx.sbx_load_particles(x, v, m, comp, gal)
        rec = {k: [] for k in ("t", "e_heat", "sig_R", "sig_z", "rms_z")}
        t_steps = 0.0
        k = 0
        while True:
            d = ctx.sbx_disc_analysis(n_bins, annulus, n_z, z_max)
            rec["t"].append(k * dt)
            rec["e_heat"].append(d["e_heat"])
            rec["sig_R"].append(d["sig_R"])
            rec["sig_z"].append(d["sig_z"])
            rec["rms_z"].append(float(np.mean(d["bin_rms_z"])))
            if k >= steps:
                break
            n = min(every, steps - k)
            ctx.sbx_sync()
            t0 = time.perf_counter()
            ctx.sbx_step(dt, n)
            ctx.sbx_sync()
            t_steps += time.perf_counter() - t0
            k += n
    finally:
        ctx.close()
    t = np.asarray(rec["t"])
    e = np.asarray(rec["e_heat"])
    slope = float(np.polyfit(t, e, 1)[0]) if len(t) > 1 else 0.0
    rec.update(N=N, q=q, steps=steps, dt=dt, steps_s=t_steps,
               heating_rate=slope, heating_rate_rel=slope / e[0] if e[0] > 0 else None)
    return rec


def sweep(x, v, m, comp, gal, Ns=(64, 128), qs=(1.0, 0.5, 0.25), steps=400, every=100, dt=0.01,
          G=1.0, prec=sbx.SBX_FP32, radii=(1.0, 4.0, 20.0), **kw):
    """run() for every (N, q); a configuration whose middle grid is below
    q_crit of Eq. 9 is reported as skipped."""
    out = []
    for N in Ns:
        for q in qs:
            qc = sbx.sbx_q_crit(N, radii[0], radii[1], radii[2])
            if q < qc:
                out.append({"N": N, "q": q, "skipped": f"q below q_crit = {qc:.3f} (Eq. 9)"})
                continue
            out.append(run(x, v, m, comp, gal, N, q, steps, every, dt, G=G, prec=prec, radii=radii,
                           **kw))
    return out
