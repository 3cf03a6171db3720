"""Helpers shared by the GPU tests: converting the seeded set-ups for the
oracle and for the library, rounding inputs to the device precision."""
import numpy as np

import synth
from oracle import pm_oracle as O


def oracle_hier(hs: synth.HierSpec) -> O.Hierarchy:
    if len(hs.levels) == 1:
        L = hs.levels[0]
        return O.Hierarchy([O.Level(L.N, L.R, L.q, centre=hs.centre)], "fixed", hs.centre)
    lv = [O.Level(L.N, L.R, L.q) for L in hs.levels[:2]]
    L3 = hs.levels[2]
    lv.append(O.Level(L3.N, L3.R, L3.q, centre=hs.outer_centre))
    return O.Hierarchy(lv, hs.centring, hs.centre)


def sbx_hier(hs: synth.HierSpec):
    from paper_1210_1736_amd import sbx
    cent = {"com": sbx.SBX_CENTRE_COM, "density": sbx.SBX_CENTRE_DENSITY}.get(hs.centring,
                                                                              sbx.SBX_CENTRE_FIXED)
    return sbx.make_hierarchy([(L.N, L.R, L.q) for L in hs.levels], cent, hs.centre, hs.outer_centre)


def rounded(a, prec):
    """Values as the device stores them, back in float64."""
    from paper_1210_1736_amd import sbx
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if prec == sbx.SBX_FP32 else a.copy()


def make_ctx(w: synth.Workload, prec, taylor=1, h0_mode=0):
    from paper_1210_1736_amd import sbx
    ctx = sbx.Context(prec=prec, G=w.G, taylor=taylor, h0_mode=h0_mode)
    ctx.sbx_build_grids([sbx_hier(h) for h in w.hier])
    ctx.sbx_load_particles(w.x, w.v, w.m, w.comp, w.gal)
    return ctx


def oracle_system(w: synth.Workload, taylor=True, h0_mode=0):
    return O.System([oracle_hier(h) for h in w.hier], G=w.G, h0_mode=h0_mode, taylor=taylor)


def oracle_inputs(w: synth.Workload, prec):
    return rounded(w.x, prec), rounded(w.v, prec), rounded(w.m, prec)


def rel_err_vec(a, b):
    """|a - b| per row over the rms row norm of b."""
    rms = np.sqrt(np.mean(np.sum(b * b, axis=1)))
    return np.linalg.norm(a - b, axis=1) / rms


def small_galaxy(scale=0.005, N=64, centring="com", q=0.25):
    """The disc galaxy at reduced particle count on 3 levels of N^3 cells."""
    w = synth.disc_galaxy(scale=scale, N=N)
    w.hier = [synth.HierSpec([synth.LevelSpec(N, 1.0, q), synth.LevelSpec(N, 4.0, q),
                              synth.LevelSpec(N, 20.0, 1.0)], centring=centring)]
    return w
