"""More than two galaxies (Sec. 2.1: the number of galaxies is not fixed):
a disc galaxy and five Plummer satellites, each with its own three-level
hierarchy on the shared global grid, against the oracle's separate solves.
Bars as in test_gpu_parity."""
import numpy as np
import pytest

import synth
from oracle import pm_oracle as O
from tests import common as T

pytestmark = pytest.mark.gpu

PRECS = [0, 1]  # SBX_FP32, SBX_FP64


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


def _system(n_sat=5, N=32):
    w = T.small_galaxy(scale=0.002, N=N, centring="com", q=1.0)
    rng = np.random.default_rng(np.random.SeedSequence([1210, 1736, 950]))
    xs, vs, ms, comps, gals = [w.x], [w.v], [w.m], [w.comp], [w.gal]
    hier = list(w.hier)
    for k in range(n_sat):
        n = 2000 + 500 * k
        p, r = synth.plummer_positions(rng, n, 0.4, 3.0)
        ang = 2.0 * np.pi * k / n_sat
        c = np.array([7.0 * np.cos(ang), 7.0 * np.sin(ang), 0.5 * (k - 2)])
        v = synth.plummer_velocities(rng, r, 0.05, 0.4)
        xs.append(p + c)
        vs.append(v + np.array([-np.sin(ang), np.cos(ang), 0.0]) * 0.3)
        ms.append(np.full(n, 0.05 / n))
        comps.append(np.full(n, 7, np.int8))
        gals.append(np.full(n, k + 1, np.int8))
        hier.append(synth.HierSpec([synth.LevelSpec(N, 1.0, 1.0), synth.LevelSpec(N, 6.0, 1.0),
                                    synth.LevelSpec(N, 20.0, 1.0)], centring="com"))
    w.x = np.concatenate(xs)
    w.v = np.concatenate(vs)
    w.m = np.concatenate(ms)
    w.comp = np.concatenate(comps)
    w.gal = np.concatenate(gals)
    w.hier = hier
    return w


@pytest.mark.parametrize("prec", PRECS)
def test_six_galaxies_forces_and_classes(sbx, prec):
    w = _system()
    assert len(w.hier) == 6
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, prec)
    lost = sysm.lost_now(x)
    centres = sysm.centres(x, m, w.gal, lost)
    pots = sysm.potentials(x, m, w.gal, lost, centres)
    ctx = T.make_ctx(w, prec)
    acc, _ = ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    for g in range(6):
        assert np.allclose(cg[g], centres[g], rtol=0, atol=1e-13 * (1 + np.abs(centres[g]).max()))
        cls_ref, idx_ref = O.classify(x, sysm.h[g], cg[g])
        idx, cls = ctx.sbx_get_indices(g, 0)
        assert np.array_equal(cls, cls_ref), g
        assert np.array_equal(idx.astype(np.int64), idx_ref[0]), g
    a_ref = sysm.accel(x, m, w.gal, lost, centres, pots)
    e = T.rel_err_vec(acc, a_ref)
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3


def test_eight_galaxies_steps_fp64_and_merge(sbx):
    w = _system(n_sat=7)
    assert len(w.hier) == 8
    sysm = T.oracle_system(w)
    x, v, m = w.x.copy(), w.v.copy(), w.m.copy()
    lost = np.zeros(w.n, bool)
    for _ in range(2):
        x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt)
    for merge in (0, 1):
        ctx = sbx.Context(prec=sbx.SBX_FP64, G=w.G)
        ctx.sbx_set_outer_merge(merge)
        ctx.sbx_build_grids([T.sbx_hier(h) for h in w.hier])
        ctx.sbx_load_particles(w.x, w.v, w.m, w.comp, w.gal)
        ctx.sbx_step(w.dt, 2)
        xg, vg, lg = ctx.sbx_get_particles()
        assert np.array_equal(lg, lost), merge
        assert np.max(np.abs(xg - x)) < 1e-10, merge
        assert np.max(np.abs(vg - v)) < 1e-8, merge
        ctx.close()


def test_nine_galaxies_rejected(sbx):
    w = _system(n_sat=8)
    ctx = sbx.Context(prec=sbx.SBX_FP64, G=w.G)
    with pytest.raises(sbx.SbxError):
        ctx.sbx_build_grids([T.sbx_hier(h) for h in w.hier])
