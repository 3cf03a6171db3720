"""GPU parity of density-maximum centring (Sec. 2.1: the inner and middle
grids follow the density maximum of their galaxy) against the oracle.

The densest cell is an integer decided on exact integer cell masses on both
sides, so the chosen cell agrees exactly; the centre is the FP64 mass centre
of its 3x3x3 block, summed in a different order on the GPU: bar 1e-13 of the
centre's scale.  The oracle chains the centre from step to step as the
library does.
"""
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


def _galaxy(centre=(0.05, -0.03, 0.01), N=64, q=0.5, scale=0.005):
    w = T.small_galaxy(scale=scale, N=N, centring="density", q=q)
    w.hier[0].centre = centre
    return w


def _close(a, b, scale=1.0):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= 1e-13 * (scale + np.max(np.abs(b)))


@pytest.mark.parametrize("prec", PRECS)
def test_first_solve_centre_classes_forces(sbx, prec):
    w = _galaxy()
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, prec)
    lost = sysm.lost_now(x)
    centres = sysm.centres(x, m, w.gal, lost)
    # the search moved the centre away from the given one
    assert np.max(np.abs(centres[0] - np.asarray(w.hier[0].centre))) > 0.01
    ctx = T.make_ctx(w, prec)
    assert np.array_equal(ctx.sbx_get_centres()[0], np.asarray(w.hier[0].centre))
    acc, _ = ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    assert _close(cg[0], centres[0])
    cls_ref, idx_ref = O.classify(x, sysm.h[0], cg[0])
    for level in range(3):
        idx, cls = ctx.sbx_get_indices(0, level)
        assert np.array_equal(cls, cls_ref)
        assert np.array_equal(idx.astype(np.int64), idx_ref[level])
    pots = sysm.potentials(x, m, w.gal, lost, centres)
    a_ref = sysm.accel(x, m, w.gal, lost, centres, pots)
    e = T.rel_err_vec(acc, a_ref)
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3
    # a second solve at the same positions starts from the first one's centre
    ctx.sbx_compute_forces()
    c2 = sysm.centres(x, m, w.gal, lost, centres)
    assert _close(ctx.sbx_get_centres()[0], c2[0])


def test_steps_chain_the_centre_fp64(sbx):
    """Steps with a sort before the first solve: the sort must not move the
    centre, every solve moves it once."""
    w = _galaxy(centre=(0.08, 0.02, -0.015), N=64, q=0.5, scale=0.003)
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    ctx.sbx_set_sort_interval(2)
    sysm = T.oracle_system(w)
    x, v, m = w.x.copy(), w.v.copy(), w.m.copy()
    lost = np.zeros(w.n, bool)
    prev = None
    for k in range(4):
        x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt, prev_centres=prev)
        prev = sysm.last_centres
        ctx.sbx_step(w.dt, 1)
        assert _close(ctx.sbx_get_centres()[0], prev[0]), k
    xg, vg, lg = ctx.sbx_get_particles()
    assert np.array_equal(lg, lost)
    assert np.max(np.abs(xg - x)) < 1e-10
    assert np.max(np.abs(vg - v)) < 1e-8


@pytest.mark.parametrize("prec", PRECS)
def test_galaxy_and_satellite_density(sbx, prec):
    """Both galaxies density-centred, each on its own particles."""
    w = synth.galaxy_satellite(scale=0.004, N=64)
    for h in w.hier:
        h.levels = [synth.LevelSpec(64, L.R, 1.0) for L in h.levels]
        h.centring = "density"
    sat = w.x[w.gal == 1].mean(axis=0)            # the satellite's starting place
    w.hier[1].centre = tuple(sat + np.array([0.04, -0.05, 0.03]))
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, prec)
    lost = sysm.lost_now(x)
    centres = sysm.centres(x, m, w.gal, lost)
    ctx = T.make_ctx(w, prec)
    ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    for g in range(2):
        assert _close(cg[g], centres[g]), g
        cls_ref, _ = O.classify(x, sysm.h[g], cg[g])
        _, cls = ctx.sbx_get_indices(g, 0)
        assert np.array_equal(cls, cls_ref)


def test_nothing_on_the_inner_grid_keeps_the_centre(sbx):
    w = _galaxy(centre=(30.0, 0.0, 0.0), scale=0.002)   # inner grid outside the system
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    sysm = T.oracle_system(w)
    lost = sysm.lost_now(w.x)
    ref = sysm.centres(w.x, w.m, w.gal, lost)[0]
    assert np.array_equal(ref, np.asarray(w.hier[0].centre))
    ctx.sbx_compute_forces()
    assert np.array_equal(ctx.sbx_get_centres()[0], ref)


def test_batch_matches_single_context(sbx):
    """A density-centred instance stepped in a batch (one graph per step)
    next to a centre-of-mass one: centres and positions agree with the same
    instance stepped alone."""
    wd = _galaxy(scale=0.002, N=32, q=1.0)
    wc = T.small_galaxy(scale=0.002, N=32, centring="com", q=1.0)
    solo = T.make_ctx(wd, sbx.SBX_FP64)
    solo.sbx_step(wd.dt, 5)
    a = T.make_ctx(wd, sbx.SBX_FP64)
    b = T.make_ctx(wc, sbx.SBX_FP64)
    bt = sbx.Batch([a, b])
    bt.sbx_batch_step(wd.dt, 5)
    bt.sbx_batch_sync()
    bt.close()
    assert _close(a.sbx_get_centres()[0], solo.sbx_get_centres()[0])
    xa, _, la = a.sbx_get_particles()
    xs, _, ls = solo.sbx_get_particles()
    assert np.array_equal(la, ls)
    assert np.max(np.abs(xa - xs)) < 1e-11
