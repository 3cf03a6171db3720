"""GPU parity of the disc diagnostics (sbx_disc_analysis) against the
oracle: equal-number radial bins decided identically (bin radii, circular
velocities and thickness within rounding), heat, annulus dispersions and
vertical profile.

Bars: FP64 and FP32 contexts (the FP32 one on FP32-rounded inputs, the
oracle on the same values): bin statistics and heat within 1e-10 relative
(sums of up to millions of FP64 terms in another order), dispersions within
1e-10, profile within 1e-10 of its maximum."""
import numpy as np
import pytest

import synth
from oracle import pm_oracle as O
from tests import common as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


def _galaxy(scale):
    w = T.small_galaxy(scale=scale, N=64, centring="fixed", q=0.5)
    w.hier[0].centre = (0.013, -0.021, 0.004)
    return w


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("steps", [0, 3])
def test_disc_analysis_matches_oracle(sbx, prec, steps):
    w = _galaxy(0.02)
    ctx = T.make_ctx(w, prec)
    ctx.sbx_step(w.dt, steps)
    xg, vg, lg = ctx.sbx_get_particles()
    q = dict(n_bins=40, annulus=(2.8, 3.6), n_z=24, z_max=0.6)
    got = ctx.sbx_disc_analysis(**q)
    ref = O.disc_analysis(xg, vg, w.m if prec == 1 else T.rounded(w.m, prec), w.comp, w.gal, lg,
                          w.hier[0].centre, q["n_bins"], q["annulus"], q["n_z"], q["z_max"])
    assert got["n_disc"] == ref["n_disc"] and got["n_annulus"] == ref["n_annulus"]
    for k in ("bin_r", "bin_vc", "bin_rms_z"):
        assert np.allclose(got[k], ref[k], rtol=1e-10, atol=1e-12), k
    for k in ("e_heat", "sig_R", "sig_phi", "sig_z", "sig_tot2"):
        assert got[k] == pytest.approx(ref[k], rel=1e-10), k
    assert np.allclose(got["bulk_v"], ref["bulk_v"], rtol=1e-10, atol=1e-14)
    assert np.abs(got["rho_z"] - ref["rho_z"]).max() <= 1e-10 * np.abs(ref["rho_z"]).max()


def test_disc_analysis_full_galaxy_runs(sbx):
    """The disc of the 8.5M-particle galaxy: 100 bins; checked against the
    oracle on the same state."""
    w = synth.disc_galaxy(scale=0.25)
    w.hier[0].centring = "fixed"
    ctx = T.make_ctx(w, sbx.SBX_FP32)
    got = ctx.sbx_disc_analysis(100, (3.0, 3.4), 40, 1.0)
    xg, vg, lg = ctx.sbx_get_particles()
    ref = O.disc_analysis(xg, vg, T.rounded(w.m, 0), w.comp, w.gal, lg, (0, 0, 0), 100,
                          (3.0, 3.4), 40, 1.0)
    assert np.allclose(got["bin_r"], ref["bin_r"], rtol=1e-10)
    assert got["e_heat"] == pytest.approx(ref["e_heat"], rel=1e-10)
    assert got["sig_z"] == pytest.approx(ref["sig_z"], rel=1e-10)


def test_disc_analysis_errors(sbx):
    w = _galaxy(0.002)
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    for bad in (dict(n_bins=0, annulus=(1, 2), n_z=4, z_max=1),
                dict(n_bins=4, annulus=(2, 1), n_z=4, z_max=1),
                dict(n_bins=4, annulus=(1, 2), n_z=0, z_max=1),
                dict(n_bins=4, annulus=(1, 2), n_z=4, z_max=0)):
        with pytest.raises(sbx.SbxError) as e:
            ctx.sbx_disc_analysis(**bad)
        assert e.value.status == sbx.SBX_EINVAL
    with pytest.raises(sbx.SbxError) as e:
        ctx.sbx_disc_analysis(4, (1, 2), 4, 1.0, comp=7)
    assert e.value.status == sbx.SBX_ESTATE


@pytest.mark.parametrize("prec", [0, 1])
def test_disc_modes_match_oracle(sbx, prec):
    w = _galaxy(0.02)
    ctx = T.make_ctx(w, prec)
    ctx.sbx_step(w.dt, 2)
    xg, _, lg = ctx.sbx_get_particles()
    got = ctx.sbx_disc_modes(30, 6.0, 4)
    ref = O.disc_modes(xg, w.m if prec == 1 else T.rounded(w.m, prec), w.comp, w.gal, lg,
                       w.hier[0].centre, 30, 6.0, 4)
    scale = np.abs(ref[:, 0]).max()
    assert np.abs(got - ref).max() <= 1e-10 * scale
