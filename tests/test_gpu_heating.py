"""The reduced heating experiment (Sec. 4, Table 3) on the GPU: its diagnostics
series against the oracle stepping the same galaxy (FP64, a few steps), and
the sweep's handling of configurations below q_crit (Eq. 9)."""
import numpy as np
import pytest

from oracle import pm_oracle as O
from tests import common as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


@pytest.mark.parametrize("q", [1.0, 0.5])
def test_series_match_oracle_fp64(sbx, q):
    from paper_1210_1736_amd import heating
    N, steps, every = 64, 4, 2
    w = T.small_galaxy(scale=0.002, N=N, centring="com", q=q)
    res = heating.run(w.x, w.v, w.m, w.comp, w.gal, N, q, steps, every, w.dt, G=w.G,
                      prec=sbx.SBX_FP64, n_bins=20, annulus=(2.0, 4.0), n_z=10, z_max=1.0)
    sysm = T.oracle_system(w)
    x, v, m = w.x.copy(), w.v.copy(), w.m.copy()
    lost = np.zeros(w.n, bool)
    centre = np.zeros(3)                  # the given centre until the first solve
    for i, k in enumerate(range(0, steps + 1, every)):
        if k > 0:
            for _ in range(every):
                x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt)
                centre = sysm.last_centres[0]
        ref = O.disc_analysis(x, v, m, w.comp, w.gal, lost, centre, 20, (2.0, 4.0), 10, 1.0)
        assert res["t"][i] == pytest.approx(k * w.dt)
        assert res["e_heat"][i] == pytest.approx(ref["e_heat"], rel=1e-9)
        assert res["sig_z"][i] == pytest.approx(ref["sig_z"], rel=1e-9)
        assert res["sig_R"][i] == pytest.approx(ref["sig_R"], rel=1e-9)
        assert res["rms_z"][i] == pytest.approx(np.mean(ref["bin_rms_z"]), rel=1e-9)
    assert np.isfinite(res["heating_rate"])


def test_sweep_skips_below_qcrit(sbx):
    from paper_1210_1736_amd import heating
    w = T.small_galaxy(scale=0.001, N=32, centring="com", q=1.0)
    out = heating.sweep(w.x, w.v, w.m, w.comp, w.gal, Ns=(32,), qs=(1.0, 0.3), steps=2, every=1,
                        dt=w.dt, n_bins=10, n_z=8)
    assert O.q_crit(32, 1.0, 4.0, 20.0) > 0.3
    assert "skipped" in out[1] and "skipped" not in out[0]
    assert len(out[0]["e_heat"]) == 3 and all(np.isfinite(out[0]["e_heat"]))
