"""The particle passes where a block walks more than one stretch of particles:
about 600k particles, so that the force pass (at most 2048 blocks of 256
threads) takes a second, ragged stride with the one-ahead prefetch, and the
mass assignment (8192 particles per block) ends in a partial chunk.  Two
steps against the oracle (Eq. 6 leapfrog on the Sec. 2.1 hierarchy), the
first of them with the cell reorder.

Bars as in test_gpu_parity: FP64 positions within 1e-10 and velocities
within 1e-8; FP32 form against the FP64 oracle on the same FP32-rounded
inputs, velocities within 1e-4 of the rms velocity (99th percentile) and
positions within 1e-4; loss flags exact."""
import numpy as np
import pytest

from tests import common as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


@pytest.fixture(scope="module")
def workload():
    w = T.small_galaxy(scale=0.0705, N=64, q=0.5)
    assert w.n > 2048 * 256 and w.n % 8192 != 0 and w.n % 256 != 0
    return w


@pytest.mark.parametrize("prec", [1, 0])  # SBX_FP64, SBX_FP32
def test_two_steps_multi_stride(sbx, workload, prec):
    w = workload
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, prec)
    lost = np.zeros(w.n, bool)
    for _ in range(2):
        x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt)
    ctx = T.make_ctx(w, prec)
    ctx.sbx_step(w.dt, 2)
    xg, vg, lg = ctx.sbx_get_particles()
    ctx.close()
    assert np.array_equal(lg, lost)
    if prec == sbx.SBX_FP64:
        assert np.max(np.abs(xg - x)) < 1e-10
        assert np.max(np.abs(vg - v)) < 1e-8
    else:
        vr = np.sqrt(np.mean(np.sum(v * v, axis=1)))
        ev = np.linalg.norm(vg - v, axis=1) / vr
        assert np.percentile(ev, 99) < 1e-4
        assert np.max(np.abs(xg - x)) < 1e-4
