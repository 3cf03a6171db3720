"""Edge cases of the library against the oracle: ragged particle counts
(partial wavefronts, blocks and chunks), a lone particle, zero masses,
every particle outside the grids, and the empty input."""
import numpy as np
import pytest

import synth
from tests import common as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, 970, k]))


def _nested(n, seed):
    rng = _rng(seed)
    x = rng.normal(size=(n, 3)) * np.array([0.6, 0.6, 0.2])
    v = rng.normal(size=(n, 3)) * 0.3
    m = rng.uniform(0.5, 1.5, n) / max(n, 1)
    comp = rng.integers(0, 3, n).astype(np.int8)
    gal = np.zeros(n, np.int8)
    hs = synth.HierSpec([synth.LevelSpec(32, 0.5, 0.5), synth.LevelSpec(32, 1.5, 0.5),
                         synth.LevelSpec(32, 4.0, 1.0)], centring="com")
    return synth.Workload("ragged", x, v, m, comp, gal, [hs], 0.02, 3)


@pytest.mark.parametrize("n", [1, 63, 65, 257, 2049, 4097])
@pytest.mark.parametrize("prec", [0, 1])
def test_ragged_counts_forces_and_steps(sbx, n, prec):
    """Counts that leave partial wavefronts, blocks and deposit chunks: forces
    in both precisions, FP64 steps (with a reorder at step 0)."""
    w = _nested(n, n)
    ctx = T.make_ctx(w, prec)
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, prec)
    lost = np.zeros(n, bool)
    acc, _ = ctx.sbx_compute_forces()
    a_ref = sysm.accel(x, m, w.gal, lost)
    tol = 1e-9 if prec == sbx.SBX_FP64 else 1e-3
    if n > 1:
        assert T.rel_err_vec(acc, a_ref).max() < tol
    if prec != sbx.SBX_FP64:
        return  # FP32 trajectories are compared statistically elsewhere
    for _ in range(w.steps):
        x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt)
    ctx.sbx_step(w.dt, w.steps)
    xg, vg, lg = ctx.sbx_get_particles()
    assert np.array_equal(lg, lost)
    assert np.abs(xg - x).max() < 1e-10


def test_lone_particle_feels_no_force(sbx):
    """A single particle on a cubic grid: its own cell exerts no force
    (H(0,0,0) = H(1,0,0)), so it stays where it is."""
    hs = synth.HierSpec([synth.LevelSpec(32, 2.0, 1.0)])
    x = np.array([[0.137, -0.41, 0.29]])
    w = synth.Workload("lone", x, np.zeros((1, 3)), np.array([3.0]), np.zeros(1, np.int8),
                       np.zeros(1, np.int8), [hs], 0.1, 5)
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    acc, pot = ctx.sbx_compute_forces()
    assert np.abs(acc).max() < 1e-12
    ctx.sbx_step(0.1, 5)
    xg, vg, lg = ctx.sbx_get_particles()
    assert not lg[0] and np.abs(xg - x).max() < 1e-12 and np.abs(vg).max() < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_masses_give_zero_fields(sbx, prec):
    w = _nested(3000, 11)
    w.m = np.zeros_like(w.m)
    w.hier[0].centring = "fixed"
    ctx = T.make_ctx(w, prec)
    acc, pot = ctx.sbx_compute_forces()
    assert np.all(acc == 0.0) and np.all(pot == 0.0)


def test_every_particle_outside_is_lost(sbx):
    """Particles that start outside the global grid are lost at the first
    loss test; the step runs on an empty live set."""
    w = _nested(500, 12)
    w.x = w.x + np.array([50.0, 0.0, 0.0])
    w.hier[0].centring = "fixed"
    ctx = T.make_ctx(w, sbx.SBX_FP32)
    ctx.sbx_step(w.dt, 4, diag_every=1)
    xg, vg, lg = ctx.sbx_get_particles()
    assert lg.all()
    assert np.array_equal(xg, T.rounded(w.x, sbx.SBX_FP32))
    assert ctx.sbx_count_live() == 0
    d = ctx.sbx_diagnostics(w.dt)
    assert d["n_lost"] == 500


def test_empty_input_rejected(sbx):
    ctx = sbx.Context(prec=sbx.SBX_FP64)
    with pytest.raises(sbx.SbxError) as e:
        ctx.sbx_load_particles(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0),
                               np.zeros(0, np.int8), np.zeros(0, np.int8))
    assert e.value.status == sbx.SBX_EINVAL


def test_device_entry_points_match_host(sbx):
    """Particles loaded from device memory and read back into device memory
    equal the host path, before and after steps."""
    import torch
    w = _nested(5000, 13)
    a = T.make_ctx(w, sbx.SBX_FP32)
    b = sbx.Context(prec=sbx.SBX_FP32, G=w.G)
    b.sbx_build_grids([T.sbx_hier(h) for h in w.hier])
    xd = torch.tensor(w.x, device="cuda")
    vd = torch.tensor(w.v, device="cuda")
    md = torch.tensor(w.m, device="cuda")
    cd = torch.tensor(w.comp, device="cuda")
    gd = torch.tensor(w.gal, device="cuda")
    torch.cuda.synchronize()
    b.sbx_load_particles_device(w.n, xd.data_ptr(), vd.data_ptr(), md.data_ptr(), cd.data_ptr(),
                                gd.data_ptr())
    for steps in (0, 5):
        a.sbx_step(w.dt, steps)
        b.sbx_step(w.dt, steps)
        xa, va, la = a.sbx_get_particles()
        xo = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
        vo = torch.empty_like(xo)
        lo = torch.empty(w.n, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        b.sbx_get_particles_device(xo.data_ptr(), vo.data_ptr(), lo.data_ptr())
        assert np.array_equal(lo.cpu().numpy().astype(bool), la)
        assert np.abs(xo.cpu().numpy() - xa).max() < 1e-6
        assert np.abs(vo.cpu().numpy() - va).max() < 1e-5


def test_device_entry_points_validate(sbx):
    import torch
    w = _nested(300, 14)
    ctx = sbx.Context(prec=sbx.SBX_FP64)
    ctx.sbx_build_grids([T.sbx_hier(h) for h in w.hier])
    xd = torch.tensor(w.x, device="cuda")
    vd = torch.tensor(w.v, device="cuda")
    md = torch.tensor(w.m, device="cuda")
    cd = torch.tensor(w.comp, device="cuda")
    gd = torch.tensor(w.gal, device="cuda")
    # host memory where device memory is required
    with pytest.raises(sbx.SbxError) as e:
        ctx.sbx_load_particles_device(w.n, w.x.ctypes.data, vd.data_ptr(), md.data_ptr(),
                                      cd.data_ptr(), gd.data_ptr())
    assert e.value.status == sbx.SBX_EINVAL
    # a non-finite position, a negative mass, a galaxy id beyond the hierarchies
    for which, k in (("x", 17), ("m", 41), ("gal", 99)):
        x2, m2, g2 = xd.clone(), md.clone(), gd.clone()
        if which == "x":
            x2[k, 1] = float("nan")
        elif which == "m":
            m2[k] = -1.0
        else:
            g2[k] = 2
        torch.cuda.synchronize()
        with pytest.raises(sbx.SbxError) as e:
            ctx.sbx_load_particles_device(w.n, x2.data_ptr(), vd.data_ptr(), m2.data_ptr(),
                                          cd.data_ptr(), g2.data_ptr())
        assert e.value.status == sbx.SBX_EINVAL and f"particle {k}" in str(e.value)
