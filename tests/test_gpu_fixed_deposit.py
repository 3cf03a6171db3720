"""GPU parity of the fixed-point mass assignment (cell masses as exact
integer sums of floor(m 2^s), converted once) against the oracle's
deposit_fixed, and the reproducibility it buys.

Bars: cell masses bit-exact against the oracle (FP64 and FP32: the FP32
form converts the exact total once, the oracle's total rounded to float32
is the same number); fields and forces to the bars of the float
assignment; repeated runs bitwise equal where the centres do not depend on
the particle order (fixed centres, or no cell sort: the centre-of-mass and
density-maximum centres are FP64 sums in particle order, and the sort's
order within a cell is set by atomics).
"""
import numpy as np
import pytest

from tests import common as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


PRECS = [0, 1]  # SBX_FP32, SBX_FP64


def _fixed_ctx(sbx, w, prec, **kw):
    ctx = T.make_ctx(w, prec, **kw)
    ctx.sbx_set_deterministic_deposit(1)
    return ctx


def _mass_slots(levels, prec):
    """Oracle cell masses in the library's slot order (1, 3, 2+3, 5, 4+5),
    each grid rounded to the device precision before the host-side sum of
    the two sources of a summed slot, as the library reads them out."""
    r = [T.rounded(a, prec) for a in levels]
    if len(r) == 1:
        return r
    return [r[0], r[2], r[1] + r[2], r[4], r[3] + r[4]]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("centring", ["fixed", "density"])
def test_fixed_cell_masses_bit_exact(sbx, prec, centring):
    w = T.small_galaxy(scale=0.005, N=64, centring=centring, q=0.5)
    x, v, m = T.oracle_inputs(w, prec)
    sysm = T.oracle_system(w)
    sysm.fixed_deposit = True
    lost = sysm.lost_now(x)
    ctx = _fixed_ctx(sbx, w, prec)
    acc, _ = ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    cen = sysm.centres(x, m, w.gal, lost)
    if centring == "fixed":
        assert np.array_equal(cg[0], cen[0])
    else:  # same densest cell; the mass centre around it is an FP64 sum
        assert np.abs(cg[0] - cen[0]).max() < 1e-12 * (1 + np.abs(cen[0]).max())
    cen = cg  # both sides classify at the library's centres
    pots = sysm.potentials(x, m, w.gal, lost, cen)
    for k, ref in enumerate(_mass_slots(pots[0]["M"], prec)):
        g = ctx.sbx_get_grid(0, k, 0).transpose(2, 1, 0)
        assert np.array_equal(g, ref), (k, np.abs(g - ref).max())
    # forces to the bars of the float assignment
    a_ref = sysm.accel(x, m, w.gal, lost, cen, pots)
    e = T.rel_err_vec(acc, a_ref)
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3
    ctx.close()


@pytest.mark.parametrize("prec", PRECS)
def test_fixed_and_float_assignment_agree(sbx, prec):
    """Switching the form on and off on one context: the two force sets
    agree to the rounding of the float sums."""
    w = T.small_galaxy(scale=0.005, N=64, centring="com", q=0.5)
    ctx = T.make_ctx(w, prec)
    a0, p0 = ctx.sbx_compute_forces()
    ctx.sbx_set_deterministic_deposit(1)
    a1, p1 = ctx.sbx_compute_forces()
    ctx.sbx_set_deterministic_deposit(0)
    a2, _ = ctx.sbx_compute_forces()
    tol = 1e-10 if prec == sbx.SBX_FP64 else 1e-4
    assert T.rel_err_vec(a1, a0).max() < tol
    assert T.rel_err_vec(a2, a0).max() < tol
    assert np.abs(p1 - p0).max() <= tol * np.abs(p0).max()
    ctx.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("centring,sort", [("fixed", 1), ("com", 0), ("density", 0)])
def test_fixed_assignment_runs_are_bitwise_reproducible(sbx, prec, centring, sort):
    """Two contexts stepped alike end bitwise equal: with the integer sums
    nothing in a step depends on the order of the additions, so long as the
    centres do not (fixed centres; centre of mass or density maximum only
    when the particle order is never changed)."""
    w = T.small_galaxy(scale=0.004, N=32, centring=centring, q=1.0)
    out = []
    for _ in range(2):
        c = _fixed_ctx(sbx, w, prec)
        c.sbx_set_sort_interval(sort)
        c.sbx_step(w.dt, 6)
        out.append(c.sbx_get_particles())
        c.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_fixed_assignment_batch(sbx):
    """A batch of fixed-point contexts steps like its members stepped alone
    (to FP rounding of the FFT launch shapes); a batch that mixes the two
    forms is refused."""
    w = T.small_galaxy(scale=0.003, N=32, centring="density", q=1.0)
    solo = _fixed_ctx(sbx, w, sbx.SBX_FP64)
    solo.sbx_step(w.dt, 4)
    a = _fixed_ctx(sbx, w, sbx.SBX_FP64)
    b = _fixed_ctx(sbx, w, sbx.SBX_FP64)
    bt = sbx.Batch([a, b])
    bt.sbx_batch_step(w.dt, 4)
    bt.sbx_batch_sync()
    bt.close()
    xs, _, ls = solo.sbx_get_particles()
    for c in (a, b):
        xc, _, lc = c.sbx_get_particles()
        assert np.array_equal(lc, ls)
        assert np.abs(xc - xs).max() < 1e-11
    assert np.abs(a.sbx_get_centres() - solo.sbx_get_centres()).max() < 1e-11
    plain = T.make_ctx(w, sbx.SBX_FP64)
    with pytest.raises(sbx.SbxError) as e:
        sbx.Batch([a, plain])
    assert e.value.status == sbx.SBX_EINVAL
    # the form cannot change while a context is in a batch
    bt2 = sbx.Batch([a, b])
    with pytest.raises(sbx.SbxError) as e:
        a.sbx_set_deterministic_deposit(0)
    assert e.value.status == sbx.SBX_ESTATE
    bt2.close()
    for c in (solo, a, b, plain):
        c.close()


@pytest.mark.parametrize("prec", PRECS)
def test_fixed_assignment_survives_checkpoint(sbx, tmp_path, prec):
    """The form is part of a saved state: a context loaded from the file
    steps on bitwise like the one that saved it (fixed centres: no part of
    the step depends on the particle order, which the load resets)."""
    w = T.small_galaxy(scale=0.003, N=32, centring="fixed", q=1.0)
    a = _fixed_ctx(sbx, w, prec)
    a.sbx_step(w.dt, 3)
    path = str(tmp_path / f"fix{prec}.sbx")
    a.sbx_save(path)
    a.sbx_step(w.dt, 3)
    b = sbx.Context(prec=prec, G=w.G)
    b.sbx_load(path)
    b.sbx_step(w.dt, 3)
    for ga, gb in zip(a.sbx_get_particles(), b.sbx_get_particles()):
        assert np.array_equal(ga, gb)
    # a version-1 file (no flag: header int32 fields at bytes 8..47, the flag
    # at 44) still loads, with the float assignment
    import struct
    data = open(path, "rb").read()
    assert struct.unpack_from("<ii", data, 8) == (2, prec) and struct.unpack_from("<i", data, 44)[0] == 1
    v1 = data[:8] + struct.pack("<i", 1) + data[12:44] + data[48:]
    p1 = str(tmp_path / f"v1_{prec}.sbx")
    open(p1, "wb").write(v1)
    c, d = sbx.Context(prec=prec, G=w.G), sbx.Context(prec=prec, G=w.G)
    c.sbx_load(p1)
    d.sbx_load(path)
    for gc, gd in zip(c.sbx_get_particles(), d.sbx_get_particles()):
        assert np.array_equal(gc, gd)
    c.sbx_save(p1)
    back = open(p1, "rb").read()
    assert struct.unpack_from("<i", back, 44)[0] == 0  # the float assignment
    assert back[12:44] == data[12:44]
    for o in (a, b, c, d):
        o.close()


@pytest.mark.parametrize("prec", PRECS)
def test_fixed_cell_masses_six_galaxies(sbx, prec):
    """Six galaxies (a disc and five satellites with different particle
    masses): every galaxy's cell masses bit-exact against the oracle's
    fixed-point assignment, all on the one scale of the whole particle set
    (its largest mass and count), at the library's own centres."""
    from tests.test_gpu_manygal import _system
    w = _system()
    x, v, m = T.oracle_inputs(w, prec)
    sysm = T.oracle_system(w)
    sysm.fixed_deposit = True
    lost = sysm.lost_now(x)
    ctx = _fixed_ctx(sbx, w, prec)
    ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    pots = sysm.potentials(x, m, w.gal, lost, cg)
    for g in range(len(w.hier)):
        for k, ref in enumerate(_mass_slots(pots[g]["M"], prec)):
            got = ctx.sbx_get_grid(g, k, 0).transpose(2, 1, 0)
            assert np.array_equal(got, ref), (g, k, np.abs(got - ref).max())
    ctx.close()


def test_fixed_cell_masses_full_size(sbx):
    """The benchmark galaxy at full size (8.5M particles, 3 x 128^3, FP32):
    cell masses of the fixed-point assignment bit-exact against the oracle's
    (scale s = 62 - e - 24 for 8.5M particles), at the library's centres."""
    import synth
    w = synth.disc_galaxy(scale=1.0)
    x, v, m = T.oracle_inputs(w, sbx.SBX_FP32)
    sysm = T.oracle_system(w)
    sysm.fixed_deposit = True
    lost = sysm.lost_now(x)
    ctx = _fixed_ctx(sbx, w, sbx.SBX_FP32)
    ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    pots = sysm.potentials(x, m, w.gal, lost, cg)
    for k, ref in enumerate(_mass_slots(pots[0]["M"], sbx.SBX_FP32)):
        got = ctx.sbx_get_grid(0, k, 0).transpose(2, 1, 0)
        assert np.array_equal(got, ref), (k, np.abs(got - ref).max())
    assert np.sum(ref) > 0
    ctx.close()
