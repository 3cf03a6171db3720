"""Seeded input generators: the paper's model numbers they rest on."""
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G_KPC = 4.30091e-6  # kpc (km/s)^2 / Msun


def test_disc_truncation_fraction():
    """Sec. 3.1: cutting the exponential disc at 10 h drops (1 + 10) e^-10 of
    the mass, the quoted 0.05 per cent."""
    frac = (1 + 10) * math.exp(-10)
    assert frac == pytest.approx(4.99e-4, rel=1e-3)
    assert 1 - synth._disc_mass_frac(np.array([10.0]), 1.0, 1e9)[0] == pytest.approx(frac, rel=1e-9)


def test_table4_orbit_setup():
    """Table 4: R_P = R_A (1 - e)/(1 + e); both speeds imply the same enclosed
    mass M(<25 kpc) ~ 1.747e11 Msun by v^2 = G M (1 - e)/R_A."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "table4_orbits.txt"))
            if ln.strip() and not ln.startswith("#")]
    masses = []
    for e, v, RA, RP in (map(float, r) for r in rows):
        assert synth.pericentre(RA, e) == pytest.approx(RP, abs=0.015)
        masses.append(v * v * RA / ((1 - e) * G_KPC))
        _, vel = synth.point_mass_orbit(masses[-1], RA, e, 0.0, G=G_KPC)
        assert np.linalg.norm(vel) == pytest.approx(v, rel=1e-12)
    assert masses[0] == pytest.approx(1.747e11, rel=1e-3)
    assert masses[1] == pytest.approx(masses[0], rel=2e-3)


def test_table2_mass_ratios():
    """Table 2: halo particles are ten times heavier than disc particles; the
    bulge and halo masses relative to the disc."""
    gm = synth.GalaxyModel()
    assert gm.M_bulge == pytest.approx(0.444, abs=1e-3)
    assert gm.M_halo == pytest.approx(4.149, abs=1e-3)
    assert 20.0e10 / 2.15e6 / (4.82e10 / 5.19e6) == pytest.approx(10.0, rel=0.01)


def test_galaxy_generator_shapes_and_seeding():
    w1 = synth.disc_galaxy(scale=0.002)
    w2 = synth.disc_galaxy(scale=0.002)
    assert np.array_equal(w1.x, w2.x) and np.array_equal(w1.v, w2.v)
    n_d = int(2_000_000 * 0.002)
    d = w1.x[w1.comp == synth.DISC]
    assert d.shape[0] == n_d
    R = np.hypot(d[:, 0], d[:, 1])
    assert R.max() < 10.0 and np.abs(d[:, 2]).max() < 1.0
    # exponential disc: mean radius of Sigma ~ e^-R is ~2 h (truncated)
    assert 1.8 < R.mean() < 2.1
    assert abs(w1.m.sum() - (1 + 0.444 + 4.149)) < 0.01
    h = w1.x[w1.comp == synth.HALO]
    assert np.linalg.norm(h, axis=1).max() < 18.0


def test_plummer_generator_moments():
    w = synth.plummer_cube(n=50_000)
    r = np.linalg.norm(w.x, axis=1)
    assert r.max() < 4.5
    # half-mass radius of the truncated sphere: M(<r)/M(<4.5) = 1/2
    Rt = 4.5; u = 0.5 * Rt ** 3 / (Rt ** 2 + 1) ** 1.5
    rh = 1.0 / math.sqrt(u ** (-2 / 3) - 1)
    assert np.median(r) == pytest.approx(rh, rel=0.02)
    # virial-like check: 2 K ~ |W| within sampling and truncation
    K = 0.5 * np.sum(w.m * np.sum(w.v ** 2, axis=1))
    assert 0.12 < K < 0.16
