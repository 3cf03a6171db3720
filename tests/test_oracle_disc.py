"""Pins of the oracle's disc diagnostics against closed forms."""
import numpy as np
import pytest

from oracle import pm_oracle as O


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, 980, k]))


def _antipodal(R, ph, z):
    """Each point together with its mirror through the axis (phi + pi, -z):
    mass-weighted mean velocities of rotating sets vanish."""
    p = np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)
    t = np.stack([-np.sin(ph), np.cos(ph), 0 * ph], axis=1)
    return np.concatenate([p, -p]), np.concatenate([t, -t])


def _ring_pairs(n_pairs, v0, a, rng):
    """Particles in pairs at the same (R, phi, z) with v = v0 phi-hat +-
    a phi-hat, and the mirror of every pair: every bin's mean v_phi is
    exactly v0 when no pair is split, and the mean velocity is zero."""
    R = rng.uniform(0.5, 5.0, n_pairs)
    ph = rng.uniform(0, 2 * np.pi, n_pairs)
    z = rng.normal(size=n_pairs) * 0.1
    p, t = _antipodal(R, ph, z)
    x = np.repeat(p, 2, axis=0)
    t = np.repeat(t, 2, axis=0)
    s = np.tile([1.0, -1.0], 2 * n_pairs)
    v = t * (v0 + s * a)[:, None]
    return x, v


def test_flat_rotation_has_no_heat():
    """A disc in pure rotation at constant speed: every bin mean is that speed
    and the interpolation is exact, so the heat is zero."""
    rng = _rng(1)
    h = 1000
    x, t = _antipodal(rng.uniform(0.2, 6.0, h), rng.uniform(0, 2 * np.pi, h), rng.normal(size=h) * 0.1)
    v = 1.3 * t
    n = 2 * h
    m = np.full(n, 1.0 / n)
    out = O.disc_analysis(x, v, m, np.zeros(n, np.int8), np.zeros(n, np.int8), np.zeros(n, bool),
                          (0, 0, 0), 20, (2.0, 3.0), 10, 0.5)
    assert out["e_heat"] == pytest.approx(0.0, abs=1e-26)
    assert np.allclose(out["bin_vc"], 1.3, rtol=1e-14)
    assert out["sig_phi"] == pytest.approx(0.0, abs=1e-7)


def test_paired_random_motion_heat_is_exact():
    """Pairs with v_phi = v0 +- a: bin means are v0, so the heat is exactly
    sum 1/2 m a^2; the dispersion in phi is a."""
    rng = _rng(2)
    n_pairs, v0, a = 1000, 0.9, 0.07
    x, v = _ring_pairs(n_pairs, v0, a, rng)
    n = 4 * n_pairs
    m = np.full(n, 2.0 / n)
    out = O.disc_analysis(x, v, m, np.zeros(n, np.int8), np.zeros(n, np.int8), np.zeros(n, bool),
                          (0, 0, 0), 100, (0.0, 10.0), 8, 1.0)
    assert out["e_heat"] == pytest.approx(0.5 * np.sum(m) * a * a, rel=1e-12)
    assert out["sig_phi"] == pytest.approx(a, rel=1e-10)
    assert out["sig_R"] == pytest.approx(0.0, abs=1e-12)


def test_equal_number_bins_and_profile_mass():
    """Bin sizes differ by at most one, in index order of the remainder; the
    vertical profile integrates to the annulus mass inside |z| < z_max."""
    rng = _rng(3)
    n = 1237
    x = rng.normal(size=(n, 3)) * np.array([2.0, 2.0, 0.2])
    v = rng.normal(size=(n, 3)) * 0.2
    m = rng.uniform(0.5, 1.5, n)
    out = O.disc_analysis(x, v, m, np.zeros(n, np.int8), np.zeros(n, np.int8), np.zeros(n, bool),
                          (0.1, -0.2, 0.0), 13, (1.0, 2.5), 16, 0.4)
    assert out["bin_sizes"].sum() == n
    assert out["bin_sizes"].max() - out["bin_sizes"].min() <= 1
    assert list(out["bin_sizes"][:n % 13]) == [n // 13 + 1] * (n % 13)
    assert np.all(np.diff(out["bin_r"]) > 0)
    d = x - np.array([0.1, -0.2, 0.0])
    R = np.hypot(d[:, 0], d[:, 1])
    a = (R >= 1.0) & (R < 2.5) & (np.abs(d[:, 2]) < 0.4) & (d[:, 2] >= -0.4)
    area = np.pi * (2.5 ** 2 - 1.0 ** 2)
    assert np.sum(out["rho_z"]) * area * (0.8 / 16) == pytest.approx(np.sum(m[a]), rel=1e-12)


def test_bulk_motion_is_not_heat():
    """A uniform velocity added to every disc particle changes nothing."""
    rng = _rng(4)
    n = 800
    x = rng.normal(size=(n, 3)) * np.array([2.0, 2.0, 0.2])
    v = rng.normal(size=(n, 3)) * 0.2
    m = rng.uniform(0.5, 1.5, n)
    args = (np.zeros(n, np.int8), np.zeros(n, np.int8), np.zeros(n, bool), (0, 0, 0), 10, (1.0, 2.0), 8, 0.5)
    a = O.disc_analysis(x, v, m, *args)
    b = O.disc_analysis(x, v + np.array([0.3, -1.1, 0.2]), m, *args)
    assert b["e_heat"] == pytest.approx(a["e_heat"], rel=1e-10)
    assert b["sig_R"] == pytest.approx(a["sig_R"], rel=1e-10)


def test_modes_of_uniform_ring_and_two_arm_pattern():
    """A ring of equal masses at equally spaced angles has A_0 = mass / area
    and no other modes below the ring's count; masses modulated by
    1 + e cos(2 phi) add A_2 = e A_0 / 2 and nothing at m = 1."""
    K = 360
    ph = 2 * np.pi * (np.arange(K) + 0.25) / K
    R = 2.5
    x = np.stack([R * np.cos(ph), R * np.sin(ph), 0 * ph], axis=1)
    m = np.full(K, 1.0 / K)
    z = np.zeros(K, np.int8)
    A = O.disc_modes(x, m, z, z, np.zeros(K, bool), (0, 0, 0), 5, 5.0, 4)
    S = np.pi * (3 ** 2 - 2 ** 2)
    assert A[2, 0].real == pytest.approx(1.0 / S, rel=1e-12)
    assert np.abs(A[2, 1:]).max() < 1e-14
    assert np.abs(A[[0, 1, 3, 4]]).max() == 0.0
    e = 0.3
    m2 = m * (1 + e * np.cos(2 * ph))
    A2 = O.disc_modes(x, m2, z, z, np.zeros(K, bool), (0, 0, 0), 5, 5.0, 4)
    assert abs(A2[2, 2]) == pytest.approx(0.5 * e / S, rel=1e-12)
    assert abs(A2[2, 1]) < 1e-14 and abs(A2[2, 3]) < 1e-14
