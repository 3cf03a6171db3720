"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the formula
under test: the FFT route is checked against the direct sum of Eq. 1, the
field and the forces against closed forms and continuum limits, the geometry
against the printed tables, the integrator against exact discrete solutions.
"""
import math
import os

import numpy as np
import pytest

from oracle import pm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, 900, k]))


# ---------------------------------------------------------------- P1 -------
@pytest.mark.parametrize("N,q,h0", [(8, 1.0, 0), (16, 1.0, 0), (16, 0.25, 0), (16, 0.5, 2), (32, 1.0, 0)])
def test_fft_route_equals_direct_sum(N, q, h0):
    """Doubled-grid DFT convolution (Eqs. 3-5) reproduces Eq. 1 exactly."""
    L = O.Level(N, 3.0, q)
    rng = _rng(N)
    M = np.zeros((N, N, N))
    cells = rng.integers(0, N, size=(60 if N == 32 else 200, 3))
    np.add.at(M, tuple(cells.T), rng.uniform(0.1, 1.0, cells.shape[0]))
    Hh, _ = O.green_hat(L, h0)
    a = O.solve_fft(M, Hh, G=1.7)
    b = O.solve_direct(M, L, G=1.7, h0_mode=h0)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_periodic_convolution_would_fail():
    """Negative control: without doubling (periodic N-grid) Eq. 1 is not met,
    so the check above can tell isolated from periodic boundaries."""
    N = 16
    L = O.Level(N, 3.0)
    M = np.zeros((N, N, N)); M[1, 2, 3] = 1.0; M[12, 9, 14] = 2.0
    H = O.green_table(L)
    k = np.arange(N); fold = np.minimum(k, N - k)
    Hp = H[fold[:, None, None], fold[None, :, None], fold[None, None, :]]
    per = np.fft.ifftn(np.fft.fftn(M) * np.fft.fftn(Hp)).real
    ref = O.solve_direct(M, L)
    assert np.max(np.abs(per - ref)) > 1e-2 * np.max(ref)


# ---------------------------------------------------------------- P2 -------
@pytest.mark.parametrize("q", [1.0, 0.25])
def test_point_mass_field_closed_form(q):
    """A unit mass in one cell: Phi = G m / |physical lag| everywhere else,
    G m h0 in its own cell (Eqs. 1-2 with physical cell lengths)."""
    N = 32
    L = O.Level(N, 2.0, q)
    s = np.array([7, 20, 13])
    M = np.zeros((N, N, N)); M[tuple(s)] = 0.3
    Hh, _ = O.green_hat(L)
    Phi = O.solve_fft(M, Hh, G=2.0)
    g = np.indices((N, N, N)).reshape(3, -1).T
    dist = np.sqrt((((g - s) * L.lengths) ** 2).sum(axis=1))
    own = np.all(g == s, axis=1)
    expect = np.where(own, 2.0 * 0.3 / L.l, 2.0 * 0.3 / np.where(own, 1.0, dist))
    assert np.allclose(Phi.reshape(-1), expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("q", [1.0, 0.25])
def test_point_mass_force_continuum_limit(q):
    """Eq. 8 on the grid field of a point mass tends to G m / r^2 towards the
    mass, with error O((l/r)^2); the Taylor terms of Eq. 8 reduce the error
    (this fixes the sign and origin of the in-cell offset Delta)."""
    N = 64
    L = O.Level(N, 6.0, q)
    h = O.Hierarchy([L])
    sysm = O.System([h], G=1.0)
    rng = _rng(3)
    # heavy particle at a cell centre, massless probes around it
    src = np.zeros((1, 3))
    r = rng.uniform(12 * L.l, 24 * L.l, 400)
    d = rng.normal(size=(400, 3)); d /= np.linalg.norm(d, axis=1)[:, None]
    d[:, 2] *= q  # stay inside the flattened box
    probes = d * r[:, None]
    x = np.concatenate([src, probes])
    m = np.concatenate([[1.0], np.zeros(400)])
    gal = np.zeros(401, np.int8); lost = np.zeros(401, bool)
    acc = sysm.accel(x, m, gal, lost)[1:]
    rr = np.linalg.norm(probes, axis=1)
    exact = -probes / rr[:, None] ** 3
    err_t = np.linalg.norm(acc - exact, axis=1) / np.linalg.norm(exact, axis=1)
    sysm.taylor = False
    acc0 = sysm.accel(x, m, gal, lost)[1:]
    err_c = np.linalg.norm(acc0 - exact, axis=1) / np.linalg.norm(exact, axis=1)
    lmax = L.l
    assert np.all(err_t < 4.0 * (lmax / rr) ** 2 + 1e-12)
    assert np.median(err_t) < 0.5 * np.median(err_c)
    # direction: attractive
    assert np.all(np.sum(acc * probes, axis=1) < 0)


# ---------------------------------------------------------------- P3 -------
def test_lone_particle_feels_no_self_force():
    """h0 = H(1,0,0): a lone particle anywhere in its cubic cell feels zero
    force (its own cell enters Eq. 8 only through the symmetric stencil)."""
    N = 16
    L = O.Level(N, 3.0)
    sysm = O.System([O.Hierarchy([L])])
    rng = _rng(4)
    for _ in range(20):
        x = ((rng.integers(3, N - 4, 3) - N / 2) + rng.uniform(-0.5, 0.5, 3)) * L.l
        a = sysm.accel(x[None, :], np.ones(1), np.zeros(1, np.int8), np.zeros(1, bool))
        assert np.max(np.abs(a)) < 1e-12 / L.l ** 2
    sys2 = O.System([O.Hierarchy([L])], h0_mode=2)
    x = np.array([[0.3 * L.l, 0.0, 0.0]])
    a2 = sys2.accel(x, np.ones(1), np.zeros(1, np.int8), np.zeros(1, bool))
    assert abs(a2[0, 0]) > 1e-3 / L.l ** 2  # h0 = 0 does leave a self-force


# ---------------------------------------------------------------- P4 -------
def test_momentum_conservation_central_differences():
    """Central differences of a symmetric H are antisymmetric: sum m a = 0."""
    N = 32
    L = O.Level(N, 4.0)
    sysm = O.System([O.Hierarchy([L])], taylor=False)
    rng = _rng(5)
    n = 3000
    x = rng.normal(size=(n, 3)) * 1.0
    x = np.clip(x, -3.5, 3.5)
    m = rng.uniform(0.5, 1.5, n) / n
    a = sysm.accel(x, m, np.zeros(n, np.int8), np.zeros(n, bool))
    P = (m[:, None] * a).sum(axis=0)
    scale = (m[:, None] * np.abs(a)).sum()
    assert np.max(np.abs(P)) < 1e-13 * scale


# ---------------------------------------------------------------- P5 -------
def test_plummer_sphere_potential_and_force():
    """Plummer sphere (G = M = a = 1) on a 64^3 grid of side 10a: PM potential
    and force match the truncated-Plummer closed forms away from the cell scale.

    phi(r) = -M_inf / sqrt(r^2 + a^2) + (M_inf / a)(1 + R_t^2/a^2)^(-3/2) for
    r < R_t, M_inf = M (R_t^2 + a^2)^(3/2) / R_t^3; |a| = M(<r)/r^2."""
    import synth
    w = synth.plummer_cube(n=100_000)
    h = O.Hierarchy([O.Level(64, 5.0)])
    sysm = O.System([h])
    lost = np.zeros(w.n, bool)
    acc, P = sysm.accel(w.x, w.m, w.gal, lost, want_pot=True)
    r = np.linalg.norm(w.x, axis=1)
    Rt = 4.5
    Minf = (Rt ** 2 + 1) ** 1.5 / Rt ** 3
    phi_exact = -Minf / np.sqrt(r * r + 1) + Minf * (1 + Rt * Rt) ** -1.5
    sel = (r > 0.5) & (r < 4.0)
    rel = np.abs(-P[sel] - phi_exact[sel]) / np.abs(phi_exact[sel])
    assert np.median(rel) < 5e-3 and np.percentile(rel, 99) < 2e-2
    ar = -np.sum(acc * w.x, axis=1) / r
    Menc = Minf * r ** 3 / (r * r + 1) ** 1.5
    # grid softening of the NGP force decays as (l/r)^2; shot noise ~ 1e-3
    l = 10.0 / 60.0
    bins = np.linspace(0.6, 4.4, 12)
    for lo, hi in zip(bins[:-1], bins[1:]):
        s = (r > lo) & (r < hi)
        tol = (l / lo) ** 2 + 4e-3
        assert abs(np.mean(ar[s] * r[s] ** 2 / Menc[s]) - 1.0) < tol, (lo, hi)


# ---------------------------------------------------------------- P6 -------
def test_hierarchy_point_mass_each_class():
    """Nested grids: a point mass at the galaxy centre reaches core, ring and
    outer probes through their own grids (grid-selection rule, Sec. 2.1) with
    G m / r^2 each; core and ring probes sit on flattened grids."""
    h = O.Hierarchy([O.Level(64, 1.0, 0.5), O.Level(64, 4.0, 0.5), O.Level(64, 20.0)],
                    centring="fixed")
    sysm = O.System([h])
    rng = _rng(6)
    radii = {O.CORE: (0.3, 0.8), O.RING: (1.6, 3.0), O.OUTER: (8.0, 16.0)}
    for cls_want, (lo, hi) in radii.items():
        d = rng.normal(size=(200, 3)); d /= np.linalg.norm(d, axis=1)[:, None]
        d[:, 2] *= 0.3
        probes = d * rng.uniform(lo, hi, 200)[:, None]
        x = np.concatenate([np.zeros((1, 3)), probes])
        m = np.concatenate([[1.0], np.zeros(200)])
        cls, _ = O.classify(probes, h, np.zeros(3))
        assert np.all(cls == cls_want)
        acc = sysm.accel(x, m, np.zeros(201, np.int8), np.zeros(201, bool))[1:]
        rr = np.linalg.norm(probes, axis=1)
        exact = -probes / rr[:, None] ** 3
        err = np.linalg.norm(acc - exact, axis=1) / np.linalg.norm(exact, axis=1)
        assert np.percentile(err, 95) < 2e-2, (cls_want, np.percentile(err, 95))


def test_hierarchy_matches_single_fine_grid():
    """A compact Plummer sphere on three nested grids and on one fine grid give
    the same forces within the coarse grids' resolution."""
    import synth
    w = synth.plummer_cube(n=20_000)
    x = w.x * 0.2  # a = 0.2
    sel = np.linalg.norm(x, axis=1) < 0.9
    x, m = x[sel], w.m[sel]
    n = x.shape[0]
    h3 = O.Hierarchy([O.Level(64, 0.5), O.Level(64, 2.0), O.Level(64, 8.0)])
    h1 = O.Hierarchy([O.Level(128, 1.0)])
    a3 = O.System([h3]).accel(x, m, np.zeros(n, np.int8), np.zeros(n, bool))
    a1 = O.System([h1]).accel(x, m, np.zeros(n, np.int8), np.zeros(n, bool))
    r = np.linalg.norm(x, axis=1)
    s = r > 0.1
    err = np.linalg.norm(a3[s] - a1[s], axis=1) / np.linalg.norm(a1[s], axis=1)
    assert np.median(err) < 0.03


# ---------------------------------------------------------------- P7 -------
def test_table3_vertical_resolution_and_qcrit():
    """l_z = q * 2R/(N-4) with R_out = 28 kpc reproduces Table 3 (in pc); the
    '-' entry is exactly the one below q_crit of Eq. 9."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "table3_vertical_resolution.txt"))
            if ln.strip() and not ln.startswith("#")]
    Ns = [64, 128, 256, 512]
    misprints = {(0.125, 256)}  # printed 27, computes to 27.8
    for row in rows:
        q = float(row[0])
        for N, cell in zip(Ns, row[1:]):
            L = O.Level(N, 28.0, q)
            qc = O.q_crit(N, 3.5, 28.0, 105.0)
            if cell == "-":
                assert q < qc
                continue
            assert q >= qc
            tol = 1.0 if (q, N) in misprints else 0.5
            assert abs(L.lz * 1000.0 - float(cell)) <= tol, (q, N, L.lz * 1000)
    assert O.q_crit(64, 3.5, 28, 105) == pytest.approx(0.25)
    assert O.q_crit(128, 3.5, 28, 105) == pytest.approx(0.125)
    assert O.q_crit(256, 3.5, 28, 105) == pytest.approx(0.125)
    assert O.q_crit(128, 1.0, 4.0, 20.0) == pytest.approx(0.25)


def test_validate_rejects_below_qcrit():
    ok = O.Hierarchy([O.Level(128, 1.0, 0.25), O.Level(128, 4.0, 0.25), O.Level(128, 20.0)])
    O.validate_hierarchy(ok)
    bad = O.Hierarchy([O.Level(128, 1.0, 0.2), O.Level(128, 4.0, 0.2), O.Level(128, 20.0)])
    with pytest.raises(ValueError):
        O.validate_hierarchy(bad)
    with pytest.raises(ValueError):
        O.validate_hierarchy(ok, first_galaxy=False)


# ---------------------------------------------------------------- cells ----
def test_ngp_cell_edges_and_membership():
    """Eq. 7 nearest cell: cell centres map to themselves, +-0.49 cell stays,
    +-0.51 moves; usable range [2, N-3]; class precedence on a flattened
    hierarchy including radii exactly at R (coarser class)."""
    L = O.Level(32, 7.0)
    c = np.array([0.25, -0.5, 1.0])
    k = np.array([2, 16, 29])
    for f, shift in [(0.0, 0), (0.49, 0), (-0.49, 0), (0.51, 1), (-0.51, -1)]:
        x = c + ((k - 16) + f) * L.l
        idx, _ = O.ngp_cell(x[None, :], c, L)
        assert np.all(idx[0] == k + shift)
    assert O.in_usable(np.array([[2, 2, 2]]), 32)[0]
    assert not O.in_usable(np.array([[1, 2, 2]]), 32)[0]
    assert O.in_usable(np.array([[29, 29, 29]]), 32)[0]
    assert not O.in_usable(np.array([[30, 29, 29]]), 32)[0]
    h = O.Hierarchy([O.Level(64, 1.0, 0.5), O.Level(64, 4.0, 0.5), O.Level(64, 20.0)])
    pts = np.array([[0.5, 0, 0], [0, 0, 0.2], [0, 0, 0.45], [1.0, 0, 0], [0, 0, 0.5],
                    [2.0, 0, 0], [0, 0, 1.9], [4.0, 0, 0], [0, 0, 2.5], [15.0, 0, 0],
                    [19.99, 0, 0], [21.0, 0, 0]])
    want = [O.CORE, O.CORE, O.CORE, O.RING, O.RING,
            O.RING, O.RING, O.OUTER, O.OUTER, O.OUTER,
            O.LOST, O.LOST]
    cls, _ = O.classify(pts, h, np.zeros(3))
    assert list(cls) == want


# ---------------------------------------------------------------- P8 -------
def test_leapfrog_uniform_acceleration_is_exact_parabola():
    """Eq. 6 with constant a: x_n = x_0 + n dt v_{-1/2} + a dt^2 n(n+1)/2."""
    x = np.array([[0.1, -0.2, 0.3]]); v = np.array([[1.0, 0.5, -0.25]])
    a = np.array([[0.0, 0.0, -2.0]]); dt = 0.125
    x0, v0 = x.copy(), v.copy()
    for _ in range(16):
        x, v = O.leapfrog_kd(x, v, a, dt)
    n = 16
    assert np.allclose(x, x0 + n * dt * v0 + a * dt * dt * n * (n + 1) / 2, rtol=0, atol=1e-14)
    assert np.allclose(v, v0 + n * dt * a, rtol=0, atol=1e-14)


def test_leapfrog_harmonic_phase():
    """Linear force a = -w^2 x: the kick-drift leapfrog advances the phase by
    theta with cos(theta) = 1 - w^2 dt^2 / 2 (exact discrete solution)."""
    w, dt = 1.3, 0.1
    th = math.acos(1 - 0.5 * (w * dt) ** 2)
    x = np.array([[1.0, 0, 0]])
    # choose v_{-1/2} so that x_n = cos(n theta): x_1 = cos(theta)
    v = np.array([[(math.cos(th) - 1.0) / dt + dt * w * w, 0, 0]])
    for n in range(1, 200):
        x, v = O.leapfrog_kd(x, v, -w * w * x, dt)
        assert abs(x[0, 0] - math.cos(n * th)) < 1e-11


def test_step_drifts_only_live_and_flags_loss():
    """Particles beyond the global grid are lost at once and never move."""
    h = O.Hierarchy([O.Level(32, 4.0)])
    sysm = O.System([h])
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [5.0, 0.0, 0.0], [3.95, 0.0, 0.0]])
    v = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    m = np.array([1.0, 0.0, 0.0, 0.0])
    gal = np.zeros(4, np.int8); lost = np.zeros(4, bool)
    x1, v1, lost1, _ = sysm.step(x, v, m, gal, lost, 0.1)
    assert list(lost1) == [False, False, True, True]
    assert np.all(x1[2] == x[2]) and np.all(v1[2] == v[2])
    x2, v2, lost2, _ = sysm.step(x1, v1, m, gal, lost1, 0.1)
    assert np.all(x2[3] == x1[3])


# ---------------------------------------------------------------- P9 -------
def test_translation_by_whole_cells():
    """Isolated boundaries: moving every particle by whole cells inside the
    active region leaves all forces unchanged (periodic images would not)."""
    N = 32
    L = O.Level(N, 4.0)
    sysm = O.System([O.Hierarchy([L])])
    rng = _rng(9)
    n = 500
    x = rng.normal(size=(n, 3)) * 0.6 - 1.0
    m = rng.uniform(0.5, 1.5, n)
    z = np.zeros(n, np.int8); lost = np.zeros(n, bool)
    a0 = sysm.accel(x, m, z, lost)
    shift = np.array([5, 3, 6]) * L.l
    a1 = sysm.accel(x + shift, m, z, lost)
    assert np.max(np.abs(a1 - a0)) < 1e-11 * np.max(np.abs(a0))


def test_superposition_of_galaxies_fields():
    """Fields add: potentials of disjoint mass sets sum to that of the union."""
    N = 16
    L = O.Level(N, 2.0, 0.5)
    Hh, _ = O.green_hat(L)
    rng = _rng(10)
    A = rng.uniform(size=(N, N, N)) * (rng.uniform(size=(N, N, N)) < 0.1)
    B = rng.uniform(size=(N, N, N)) * (rng.uniform(size=(N, N, N)) < 0.1)
    lhs = O.solve_fft(A + B, Hh)
    rhs = O.solve_direct(A, L) + O.solve_direct(B, L)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


# ---------------------------------------------------------------- P10 ------
@pytest.mark.parametrize("N,q", [(16, 1.0), (32, 0.25)])
def test_green_hat_real_and_even(N, q):
    """The DFT of the mirrored H is real and even per axis (Sec. 2.1)."""
    L = O.Level(N, 1.0, q)
    Hh, rel_imag = O.green_hat(L)
    assert rel_imag < 1e-14
    k = np.arange(2 * N); r = (2 * N - k) % (2 * N)
    assert np.allclose(Hh, Hh[r, :, :], rtol=1e-13, atol=1e-13 * np.abs(Hh).max())
    assert np.allclose(Hh, Hh[:, r, :], rtol=1e-13, atol=1e-13 * np.abs(Hh).max())
    assert np.allclose(Hh, Hh[:, :, r], rtol=1e-13, atol=1e-13 * np.abs(Hh).max())


# ---------------------------------------------------------------- energy ---
def test_energy_of_two_bodies():
    """Diagnostics: W of two distant unit-ish masses equals -G m1 m2 / d on the
    grid (the pair energy split half and half), E_kin and L of known motion."""
    L = O.Level(64, 8.0)
    sysm = O.System([O.Hierarchy([L])])
    cells = np.array([[20, 32, 32], [44, 32, 32]])
    x = (cells - 32) * L.l
    m = np.array([0.7, 0.4])
    v = np.array([[0.0, 0.3, 0.0], [0.0, -0.2, 0.0]])
    comp = np.array([0, 1], np.int8)
    d = sysm.diagnostics(x, v, m, comp, np.zeros(2, np.int8), np.zeros(2, bool), dt=0.0)
    dist = 24 * L.l
    # each body's potential also contains its own-cell term h0 * m
    self_e = 0.5 * (m ** 2).sum() / L.l
    assert d["epot"].sum() == pytest.approx(-(m[0] * m[1] / dist) - self_e, rel=1e-12)
    assert d["ekin"][0] == pytest.approx(0.5 * 0.7 * 0.09, rel=1e-12)
    Lz = 0.7 * x[0, 0] * 0.3 + 0.4 * x[1, 0] * (-0.2)
    assert d["L"][:, 2].sum() == pytest.approx(Lz, rel=1e-12)


# ------------------------------------------------- Eq. 8 Taylor form --------
def test_taylor_form_exact_on_quadratic_field():
    """Central differences of a quadratic are exact, so on a grid holding
    Phi(r) = c0 + g.r + 1/2 r.A.r at the cell centres Eq. 8 gives grad Phi
    exactly and the quadratic Taylor form (the potential at a particle) gives
    Phi exactly, anywhere in a cell.  Anisotropic cells (q = 1/2), a shifted
    grid centre and a full symmetric A with distinct entries catch a swapped
    offset, a dropped 1/2, a sign or an l/lz mix-up."""
    N = 16
    c = np.array([0.3, -0.2, 0.1])
    L = O.Level(N, 2.0, 0.5, centre=c)
    c0, g = 0.7, np.array([0.11, -0.23, 0.37])
    A = np.array([[1.3, 0.4, -0.7], [0.4, -0.9, 0.25], [-0.7, 0.25, 2.1]])
    i = np.arange(N)
    R = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).astype(float)
    R = (R - N / 2.0) * L.lengths
    Phi = c0 + R @ g + 0.5 * np.einsum("...a,ab,...b->...", R, A, R)
    rng = _rng(40)
    cells = rng.integers(3, N - 3, size=(200, 3))
    x = c + (cells - N / 2.0 + rng.uniform(-0.49, 0.49, size=(200, 3))) * L.lengths
    sysm = O.System([O.Hierarchy([L], "fixed", c)])
    acc, pot = sysm.field_at(x, [c], [{"Phi": [Phi]}])
    r = x - c
    assert np.allclose(acc, g + r @ A, rtol=1e-12, atol=1e-12)
    assert np.allclose(pot, c0 + r @ g + 0.5 * np.einsum("na,ab,nb->n", r, A, r), rtol=1e-12,
                       atol=1e-12)
    # the offsets really span the cells (not only their centres)
    idx, d = O.ngp_cell(x, c, L)
    assert np.array_equal(idx, cells)
    assert np.abs(O.cell_offset(d, idx, L) / L.lengths).max() > 0.45


# ------------------------------------------------------- diagnostics --------
def test_diagnostics_half_kick_at_nonzero_dt():
    """E_kin and L use v_sync = v(t - dt/2) + dt/2 a(t), which is the mean of
    the staggered velocities before and after the step's kick (Eq. 6; the
    kick is pinned by the parabola test).  A dropped or doubled half kick
    gives the old or the new staggered velocity instead.  A particle outside
    the global grid is lost before the sums."""
    L = O.Level(32, 2.5)
    sysm = O.System([O.Hierarchy([L])])
    rng = _rng(41)
    n = 300
    x = rng.normal(size=(n, 3)) * 0.5
    x[0] = [3.0, 0.0, 0.0]                        # off the grid: lost
    v = rng.normal(size=(n, 3)) * 0.3
    m = rng.uniform(0.5, 1.5, n) / n
    comp = (rng.uniform(size=n) < 0.4).astype(np.int8)
    gal = np.zeros(n, np.int8)
    lost = np.zeros(n, bool)
    dt = 0.05
    d = sysm.diagnostics(x, v, m, comp, gal, lost, dt)
    x1, v1, lost1, acc = sysm.step(x, v, m, gal, lost, dt)
    assert lost1[0] and not lost1[1:].any()
    vs = 0.5 * (v + v1)
    for c in (0, 1):
        s = (comp == c) & ~lost1
        assert d["ekin"][c] == pytest.approx(0.5 * np.sum(m[s] * np.sum(vs[s] ** 2, axis=1)), rel=1e-13)
        Lc = np.sum(m[s, None] * np.cross(x[s], vs[s]), axis=0)
        assert np.allclose(d["L"][c], Lc, rtol=1e-12, atol=1e-15)
    # the half kick is a visible part of E_kin here
    s = (comp == 0) & ~lost1
    e_old = 0.5 * np.sum(m[s] * np.sum(v[s] ** 2, axis=1))
    assert abs(d["ekin"][0] / e_old - 1.0) > 1e-4
    assert d["n_lost"] == 1


def test_disc_dispersions_hand_placed():
    """sigma_R and sigma_z of the disc (live component 0 of galaxy 0) about
    galaxy 0's centre, unweighted, on four particles whose radial and vertical
    velocities are (1, 3, -1, 5) and (0.2, -0.4, 0.6, 0): sigma_R = sqrt(5),
    sigma_z = sqrt(0.13).  A bulge particle and a lost disc particle with
    large velocities must not enter."""
    c = np.array([0.5, -0.25, 0.0])
    L = O.Level(32, 2.5, centre=c)
    sysm = O.System([O.Hierarchy([L], "fixed", c)])
    d = np.array([[1.0, 0.0, 0.1], [0.0, 1.0, -0.1], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.05],
                  [0.3, 0.3, 0.0], [0.2, -0.1, 0.0]])
    v = np.array([[1.0, 0.7, 0.2], [0.3, 3.0, -0.4], [1.0, -0.5, 0.6], [0.1, -5.0, 0.0],
                  [9.0, 9.0, 9.0], [-7.0, 8.0, -6.0]])
    x = c + d
    m = np.array([1.0, 2.0, 0.5, 1.5, 3.0, 1.0]) * 1e-3
    comp = np.array([0, 0, 0, 0, 1, 0], np.int8)
    lost = np.array([False] * 5 + [True])
    out = sysm.diagnostics(x, v, m, comp, np.zeros(6, np.int8), lost, 0.0)
    assert out["disc_sigR"] == pytest.approx(np.sqrt(5.0), rel=1e-14)
    assert out["disc_sigz"] == pytest.approx(np.sqrt(0.13), rel=1e-13)


# ------------------------------------------------------- centre of mass -----
def test_centre_of_mass_hand_placed():
    """Centre-of-mass centring (Sec. 2.1) of two galaxies: each galaxy's live
    particles only.  Galaxy 0: masses 1, 2, 3 at (0,0,0), (1,0,0), (0,1,0.5)
    -> (1/3, 1/2, 1/4); galaxy 1: masses 2, 2 at (3,0,0), (5,2,0) -> (4,1,0).
    A heavy lost particle in each galaxy is left out."""
    lv = lambda: [O.Level(32, 1.0), O.Level(32, 4.0), O.Level(32, 20.0)]
    sysm = O.System([O.Hierarchy(lv(), "com"), O.Hierarchy(lv(), "com")])
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.5], [5, 5, 5], [3, 0, 0], [5, 2, 0], [-3, -3, 0]],
                 float)
    m = np.array([1.0, 2.0, 3.0, 10.0, 2.0, 2.0, 7.0])
    gal = np.array([0, 0, 0, 0, 1, 1, 1], np.int8)
    lost = np.array([False, False, False, True, False, False, True])
    c = sysm.centres(x, m, gal, lost)
    assert np.allclose(c[0], [1.0 / 3.0, 0.5, 0.25], rtol=1e-15, atol=0)
    assert np.allclose(c[1], [4.0, 1.0, 0.0], rtol=1e-15, atol=0)


# ------------------------------------------------- H(0,0,0) readings -------
@pytest.mark.parametrize("sides", [(1.0, 1.0, 1.0), (1.0, 1.0, 0.25), (0.3, 0.3, 0.15)])
def test_cell_mean_h0_against_quadrature(sides):
    """h0_mode 1: the mean of 1/r over the cell, from the closed form of the
    potential of a uniform prism, against adaptive cubature of 1/r over one
    octant (unit cube: 2.3800773640)."""
    from scipy import integrate
    lx, ly, lz = sides
    f = lambda z, y, x: 1.0 / np.sqrt(x * x + y * y + z * z)
    v, _ = integrate.tplquad(f, 0, lx / 2, 0, ly / 2, 0, lz / 2, epsabs=1e-13, epsrel=1e-12)
    ref = 8.0 * v / (lx * ly * lz)
    assert O.cell_mean_inverse_distance(lx, ly, lz) == pytest.approx(ref, rel=1e-11)
    L = O.Level(16, 1.0, lz / lx)
    assert O.h0_value(L, 1) == pytest.approx(O.cell_mean_inverse_distance(L.l, L.l, L.lz), rel=1e-15)
    if sides == (1.0, 1.0, 1.0):
        assert ref == pytest.approx(2.3800773640, abs=1e-10)


def test_h0_mode_changes_only_the_own_cell_term():
    """The three readings of H(0,0,0) differ only in the zero-lag term: the
    fields of a point mass differ by G m (h0 - h0') in its own cell alone."""
    N = 16
    L = O.Level(N, 2.0, 0.5)
    M = np.zeros((N, N, N)); M[5, 7, 9] = 0.8
    f = {k: O.solve_fft(M, O.green_hat(L, k)[0]) for k in (0, 1, 2)}
    for a, b in ((0, 1), (1, 2), (0, 2)):
        d = f[a] - f[b]
        want = 0.8 * (O.h0_value(L, a) - O.h0_value(L, b))
        assert d[5, 7, 9] == pytest.approx(want, rel=1e-11)
        d[5, 7, 9] = 0.0
        assert np.abs(d).max() < 1e-12 * np.abs(f[a]).max()


# ---------------------------------------- fixed-point mass assignment -------
def _fixed_exact(idx, m, N, shift):
    """The fixed-point cell masses with Python integers and fractions, one
    particle at a time: floor(m 2^s) by exact rational arithmetic, exact
    integer totals, one rounding to float64 at the end."""
    from fractions import Fraction
    tot = {}
    for (a, b, c), mm in zip(idx.tolist(), m.tolist()):
        qi = math.floor(Fraction(mm) * 2 ** shift)
        tot[(a, b, c)] = tot.get((a, b, c), 0) + qi
    out = np.zeros((N, N, N))
    for k, t in tot.items():
        out[k] = float(Fraction(t, 2 ** shift))  # correctly rounded
    return out, tot


@pytest.mark.parametrize("seed", [0, 1])
def test_fixed_deposit_against_exact_rationals(seed):
    """deposit_fixed against exact rational arithmetic on random masses over
    many decades (every cell total correctly rounded), within the bound of
    the truncation (K 2^-s for K particles) of the exact real sums, and
    bitwise independent of the order of the particles."""
    rng = np.random.default_rng(seed)
    N, n = 4, 3000
    idx = rng.integers(0, N, (n, 3))
    idx[: n // 2] = (1, 2, 3)  # one crowded cell
    m = rng.random(n) * 10.0 ** rng.integers(-8, 1, n)
    s = O.density_mass_shift(m)
    got = O.deposit_fixed(idx, m, N, s)
    want, tot = _fixed_exact(idx, m, N, s)
    assert np.array_equal(got, want)
    assert max(abs(t) for t in tot.values()) < 2 ** 62
    from fractions import Fraction
    flat = [tuple(r) for r in idx.tolist()]
    for key in set(flat):
        exact = sum(Fraction(mm) for k, mm in zip(flat, m.tolist()) if k == key)
        K = flat.count(key)
        assert 0 <= exact - Fraction(got[key]) <= Fraction(K, 2 ** s) + Fraction(got[key]) * 2 ** -52
    perm = rng.permutation(n)
    assert np.array_equal(O.deposit_fixed(idx[perm], m[perm], N, s), got)


def test_fixed_deposit_closed_forms():
    """Dyadic masses at the scale are exact: n equal masses in one cell give
    n m; the largest mass times the particle count stays below 2^62 at the
    scale (the worst cell of the set); a mass below 2^-s rounds to zero."""
    n = 1000
    m = np.full(n, 0.375)
    idx = np.zeros((n, 3), np.int64)
    s = O.density_mass_shift(m)
    assert s == 62 + 1 - 10  # 0.375 < 2^-1, 1000 < 2^10
    M = O.deposit_fixed(idx, m, 2, s)
    assert M[0, 0, 0] == 375.0 and np.count_nonzero(M) == 1
    assert n * math.floor(0.375 * 2 ** s) < 2 ** 62
    m2 = np.array([0.0, 1.0])
    s2 = O.density_mass_shift(m2)
    m2[0] = 2.0 ** -(s2 + 1)
    M2 = O.deposit_fixed(np.array([[0, 0, 0], [1, 1, 1]]), m2, 2, s2)
    assert M2[0, 0, 0] == 0.0 and M2[1, 1, 1] == 1.0


def test_fixed_deposit_system_matches_float_sums():
    """The fixed-point reading changes the solve only at the level of the
    truncation and of the summation order: the cell masses and fields of a
    three-level disc galaxy with either assignment agree to 1e-13 of their
    largest values."""
    from tests import common as T
    w = T.small_galaxy(scale=0.002, N=32, centring="fixed", q=1.0)
    res = []
    for fixed in (False, True):
        sysm = O.System([T.oracle_hier(h) for h in w.hier], G=w.G, fixed_deposit=fixed)
        lost = sysm.lost_now(w.x)
        cen = sysm.centres(w.x, w.m, w.gal, lost)
        res.append(sysm.potentials(w.x, w.m, w.gal, lost, cen)[0])
    for key in ("M", "Phi"):
        for a, b in zip(res[0][key], res[1][key]):
            assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
