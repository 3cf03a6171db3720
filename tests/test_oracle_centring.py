"""Pins of the oracle's density-maximum centring (Sec. 2.1: the inner and
middle grids follow the density maximum of their galaxy).

The paper names the density maximum but not how it is found; the oracle's
reading (exact integer cell masses on the inner grid at the previous centre,
the densest cell with ties to the lowest (z, y, x) index, then the centre of
mass of its 3x3x3 block) is pinned here by closed forms: centroids of point
sets placed by hand, the tie rule, the mask, the integer range and a sampled
Plummer sphere whose centre is known.
"""
import numpy as np
import pytest

from oracle import pm_oracle as O
import synth

# N = 16, R = 6: cell length exactly 1 in x and y, q = 1/2 in z.
L = O.Level(16, 6.0, 0.5)


def cell_point(a, b, c, frac=(0.0, 0.0, 0.0), prev=(0.0, 0.0, 0.0)):
    """Position at fractional offset `frac` (in cells) from the centre of
    cell (a, b, c) of L placed at `prev`."""
    return np.array([prev[0] + (a - 8 + frac[0]) * 1.0,
                     prev[1] + (b - 8 + frac[1]) * 1.0,
                     prev[2] + (c - 8 + frac[2]) * 0.5])


def pairs_around(p, deltas):
    """Points p + d and p - d for each d: their centroid is p."""
    out = []
    for d in deltas:
        out.append(p + d)
        out.append(p - d)
    return np.array(out)


DELTAS = [np.array([0.2, 0.1, 0.05]), np.array([-0.1, 0.05, 0.02]), np.array([0.05, -0.08, -0.04])]


def background(rng, avoid, n=40, lo=0, hi=15):
    """Unit masses at cell centres of distinct random cells at least two
    cells (max norm) from every cell in `avoid`."""
    pts, used = [], set()
    while len(pts) < n:
        a, b, c = (int(v) for v in rng.integers(lo, hi + 1, 3))
        if (a, b, c) in used or any(max(abs(a - u[0]), abs(b - u[1]), abs(c - u[2])) < 2 for u in avoid):
            continue
        used.add((a, b, c))
        pts.append(cell_point(a, b, c))
    return np.array(pts)


def run(x, m, mask=None, prev=(0.0, 0.0, 0.0)):
    mask = np.ones(len(m), bool) if mask is None else mask
    return O.density_max_centre(x, m, mask, L, np.asarray(prev, float), O.density_mass_shift(m))


def test_single_clump_centroid():
    rng = np.random.default_rng(1)
    p = cell_point(10, 5, 9, (0.1, 0.1, -0.1))
    clump = pairs_around(p, DELTAS)                     # 6 unit masses in one cell
    bg = background(rng, [(10, 5, 9)])                  # one unit mass per cell elsewhere
    x = np.vstack([clump, bg])
    m = np.ones(len(x))
    c = run(x, m)
    assert np.allclose(c, p, rtol=0, atol=1e-14)
    # the particle order does not matter
    perm = rng.permutation(len(x))
    assert np.allclose(run(x[perm], m[perm]), p, rtol=0, atol=1e-14)


def test_window_takes_the_neighbouring_cells():
    rng = np.random.default_rng(2)
    p = cell_point(10, 5, 9, (0.1, 0.1, -0.1))
    q = cell_point(11, 5, 8)                            # adjacent cell (+1, 0, -1)
    r = cell_point(12, 5, 9)                            # two cells away: outside
    clump = pairs_around(p, DELTAS)
    x = np.vstack([clump, [q], [r], background(rng, [(10, 5, 9), (11, 5, 8), (12, 5, 9)])])
    m = np.ones(len(x))
    m[6] = 2.0
    m[7] = 5.0                                          # heavier but alone: 5 < 6
    c = run(x, m)
    assert np.allclose(c, (6.0 * p + 2.0 * q) / 8.0, rtol=0, atol=1e-14)


def test_ties_go_to_the_lowest_zyx_cell():
    # equal totals in three cells; the lowest (z, y, x) index is (12, 12, 4)
    cells = [(4, 4, 12), (12, 12, 4), (13, 12, 4)]
    ps = [cell_point(*b, (0.05, -0.1, 0.2)) for b in cells]
    x = np.vstack([pairs_around(p, DELTAS[:2]) for p in ps])
    m = np.ones(len(x))
    # (12, 12, 4) and (13, 12, 4) are neighbours: their block holds both
    c = run(x, m)
    assert np.allclose(c, 0.5 * (ps[1] + ps[2]), rtol=0, atol=1e-14)
    # without the third cell the tie is between (4, 4, 12) and (12, 12, 4)
    c2 = run(x[:8], m[:8])
    assert np.allclose(c2, ps[1], rtol=0, atol=1e-14)
    # reversed listing, same answer
    c3 = run(x[:8][::-1], m[:8][::-1])
    assert np.allclose(c3, ps[1], rtol=0, atol=1e-14)


def test_mask_excludes_other_galaxies_and_lost():
    rng = np.random.default_rng(3)
    p = cell_point(6, 9, 7, (-0.2, 0.1, 0.1))
    decoy = cell_point(9, 9, 9)
    inside = cell_point(7, 9, 7)                        # in the clump's block
    clump = pairs_around(p, DELTAS)
    x = np.vstack([clump, np.repeat([decoy], 5, axis=0), [inside],
                   background(rng, [(6, 9, 7), (9, 9, 9)])])
    m = np.ones(len(x))
    m[6:12] = 100.0
    mask = np.ones(len(x), bool)
    mask[6:12] = False                                  # another galaxy's or lost particles
    assert np.allclose(run(x, m, mask), p, rtol=0, atol=1e-14)


def test_previous_centre_places_the_grid():
    prev = (0.37, -1.25, 0.3)
    p = cell_point(5, 11, 6, (0.1, -0.1, 0.05), prev)
    x = pairs_around(p, DELTAS)
    # a heavier clump that is on the grid only without the shift of the centre
    far = cell_point(15, 15, 15, (0.4, 0.4, 0.4))
    x = np.vstack([x, [far] * 7])
    m = np.ones(len(x))
    assert np.allclose(run(x, m, prev=prev), p, rtol=0, atol=1e-14)


def test_nothing_on_the_grid_keeps_the_previous_centre():
    x = np.array([[30.0, 0.0, 0.0], [0.0, -30.0, 0.0], [0.0, 0.0, 10.0]])
    m = np.ones(3)
    prev = np.array([0.5, 0.25, -0.125])
    assert np.array_equal(run(x, m, prev=prev), prev)
    assert np.array_equal(run(x, m, np.zeros(3, bool), prev), prev)


def test_integer_totals_do_not_overflow():
    # every particle at the largest mass in one cell: the total is as large as
    # the scale allows and must still be the maximum
    p = cell_point(8, 8, 8, (0.1, 0.2, -0.1))
    n = 5001
    x = np.repeat([p], n, axis=0)
    x[-1] = cell_point(2, 2, 2)
    m = np.full(n, 3.0)
    s = O.density_mass_shift(m)
    assert n * 3.0 * 2.0 ** s < 2.0 ** 62
    assert np.allclose(run(x, m), p, rtol=0, atol=1e-13)


def test_small_masses_still_count():
    # 3 light particles (2^-20 of the largest mass) outweigh 2 others of 2^-19.5
    a = cell_point(4, 4, 4, (0.1, 0.1, 0.1))
    b = cell_point(10, 10, 10, (-0.1, 0.2, 0.0))
    heavy = cell_point(2, 13, 2)
    x = np.vstack([[a] * 3, [b] * 2, [heavy]])
    m = np.array([2.0 ** -20] * 3 + [2.0 ** -19.5] * 2 + [1.0])
    # the heavy particle's cell wins outright
    assert np.allclose(run(x, m), heavy, rtol=0, atol=1e-14)
    # without it the light cells decide: 3 * 2^-20 > 2 * 2^-19.5
    mask = np.array([True] * 5 + [False])
    assert np.allclose(run(x, m, mask), a, rtol=0, atol=1e-14)


@pytest.mark.parametrize("q", [1.0, 0.5])
def test_plummer_sphere_centre_found(q):
    rng = np.random.default_rng(11)
    Lp = O.Level(32, 3.0, q)                            # cell 0.214, z cell 0.214 q
    c0 = np.array([0.31, -0.17, 0.08])
    x = synth.plummer_positions(rng, 40_000, 0.3, 3.0)[0] * np.array([1.0, 1.0, q]) + c0
    m = np.full(len(x), 1.0 / len(x))
    c = O.density_max_centre(x, m, np.ones(len(x), bool), Lp, np.zeros(3), O.density_mass_shift(m))
    # within about one cell of the true centre, starting from the origin
    assert np.all(np.abs(c - c0) < 0.6 * Lp.lengths)
    # a second pass from the found centre stays there
    c2 = O.density_max_centre(x, m, np.ones(len(x), bool), Lp, c, O.density_mass_shift(m))
    assert np.all(np.abs(c2 - c0) < 0.6 * Lp.lengths)


def test_system_step_chains_the_centre():
    rng = np.random.default_rng(5)
    lv = [O.Level(16, 2.0, 1.0), O.Level(16, 6.0, 1.0), O.Level(16, 12.0, 1.0)]
    h = O.Hierarchy(lv, "density", (0.0, 0.0, 0.0))
    sysm = O.System([h])
    c0 = np.array([0.6, -0.4, 0.2])
    x = synth.plummer_positions(rng, 3000, 0.4, 4.0)[0] + c0
    v = np.zeros_like(x)
    m = np.full(len(x), 1.0 / len(x))
    gal = np.zeros(len(x), np.int8)
    lost = np.zeros(len(x), bool)
    c_first = sysm.centres(x, m, gal, lost)[0]
    x1, v1, lost1, _ = sysm.step(x, v, m, gal, lost, 1e-3)
    assert np.array_equal(sysm.last_centres[0], c_first)
    # the next step starts from the stored centre, not from the hierarchy's
    cn = sysm.centres(x1, m, gal, lost1, sysm.last_centres)[0]
    x2, _, _, _ = sysm.step(x1, v1, m, gal, lost1, 1e-3, prev_centres=sysm.last_centres)
    assert np.array_equal(sysm.last_centres[0], cn)
    assert np.all(np.abs(cn - c0) < 1.5 * lv[0].lengths)
