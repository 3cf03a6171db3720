"""Plain FP64 CPU oracle of the nested-grid particle-mesh field solve.

Method: Bien, Brandt & Just (2012), "Simulating sinking satellites with
Superbox-10", Sec. 2 (Eqs. 1-9, Fig. 2 and the grid-selection rule).

TEST INFRASTRUCTURE. This module is the reference the GPU library is checked
against.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the HIP library and
imports nothing from it; the only thing both sides share is the seeded input
generator module, which holds none of the method's arithmetic.

Everything is float64 numpy.  Where the paper gives a plain definition (the
isolated direct sum of Eq. 1 with the Green's function of Eq. 2) the oracle
computes that definition; everything around it (nearest-grid-point cells,
Eq. 8 differencing, the five grids and their selection rule, leapfrog) is an
approximation scheme and is followed step by step in the paper's order.  The
FFT route of Eqs. 3-5 uses a library FFT (scipy.fft) as a step.

Readings of points the paper leaves open (each one is also used by the GPU
library, and listed in the design notes):
  * cell length l = 2R/(N-4) for a grid of half-extent R (Table 3 values and
    the "two cells of grid 4" in Eq. 9), z cell length q*l for flattening q;
  * grids hold cell MASS; H uses physical distances, so Eq. 1 reads
    Phi[a] = G * sum M[xi] / |(xi-a) * (lx, ly, lz)|;
  * H(0,0,0) (singular in Eq. 2) is H(1,0,0) = 1/lx by default (h0_mode 0),
    the mean of 1/r over the cell (h0_mode 1) or 0 (h0_mode 2);
  * Phi_paper = +G sum M H is positive and the acceleration is +grad Phi_paper
    (Eq. 8); the physical potential reported is phi = -Phi_paper;
  * nearest integer of Eq. 7: u = (x - c) * gamma + N/2 as separate float64
    operations (no fused multiply-add), cell a = floor(u + 0.5);
  * usable cells per axis are [2, N-3] (two empty cells at each boundary);
  * membership uses the spheroidal radius r^2 = (dx^2 + dy^2) + (dz/q)^2 with
    strict '<', core before ring before outer before lost;
  * the outermost level is the fixed global grid; leaving its usable cells
    means the particle is lost for good;
  * velocities are staggered: the input v is v(t - dt/2).

Functions whose result has no independent pin carry "parity unpinned" in
their docstring.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as _fft

# Threads of the library FFT used as a step of Eqs. 3-5 (pocketfft through
# scipy.fft; the transform is the same whatever the count): the process's
# thread budget (OMP_NUM_THREADS) when set, else the usable cores, at most 16.
_FFT_WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(
    len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1), 16)


def set_fft_workers(n: int) -> int:
    """Set the number of threads of the oracle's FFT steps; returns the old one."""
    global _FFT_WORKERS
    old, _FFT_WORKERS = _FFT_WORKERS, max(1, int(n))
    return old

CORE, RING, OUTER, LOST = 0, 1, 2, 3


# --------------------------------------------------------------------------
# Geometry (Sec. 2.1 Eq. 7; Sec. 2.2.2 Eq. 9; Table 3)
# --------------------------------------------------------------------------
class Level:
    """One grid geometry: N cells per axis, half-extent R, flattening q.

    The usable region ([2, N-3] cells, Sec. 2.1 after Eq. 8) spans N-4 cells,
    so the cell length is l = 2R/(N-4); Table 3 lists exactly these values for
    R_out = 28 kpc.  A flattened grid (Sec. 2.2.2) has z cell length q*l.
    """

    def __init__(self, N: int, R: float, q: float = 1.0, centre=(0.0, 0.0, 0.0)):
        N = int(N)
        if N < 8 or N & (N - 1):
            raise ValueError("N must be a power of two >= 8 (Sec. 2.1)")
        self.N = N
        self.R = float(R)
        self.q = float(q)
        self.centre = np.asarray(centre, dtype=np.float64)
        self.l = (2.0 * self.R) / float(N - 4)
        self.lz = self.q * self.l
        self.gx = 1.0 / self.l
        self.gz = 1.0 / self.lz
        self.inv_q = 1.0 / self.q
        self.R2 = self.R * self.R

    @property
    def lengths(self):
        return np.array([self.l, self.l, self.lz])

    @property
    def gammas(self):
        return np.array([self.gx, self.gx, self.gz])

    def same_geometry(self, other: "Level") -> bool:
        return (self.N, self.R, self.q) == (other.N, other.R, other.q) and bool(
            np.all(self.centre == other.centre))


def q_crit(N: int, R_core: float, R_out: float, R_sys: float) -> float:
    """Smallest admissible flattening of the middle grids, Eq. 9."""
    return max(R_core / R_out, 4.0 / (N - 4) * R_sys / R_out)


class Hierarchy:
    """Grids of one galaxy (Sec. 2.1, Fig. 2).

    Three levels: inner (grid 1), middle (grids 2 and 3 share it) and outer
    (grids 4 and 5, the fixed global grid).  One level: a single isolated grid
    holding every particle.  `centring` is 'fixed', 'com' (centre of mass,
    the alternative the paper names) or 'density' (the density maximum, see
    density_max_centre); it moves the inner and middle levels only.  The
    outer level keeps its own fixed centre.
    """

    def __init__(self, levels, centring="fixed", centre=(0.0, 0.0, 0.0)):
        self.levels = list(levels)
        if len(self.levels) not in (1, 3):
            raise ValueError("a hierarchy has 1 or 3 levels")
        if centring not in ("fixed", "com", "density"):
            raise ValueError("centring is 'fixed', 'com' or 'density'")
        if len(self.levels) == 1 and centring != "fixed":
            raise ValueError("a single grid is the fixed global grid")
        self.centring = centring
        self.centre = np.asarray(centre, dtype=np.float64)

    @property
    def n_levels(self):
        return len(self.levels)


def validate_hierarchy(h: Hierarchy, first_galaxy: bool = True):
    """Eq. 9 and nesting checks; raises ValueError on an invalid hierarchy."""
    if h.n_levels == 1:
        if h.levels[0].q != 1.0 and not first_galaxy:
            raise ValueError("q < 1 applies only to the first galaxy")
        return
    L1, L2, L3 = h.levels
    if not (L1.R < L2.R < L3.R):
        raise ValueError("levels must nest: R1 < R2 < R3")
    for L in (L1, L2, L3):
        if not (0.0 < L.q <= 1.0):
            raise ValueError("0 < q <= 1")
    if L3.q != 1.0:
        raise ValueError("the global grid is not flattened")
    if not first_galaxy and (L1.q != 1.0 or L2.q != 1.0):
        raise ValueError("q < 1 applies only to the first galaxy (Sec. 2.2.2)")
    qc = q_crit(L2.N, L1.R, L2.R, L3.R)
    if L2.q < qc:
        raise ValueError(f"q={L2.q} below q_crit={qc} (Eq. 9)")
    if L2.q * L2.R < L1.q * L1.R:
        raise ValueError("flattened middle grid must still cover the inner grid")


# --------------------------------------------------------------------------
# Cell index (Eq. 7) and membership (Sec. 2.1 list of grids)
# --------------------------------------------------------------------------
def ngp_cell(x, centre, L: Level):
    """Nearest-grid-point cell of Eq. 7 for positions x (n,3) about `centre`.

    Returns (idx (n,3) int64, d (n,3) float64) with d = x - centre.
    u = (x - c) * gamma + N/2 is rounded after each operation; the cell is
    floor(u + 0.5).
    """
    d = x - centre
    u = d * L.gammas
    u = u + (L.N / 2.0)
    idx = np.floor(u + 0.5).astype(np.int64)
    return idx, d


def in_usable(idx, N):
    """All three indices inside [2, N-3] (two empty cells each side)."""
    return np.all((idx >= 2) & (idx <= N - 3), axis=1)


def spheroid_r2(d, inv_q):
    dzq = d[:, 2] * inv_q
    return d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + dzq * dzq


def classify(x, h: Hierarchy, centre):
    """Class of each particle relative to one galaxy's grids.

    Three levels: core iff r1 < R1 and the cell is usable on all three levels;
    else ring iff r2 < R2 and usable on the middle and outer levels; else
    outer iff usable on the outer level; else lost.  One level: outer iff
    usable, else lost.  Returns (cls, [idx per level]).
    """
    n = x.shape[0]
    if h.n_levels == 1:
        L = h.levels[0]
        idx, _ = ngp_cell(x, centre, L)
        cls = np.where(in_usable(idx, L.N), OUTER, LOST).astype(np.int8)
        return cls, [idx]
    L1, L2, L3 = h.levels
    i1, d = ngp_cell(x, centre, L1)
    i2, _ = ngp_cell(x, centre, L2)
    i3, _ = ngp_cell(x, L3.centre, L3)
    ok1, ok2, ok3 = in_usable(i1, L1.N), in_usable(i2, L2.N), in_usable(i3, L3.N)
    core = (spheroid_r2(d, L1.inv_q) < L1.R2) & ok1 & ok2 & ok3
    ring = ~core & (spheroid_r2(d, L2.inv_q) < L2.R2) & ok2 & ok3
    outer = ~core & ~ring & ok3
    cls = np.full(n, LOST, dtype=np.int8)
    cls[outer] = OUTER
    cls[ring] = RING
    cls[core] = CORE
    return cls, [i1, i2, i3]


def level_centre(h: Hierarchy, k: int, gal_centre):
    """Centre of level k: the galaxy centre for inner/middle, fixed for outer."""
    if h.n_levels == 3 and k == 2:
        return h.levels[2].centre
    return gal_centre


def centre_of_mass(x, m, mask):
    """Centre of mass of the selected particles (Sec. 2.1 alternative centring):
    sum m x / sum m in float64 (numpy's summation order).
    """
    mm = m[mask]
    return (x[mask] * mm[:, None]).sum(axis=0) / mm.sum()


def density_mass_shift(m):
    """Binary scale of the exact integer cell masses of density_max_centre.

    s = 62 - e - b, where m_max < 2^e (e from frexp of the largest particle
    mass of the whole set, lost and other galaxies included) and b is the
    bit length of the particle count n, so n * m_max * 2^s < 2^62: every cell
    total of the integers floor(m * 2^s) fits in 62 bits.
    """
    n = int(m.shape[0])
    e = int(np.frexp(np.max(m))[1]) if n > 0 else 0
    return 62 - e - n.bit_length()


def density_max_centre(x, m, mask, L: Level, prev_centre, shift):
    """Density maximum of one galaxy (Sec. 2.1: the inner and middle grids
    follow the galaxy's density maximum).  Parity unpinned beyond the pins of
    the test suite: the paper does not say how the maximum is located.

    Reading: the selected particles' masses are binned on the cells of Eq. 7
    of the galaxy's inner grid placed at the previous centre (all N^3 cells,
    not only the usable ones).  Each mass enters as the integer
    floor(m * 2^shift), so the cell totals are exact and independent of the
    summation order.  The densest cell is the one with the largest total;
    ties go to the lowest (z, y, x) index.  The centre is the FP64 centre of
    mass of the selected particles in the 3x3x3 block of cells around it.
    With no selected particle on the grid the previous centre is kept.
    """
    prev = np.asarray(prev_centre, dtype=np.float64)
    N = L.N
    xs, ms = x[mask], m[mask]
    idx, _ = ngp_cell(xs, prev, L)
    on = np.all((idx >= 0) & (idx < N), axis=1)
    if not on.any():
        return prev.copy()
    q = np.floor(np.ldexp(ms[on], shift)).astype(np.int64)
    io = idx[on]
    lin = (io[:, 2] * N + io[:, 1]) * N + io[:, 0]
    hist = np.zeros(N ** 3, dtype=np.int64)
    np.add.at(hist, lin, q)
    if hist.max() <= 0:
        return prev.copy()
    best = int(np.argmax(hist))            # first maximum: lowest (z, y, x)
    b = np.array([best % N, (best // N) % N, best // (N * N)])
    win = np.all(np.abs(idx - b) <= 1, axis=1) & on
    mw = ms[win]
    return (xs[win] * mw[:, None]).sum(axis=0) / mw.sum()


# --------------------------------------------------------------------------
# Mass assignment (Eq. 7, Sec. 2.2.1 individual masses)
# --------------------------------------------------------------------------
def deposit(idx, m, N):
    """Cell masses M[ix, iy, iz] = sum of m over particles in that NGP cell."""
    flat = (idx[:, 0] * N + idx[:, 1]) * N + idx[:, 2]
    return np.bincount(flat, weights=m, minlength=N ** 3).reshape(N, N, N)


def deposit_fixed(idx, m, N, shift):
    """The fixed-point reading of the same cell masses (reading: cell masses
    that do not depend on the order of the additions).  Each mass becomes the
    integer floor(m 2^shift) (exact in float64 for a power-of-two scale),
    the integers are summed exactly per cell, and each total is converted
    once to float64 (rounded to nearest) and scaled by 2^-shift.  With shift
    from density_mass_shift of the whole particle set, no total reaches 2^62.
    """
    q = np.floor(np.ldexp(np.asarray(m, np.float64), shift)).astype(np.int64)
    flat = (idx[:, 0] * N + idx[:, 1]) * N + idx[:, 2]
    tot = np.zeros(N ** 3, np.int64)
    np.add.at(tot, flat, q)
    return np.ldexp(tot.astype(np.float64), -shift).reshape(N, N, N)


# --------------------------------------------------------------------------
# Green's function and the isolated solve (Eqs. 1-5)
# --------------------------------------------------------------------------
def cell_mean_inverse_distance(lx, ly, lz):
    """Mean of 1/r over a cell of sides (lx, ly, lz) about its centre.

    The integral of 1/r over the box [0,a] x [0,b] x [0,c] with r measured
    from a corner is the textbook potential of a uniform rectangular prism,
      F = bc asinh(a / sqrt(b^2 + c^2)) + ac asinh(b / sqrt(a^2 + c^2))
        + ab asinh(c / sqrt(a^2 + b^2)) - a^2/2 atan(bc / (a r))
        - b^2/2 atan(ac / (b r)) - c^2/2 atan(ab / (c r)),  r = |(a, b, c)|;
    the cell is eight such octants of half-sides.
    """
    a, b, c = 0.5 * lx, 0.5 * ly, 0.5 * lz
    r = np.sqrt(a * a + b * b + c * c)
    F = (b * c * np.arcsinh(a / np.hypot(b, c)) + a * c * np.arcsinh(b / np.hypot(a, c))
         + a * b * np.arcsinh(c / np.hypot(a, b)) - 0.5 * a * a * np.arctan(b * c / (a * r))
         - 0.5 * b * b * np.arctan(a * c / (b * r)) - 0.5 * c * c * np.arctan(a * b / (c * r)))
    return float(8.0 * F / (lx * ly * lz))


def h0_value(L: Level, h0_mode: int) -> float:
    """H(0,0,0), which Eq. 2 leaves singular: H(1,0,0) = 1/l (h0_mode 0), the
    mean of 1/r over the cell (h0_mode 1, the cell's own mass spread
    uniformly), or 0 (h0_mode 2)."""
    if h0_mode == 0:
        return 1.0 / L.l
    if h0_mode == 1:
        return cell_mean_inverse_distance(L.l, L.l, L.lz)
    if h0_mode == 2:
        return 0.0
    raise ValueError("h0_mode must be 0 (H(1,0,0)), 1 (cell mean) or 2 (zero)")


def green_table(L: Level, h0_mode: int = 0):
    """H(a,b,c) of Eq. 2 for lags 0..N per axis, physical distances."""
    a = np.arange(L.N + 1, dtype=np.float64)
    X = (a * L.l)[:, None, None]
    Y = (a * L.l)[None, :, None]
    Z = (a * L.lz)[None, None, :]
    r = np.sqrt(X * X + Y * Y + Z * Z)
    with np.errstate(divide="ignore"):
        H = 1.0 / r
    H[0, 0, 0] = h0_value(L, h0_mode)
    return H


def green_extended(L: Level, h0_mode: int = 0):
    """H on the doubled (2N)^3 grid by the mirror symmetry of Eq. 5."""
    N = L.N
    k = np.arange(2 * N)
    fold = np.minimum(k, 2 * N - k)
    H = green_table(L, h0_mode)
    return H[fold[:, None, None], fold[None, :, None], fold[None, None, :]]


def green_hat(L: Level, h0_mode: int = 0):
    """DFT of the extended Green's function (real and even, Sec. 2.1).

    Returns (Hhat real (2N)^3, max|Im| / max|Re|).
    """
    F = _fft.fftn(green_extended(L, h0_mode), workers=_FFT_WORKERS)
    rel_imag = float(np.abs(F.imag).max() / np.abs(F.real).max())
    return F.real.copy(), rel_imag


def solve_fft(M, Hhat, G=1.0):
    """Isolated potential by the doubled-grid DFT convolution (Eqs. 3-5).

    M is the N^3 cell-mass grid of the active region; the (2N)^3 work grid is
    zero outside it; Phi is kept only on the active grid.
    """
    N = M.shape[0]
    P = np.zeros((2 * N,) * 3)
    P[:N, :N, :N] = M
    rho_hat = _fft.rfftn(P, workers=_FFT_WORKERS)
    prod = rho_hat * Hhat[:, :, : N + 1]
    return G * _fft.irfftn(prod, s=P.shape, axes=(0, 1, 2), workers=_FFT_WORKERS)[:N, :N, :N]


def solve_direct(M, L: Level, G=1.0, h0_mode: int = 0):
    """Eq. 1 summed directly: Phi[a] = G sum_xi M[xi] H(xi - a).  O(N^6)."""
    N = L.N
    H = green_table(L, h0_mode)
    ar = np.arange(N)
    Phi = np.zeros((N, N, N))
    for (i, j, k) in np.argwhere(M != 0.0):
        Phi += M[i, j, k] * H[np.abs(ar - i)[:, None, None],
                              np.abs(ar - j)[None, :, None],
                              np.abs(ar - k)[None, None, :]]
    return G * Phi


# --------------------------------------------------------------------------
# Force (Eq. 8) and the potential at a particle
# --------------------------------------------------------------------------
def _stencil(Phi, idx):
    i, j, k = idx[:, 0], idx[:, 1], idx[:, 2]

    def P(di, dj, dk):
        return Phi[i + di, j + dj, k + dk]
    return P


def _derivs(Phi, idx, lengths):
    """First and second differences of Eq. 8 at the cell centre.

    D[a]    = (P(+a) - P(-a)) / (2 l_a)
    DD[a,a] = (P(+a) + P(-a) - 2 P0) / l_a^2
    DD[a,b] = (P(+a+b) - P(-a+b) + P(-a-b) - P(+a-b)) / (4 l_a l_b)
    """
    P = _stencil(Phi, idx)
    e = np.eye(3, dtype=np.int64)
    P0 = P(0, 0, 0)
    D = np.empty((3, idx.shape[0]))
    DD = np.empty((3, 3, idx.shape[0]))
    for a in range(3):
        pa = P(*e[a])
        ma = P(*(-e[a]))
        D[a] = (pa - ma) / (2.0 * lengths[a])
        DD[a, a] = (pa + ma - 2.0 * P0) / (lengths[a] * lengths[a])
        for b in range(3):
            if b == a:
                continue
            DD[a, b] = (P(*(e[a] + e[b])) - P(*(-e[a] + e[b])) + P(*(-e[a] - e[b]))
                        - P(*(e[a] - e[b]))) / (4.0 * lengths[a] * lengths[b])
    return P0, D, DD


def cell_offset(d, idx, L: Level):
    """Position inside the cell: Delta = (x - c) - (idx - N/2) * l, per axis."""
    return d - (idx - L.N / 2.0) * L.lengths


def eq8_accel(Phi, idx, delta, lengths, taylor=True):
    """Acceleration of Eq. 8 (x component and its cyclic permutations).

    a_a = D_a + DD_aa Delta_a + sum_{b != a} DD_ab Delta_b, a = +grad Phi_paper.
    taylor=False keeps only the central difference D_a.
    """
    _, D, DD = _derivs(Phi, idx, lengths)
    if not taylor:
        return D.T.copy()
    acc = np.empty((idx.shape[0], 3))
    for a in range(3):
        acc[:, a] = D[a] + sum(DD[a, b] * delta[:, b] for b in range(3))
    return acc


def taylor_potential(Phi, idx, delta, lengths, taylor=True):
    """Phi_paper at the particle: the quadratic whose gradient is Eq. 8.

    P0 + sum_a D_a Delta_a + 1/2 sum_ab DD_ab Delta_a Delta_b (the paper does
    not say how the potential at a particle is read off the grid; this form is
    exact, like Eq. 8, on a field that is quadratic in position).
    """
    P0, D, DD = _derivs(Phi, idx, lengths)
    if not taylor:
        return P0 + sum(D[a] * delta[:, a] for a in range(3))
    phi = P0.copy()
    for a in range(3):
        phi += D[a] * delta[:, a]
        for b in range(3):
            phi += 0.5 * DD[a, b] * delta[:, a] * delta[:, b]
    return phi


def leapfrog_kd(x, v, acc, dt):
    """Leapfrog of Eq. 6 with staggered velocities: kick, then drift.

    v(t + dt/2) = v(t - dt/2) + dt a(t);  x(t + dt) = x(t) + dt v(t + dt/2).
    """
    v_new = v + dt * acc
    return x + dt * v_new, v_new


# --------------------------------------------------------------------------
# The five grids of one galaxy and the grid-selection rule (Sec. 2.1)
# --------------------------------------------------------------------------
class System:
    """Galaxies with their grids, Green's tables and the per-step solve."""

    def __init__(self, hierarchies, G=1.0, h0_mode=0, taylor=True, fixed_deposit=False):
        self.h = list(hierarchies)
        self.fixed_deposit = fixed_deposit  # cell masses by deposit_fixed
        for g, hh in enumerate(self.h):
            validate_hierarchy(hh, first_galaxy=(g == 0))
        if len(self.h) > 1:
            ref = self.h[0]
            for hh in self.h:
                if hh.n_levels != 3 or not hh.levels[2].same_geometry(ref.levels[2]):
                    raise ValueError("several galaxies need 3 levels sharing the global grid")
        self.G = float(G)
        self.h0_mode = h0_mode
        self.taylor = taylor
        self.hhat = {}
        for hh in self.h:
            for L in hh.levels:
                key = (L.N, L.R, L.q)
                if key not in self.hhat:
                    self.hhat[key] = green_hat(L, h0_mode)[0]

    def solve(self, M, L: Level):
        return solve_fft(M, self.hhat[(L.N, L.R, L.q)], self.G)

    # -- per galaxy --------------------------------------------------------
    def centres(self, x, m, gal, lost, prev=None):
        """Centres of the inner and middle grids of every galaxy.

        `prev` (per galaxy) is the centre of the previous solve, used by
        density centring; the hierarchy's own centre when None.
        """
        c = []
        for g, hh in enumerate(self.h):
            if hh.centring == "com":
                c.append(centre_of_mass(x, m, (gal == g) & ~lost))
            elif hh.centring == "density":
                p = hh.centre if prev is None else prev[g]
                c.append(density_max_centre(x, m, (gal == g) & ~lost, hh.levels[0], p,
                                            density_mass_shift(m)))
            else:
                c.append(hh.centre.copy())
        return c

    def potentials(self, x, m, gal, lost, centres):
        """Grids 1..5 of each galaxy, solved separately as in the paper.

        Returns, per galaxy, dict with 'cls'/'idx' for its own particles and
        'Phi' = [Phi1..Phi5] (three levels) or [Phi] (one level), plus 'M'.
        """
        out = []
        if self.fixed_deposit:
            shift = density_mass_shift(np.asarray(m, np.float64))
            deposit = lambda i, w, N: deposit_fixed(i, w, N, shift)  # noqa: E731
        else:
            deposit = globals()["deposit"]
        for g, hh in enumerate(self.h):
            sel = (gal == g) & ~lost
            xs, ms = x[sel], m[sel]
            cls, idx = classify(xs, hh, centres[g])
            if hh.n_levels == 1:
                L = hh.levels[0]
                ok = cls == OUTER
                M = deposit(idx[0][ok], ms[ok], L.N)
                out.append({"M": [M], "Phi": [self.solve(M, L)]})
                continue
            L1, L2, L3 = hh.levels
            core, ring, outer = cls == CORE, cls == RING, cls == OUTER
            M1 = deposit(idx[0][core], ms[core], L1.N)          # grid 1: core
            M2 = deposit(idx[1][core], ms[core], L2.N)          # grid 2: core
            M3 = deposit(idx[1][ring], ms[ring], L2.N)          # grid 3: ring
            cr = core | ring
            M4 = deposit(idx[2][cr], ms[cr], L3.N)              # grid 4: r < R_out
            M5 = deposit(idx[2][outer], ms[outer], L3.N)        # grid 5: outside
            Ms = [M1, M2, M3, M4, M5]
            Ls = [L1, L2, L2, L3, L3]
            out.append({"M": Ms, "Phi": [self.solve(Mk, Lk) for Mk, Lk in zip(Ms, Ls)]})
        return out

    def accel(self, x, m, gal, lost, centres=None, pots=None, want_pot=False):
        """Acceleration (and Phi_paper) of every non-lost particle.

        For each galaxy: core -> Phi1 + Phi3 + Phi5, ring -> Phi2 + Phi3 +
        Phi5, outer -> Phi4 + Phi5, each field differenced on its own grid;
        accelerations of the galaxies add up (Sec. 2.1).
        """
        if centres is None:
            centres = self.centres(x, m, gal, lost)
        if pots is None:
            pots = self.potentials(x, m, gal, lost, centres)
        n = x.shape[0]
        acc = np.zeros((n, 3))
        phi = np.zeros(n)
        live = ~lost
        a_l, p_l = self.field_at(x[live], centres, pots)
        acc[live] = a_l
        phi[live] = p_l
        if want_pot:
            return acc, phi
        return acc

    def field_at(self, xl, centres, pots):
        """Acceleration and Phi_paper at positions xl from solved fields."""
        a_l = np.zeros((xl.shape[0], 3))
        p_l = np.zeros(xl.shape[0])
        for g, hh in enumerate(self.h):
            cls, idx = classify(xl, hh, centres[g])
            Phi = pots[g]["Phi"]
            if hh.n_levels == 1:
                terms = [(cls == OUTER, 0, Phi[0])]
            else:
                core, ring, outer = cls == CORE, cls == RING, cls == OUTER
                terms = [(core, 0, Phi[0]), (core, 1, Phi[2]), (core, 2, Phi[4]),
                         (ring, 1, Phi[1] + Phi[2]), (ring, 2, Phi[4]),
                         (outer, 2, Phi[3] + Phi[4])]
            for mask, k, F in terms:
                if not mask.any():
                    continue
                L = hh.levels[k]
                c = level_centre(hh, k, centres[g])
                ii = idx[k][mask]
                dl = cell_offset(xl[mask] - c, ii, L)
                a_l[mask] += eq8_accel(F, ii, dl, L.lengths, self.taylor)
                p_l[mask] += taylor_potential(F, ii, dl, L.lengths, self.taylor)
        return a_l, p_l

    # -- loss and stepping ---------------------------------------------------
    def lost_now(self, x):
        """Outside the usable cells of the outermost (fixed, global) grid."""
        hh = self.h[0]
        L = hh.levels[-1]
        c = L.centre if hh.n_levels == 3 else hh.centre
        idx, _ = ngp_cell(x, c, L)
        return ~in_usable(idx, L.N)

    def step(self, x, v, m, gal, lost, dt, prev_centres=None):
        """One integration cycle (Sec. 2.1): fields, Eq. 8, leapfrog of Eq. 6.

        Loss: particles outside the global grid at the start of the step (only
        possible for the initial positions) and after the drift are flagged
        lost and never move, deposit or feel a force again.  The centres are
        taken after the start-of-step loss test (density centring starts from
        prev_centres, the centres of the previous step); they are kept in
        self.last_centres.
        Returns new (x, v, lost) and the accelerations used.
        """
        x = x.copy(); v = v.copy(); lost = lost.copy()
        lost |= self.lost_now(x)
        centres = self.centres(x, m, gal, lost, prev_centres)
        self.last_centres = centres
        acc = self.accel(x, m, gal, lost, centres)
        live = ~lost
        x[live], v[live] = leapfrog_kd(x[live], v[live], acc[live], dt)
        lost |= live & self.lost_now(x)
        return x, v, lost, acc

    # -- diagnostics -----------------------------------------------------------
    def diagnostics(self, x, v, m, comp, gal, lost, dt, n_comp=8, prev_centres=None):
        """FP64 energy and angular momentum per component, disc dispersions.

        Taken at the start of a step: particles outside the global grid are
        lost first (the step's start-of-step loss test, Sec. 2.1).  v is the
        staggered v(t - dt/2); the synchronised velocity is v + dt/2 * a(t).
        W_c = 1/2 sum m phi with phi = -Phi_paper at the particle; L_c = sum
        m x cross v_sync about the origin.  Disc (component 0 of galaxy 0)
        sigma_R and sigma_z about their means (unweighted), R measured from
        galaxy 0's centre.
        """
        lost = lost | self.lost_now(x)
        centres = self.centres(x, m, gal, lost, prev_centres)
        acc, Pp = self.accel(x, m, gal, lost, centres, want_pot=True)
        live = ~lost
        vs = v + 0.5 * dt * acc
        ekin = np.zeros(n_comp); epot = np.zeros(n_comp); L = np.zeros((n_comp, 3))
        for c in range(n_comp):
            s = live & (comp == c)
            if not s.any():
                continue
            ms = m[s]
            ekin[c] = 0.5 * np.sum(ms * np.sum(vs[s] * vs[s], axis=1))
            epot[c] = 0.5 * np.sum(ms * (-Pp[s]))
            L[c] = np.sum(ms[:, None] * np.cross(x[s], vs[s]), axis=0)
        disc = live & (comp == 0) & (gal == 0)
        sR = sz = 0.0
        if disc.any():
            d = x[disc] - centres[0]
            R = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
            vR = (d[:, 0] * vs[disc, 0] + d[:, 1] * vs[disc, 1]) / R
            vz = vs[disc, 2]
            sR = float(np.sqrt(max(np.mean(vR * vR) - np.mean(vR) ** 2, 0.0)))
            sz = float(np.sqrt(max(np.mean(vz * vz) - np.mean(vz) ** 2, 0.0)))
        return {"ekin": ekin, "epot": epot, "L": L, "disc_sigR": sR, "disc_sigz": sz,
                "n_lost": int(lost.sum()), "centres": centres}


# --------------------------------------------------------------------------
# Adjoint of a leapfrog segment (reverse mode of Eqs. 1-8 and 6)
# --------------------------------------------------------------------------
def eq8_scatter_transpose(B, idx, delta, lengths, mu, taylor=True):
    """B += A^T mu: the transpose of the Eq. 8 gather for per-particle vectors
    mu (n,3).  A maps a field to the accelerations of the particles; its
    transpose spreads mu over the 19 stencil points with the same weights."""
    lx, ly, lz = lengths
    i, j, k = idx[:, 0], idx[:, 1], idx[:, 2]
    e = np.eye(3, dtype=np.int64)

    def add(off, w):
        np.add.at(B, (i + off[0], j + off[1], k + off[2]), w)
    ln = np.array([lx, ly, lz])
    for a in range(3):
        add(e[a], mu[:, a] / (2.0 * ln[a]))
        add(-e[a], -mu[:, a] / (2.0 * ln[a]))
        if not taylor:
            continue
        w2 = mu[:, a] * delta[:, a] / (ln[a] * ln[a])
        add(e[a], w2)
        add(-e[a], w2)
        add(np.zeros(3, np.int64), -2.0 * w2)
        for b in range(3):
            if b == a:
                continue
            w = mu[:, a] * delta[:, b] / (4.0 * ln[a] * ln[b])
            add(e[a] + e[b], w)
            add(-e[a] + e[b], -w)
            add(-e[a] - e[b], w)
            add(e[a] - e[b], -w)


def eq8_jacobian(Phi, idx, lengths, taylor=True):
    """d a / d x of Eq. 8 inside a cell: the matrix of second differences."""
    _, _, DD = _derivs(Phi, idx, lengths)
    if not taylor:
        return np.zeros((idx.shape[0], 3, 3))
    return np.transpose(DD, (2, 0, 1))


def segment_loss_and_grads(sysm: System, x, v, m, comp, gal, dt, nsteps, sel_comp=0, sel_gal=0,
                           lost0=None):
    """Forward: nsteps integration cycles (Eq. 6 with the fields of Sec. 2.1)
    from the state (x, v, lost0); loss L = sum over the selected particles
    (component sel_comp of galaxy sel_gal) still on the grids at the end of
    1/2 m v_z^2, with the staggered v after the last kick.  Backward: reverse
    mode of the discrete cycles.

    Particle loss (Sec. 2.1) is part of the forward: the particles that take
    part in cycle k are those live after that cycle's start-of-step loss
    test.  The reverse of cycle k re-solves the fields from exactly those
    particles, so a particle that leaves during the segment still receives
    dL/dm from the cycles in which its mass shaped the fields; a particle that
    sits out a cycle passes its adjoints through it unchanged.  The
    nearest-grid-point cells and the loss test are piecewise constant, so
    only the in-cell offsets of Eq. 8 carry a position derivative (almost
    everywhere).  Fixed centres only.  Returns (L, dL/dm, dL/dx0, dL/dv0).
    parity unpinned beyond its finite-difference and transpose pins."""
    for hh in sysm.h:
        if hh.centring != "fixed":
            raise ValueError("the segment adjoint needs fixed centres")
    lost = np.zeros(x.shape[0], bool) if lost0 is None else np.asarray(lost0, bool).copy()
    xs, lives = [], []
    xk, vk = x.copy(), v.copy()
    for _ in range(nsteps):
        # participants of this cycle: live after its start-of-step loss test
        lives.append(~(lost | sysm.lost_now(xk)))
        xs.append(xk.copy())
        xk, vk, lost, _ = sysm.step(xk, vk, m, gal, lost, dt)
    # particles lost by the end have left the system (Sec. 2.1): not counted
    sel = (comp == sel_comp) & (gal == sel_gal) & ~lost
    L = 0.5 * np.sum(m[sel] * vk[sel, 2] ** 2)
    gm = np.zeros_like(m)
    gm[sel] = 0.5 * vk[sel, 2] ** 2
    lx = np.zeros_like(x)
    lv = np.zeros_like(v)
    lv[sel, 2] = m[sel] * vk[sel, 2]
    for k in range(nsteps - 1, -1, -1):
        live = lives[k]
        out_k = ~live
        # reverse drift (x' = x + dt v'), then reverse kick (v' = v + dt a(x))
        lv = np.where(live[:, None], lv + dt * lx, lv)
        mu = np.where(live[:, None], dt * lv, 0.0)
        xk = xs[k]
        centres = sysm.centres(xk, m, gal, out_k)
        pots = sysm.potentials(xk, m, gal, out_k, centres)
        for g, hh in enumerate(sysm.h):
            cls, idx = classify(xk, hh, centres[g])
            Phi = pots[g]["Phi"]
            nl = hh.n_levels
            if nl == 1:
                terms = [(cls == OUTER, 0, [0])]
            else:
                core, ring, outer = cls == CORE, cls == RING, cls == OUTER
                # (particles, level, grids whose sum is the field)
                terms = [(core, 0, [0]), (core, 1, [2]), (core, 2, [4]),
                         (ring, 1, [1, 2]), (ring, 2, [4]), (outer, 2, [3, 4])]
            Bs = [np.zeros_like(P) for P in Phi]
            for mask, lev, grids in terms:
                msk = mask & live
                if not msk.any():
                    continue
                L_ = hh.levels[lev]
                c = level_centre(hh, lev, centres[g])
                ii = idx[lev][msk]
                dl = cell_offset(xk[msk] - c, ii, L_)
                F = sum(Phi[q] for q in grids)
                J = eq8_jacobian(F, ii, L_.lengths, sysm.taylor)
                lx[msk] += np.einsum("nab,nb->na", J, mu[msk])
                Bt = np.zeros_like(F)
                eq8_scatter_transpose(Bt, ii, dl, L_.lengths, mu[msk], sysm.taylor)
                for q in grids:
                    Bs[q] += Bt
            # mass gradient: psi = K B on each grid, read at the source cells
            # of the particles that deposited in this cycle
            own = (gal == g) & live
            if nl == 1:
                psi = sysm.solve(Bs[0], hh.levels[0])
                ok = own & (cls == OUTER)
                gm[ok] += psi[tuple(idx[0][ok].T)]
                continue
            L1, L2, L3 = hh.levels
            psis = [sysm.solve(Bs[0], L1), sysm.solve(Bs[1], L2), sysm.solve(Bs[2], L2),
                    sysm.solve(Bs[3], L3), sysm.solve(Bs[4], L3)]
            core, ring, outer = own & (cls == CORE), own & (cls == RING), own & (cls == OUTER)
            gm[core] += psis[0][tuple(idx[0][core].T)]     # grid 1
            gm[core] += psis[1][tuple(idx[1][core].T)]     # grid 2
            gm[ring] += psis[2][tuple(idx[1][ring].T)]     # grid 3
            cr = core | ring
            gm[cr] += psis[3][tuple(idx[2][cr].T)]         # grid 4
            gm[outer] += psis[4][tuple(idx[2][outer].T)]   # grid 5
    return L, gm, lx, lv


# --------------------------------------------------------------------------
# Disc diagnostics of the paper's analysis (Sec. 4.2 and 5.2-5.4: heat, thickness,
# vertical profile, velocity dispersions near the solar radius)
# --------------------------------------------------------------------------
def disc_analysis(x, v, m, comp, gal, lost, centre, n_bins, annulus, n_z, z_max,
                  disc_comp=0, disc_gal=0):
    """Diagnostics of the disc (live particles of component disc_comp of
    galaxy disc_gal), with positions relative to `centre` and velocities
    relative to the disc's mass-weighted mean velocity.

    * Radial bins of equal particle numbers (Sec. 4.2 and 5.3): particles
      ordered by cylindrical R (ties by particle index), bin k holding
      n // n_bins particles plus one for k < n % n_bins.  Per bin: mean R,
      mean circular velocity (mean v_phi) and RMS z (sqrt of mean z^2).
    * Heat (Sec. 5.3, Eq. 14): E = sum 1/2 m |v - vbar_c(R)|^2, with vbar_c the bin
      values linearly interpolated in R between the bins' mean radii (held
      constant beyond the first and last) and directed along phi.
    * In the annulus R_lo <= R < R_hi: sigma_R, sigma_phi, sigma_z (about the
      annulus means), sigma_tot^2, and the vertical density profile: mass in
      n_z equal bins of z over [-z_max, z_max) divided by the annulus area
      times the bin width (Sec. 4.2 and 5.2).
    Unweighted means over particles (the disc particles have equal masses in
    the paper's models).  parity unpinned beyond its closed-form pins.
    """
    sel = (comp == disc_comp) & (gal == disc_gal) & ~lost
    idx = np.nonzero(sel)[0]
    d = x[idx] - np.asarray(centre, dtype=np.float64)
    ms = m[idx]
    vb = np.sum(ms[:, None] * v[idx], axis=0) / np.sum(ms)
    u = v[idx] - vb
    dx, dy, z = d[:, 0], d[:, 1], d[:, 2]
    R = np.sqrt(dx * dx + dy * dy)
    with np.errstate(invalid="ignore", divide="ignore"):
        vR = np.where(R > 0, (dx * u[:, 0] + dy * u[:, 1]) / R, 0.0)
        vphi = np.where(R > 0, (dx * u[:, 1] - dy * u[:, 0]) / R, 0.0)
    vz = u[:, 2]
    n = R.shape[0]
    order = np.argsort(R, kind="stable")
    base, extra = divmod(n, n_bins)
    sizes = np.array([base + (1 if k < extra else 0) for k in range(n_bins)])
    starts = np.concatenate([[0], np.cumsum(sizes)])
    bin_r = np.zeros(n_bins); bin_vc = np.zeros(n_bins); bin_rms_z = np.zeros(n_bins)
    for k in range(n_bins):
        o = order[starts[k]:starts[k + 1]]
        if o.size == 0:
            continue
        bin_r[k] = np.mean(R[o])
        bin_vc[k] = np.mean(vphi[o])
        bin_rms_z[k] = np.sqrt(np.mean(z[o] ** 2))
    vc_at = np.interp(R, bin_r, bin_vc)
    heat = 0.5 * np.sum(ms * ((vR * vR + (vphi - vc_at) ** 2) + vz * vz))
    lo, hi = annulus
    a = (R >= lo) & (R < hi)
    na = int(a.sum())

    def sd(q):
        return float(np.sqrt(max(np.mean(q * q) - np.mean(q) ** 2, 0.0))) if na else 0.0
    sR, sphi, sz = sd(vR[a]), sd(vphi[a]), sd(vz[a])
    dz = 2.0 * z_max / n_z
    area = np.pi * (hi * hi - lo * lo)
    hz = np.zeros(n_z)
    za = z[a]
    inz = (za >= -z_max) & (za < z_max)
    k = np.floor((za[inz] + z_max) / dz).astype(int)
    k = np.minimum(k, n_z - 1)
    np.add.at(hz, k, ms[a][inz])
    rho_z = hz / (area * dz)
    return {"n_disc": n, "bulk_v": vb, "bin_r": bin_r, "bin_vc": bin_vc, "bin_rms_z": bin_rms_z,
            "bin_sizes": sizes, "e_heat": heat, "sig_R": sR, "sig_phi": sphi, "sig_z": sz,
            "sig_tot2": sR * sR + sphi * sphi + sz * sz, "n_annulus": na, "rho_z": rho_z}


def disc_modes(x, m, comp, gal, lost, centre, n_rbins, r_max, m_max, disc_comp=0, disc_gal=0):
    """Fourier coefficients of the disc's surface density (Sec. 5.6): in
    annular bins [k dR, (k+1) dR), A_m = (1/S_k) sum M exp(-i m phi) over the
    bin's particles, phi the polar angle about `centre`, S_k the bin area.
    Returns an (n_rbins, m_max + 1) complex array.  parity unpinned beyond
    its closed-form pins."""
    sel = (comp == disc_comp) & (gal == disc_gal) & ~lost
    d = x[sel] - np.asarray(centre, dtype=np.float64)
    ms = m[sel]
    R = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1])
    ph = np.arctan2(d[:, 1], d[:, 0])
    dR = r_max / n_rbins
    out = np.zeros((n_rbins, m_max + 1), complex)
    for k in range(n_rbins):
        b = (R >= k * dR) & (R < (k + 1) * dR)
        S = np.pi * dR * dR * ((k + 1) ** 2 - k ** 2)
        for q in range(m_max + 1):
            out[k, q] = np.sum(ms[b] * np.exp(-1j * q * ph[b])) / S
    return out
