"""Seeded synthetic inputs: particle models and grid set-ups of the workloads.

This module draws particles; it holds none of the field-solve arithmetic and
is the only code shared by the oracle tests and the GPU tests/benchmark.

Models follow the paper's Sec. 3 (exponential-sech^2 disc, cropped Hernquist
bulge, Plummer satellite, Table 2 mass ratios) in units of the disc scale
length h = 1 and disc mass M_disc = 1, G = 1.  The paper's galaxy was built by
an external generator and then relaxed; here velocities come from Jeans-moment
approximations, so the "equilibrium" is approximate by design.

Seeds: numpy SeedSequence([1210, 1736, workload, component]).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# component ids
DISC, BULGE, HALO, SAT = 0, 1, 2, 3


def rng_for(workload: int, component: int):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, workload, component]))


# --------------------------------------------------------------------------
# grid set-ups (plain data; the library and the oracle each interpret them)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class LevelSpec:
    N: int
    R: float
    q: float = 1.0


@dataclasses.dataclass
class HierSpec:
    levels: list
    centring: str = "fixed"          # 'fixed', 'com' or 'density'
    centre: tuple = (0.0, 0.0, 0.0)  # fixed centre (inner/middle if fixed; single grid)
    outer_centre: tuple = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray        # (n,3) float64
    v: np.ndarray        # (n,3) float64, v(t - dt/2)
    m: np.ndarray        # (n,)  float64
    comp: np.ndarray     # (n,)  int8
    gal: np.ndarray      # (n,)  int8
    hier: list           # [HierSpec] per galaxy
    dt: float
    steps: int
    G: float = 1.0

    @property
    def n(self):
        return self.x.shape[0]


# --------------------------------------------------------------------------
# spherical profiles
# --------------------------------------------------------------------------
def _iso_dirs(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def plummer_positions(rng, n, a, r_cut):
    """Radii by the inverse cumulative mass of a Plummer sphere, cut at r_cut."""
    u_max = r_cut ** 3 / (r_cut ** 2 + a ** 2) ** 1.5
    u = rng.uniform(0.0, u_max, n)
    u = np.maximum(u, 1e-300)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    return r[:, None] * _iso_dirs(rng, n), r


def plummer_velocities(rng, r, M, a, G=1.0):
    """Isotropic speeds from the Plummer distribution function by rejection
    (Aarseth, Henon & Wielen 1974): q^2 (1 - q^2)^(7/2), v = q v_esc."""
    n = r.shape[0]
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = rng.uniform(0.0, 1.0, todo.size)
        y1 = rng.uniform(0.0, 0.1, todo.size)
        ok = y1 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0 * G * M) * (r * r + a * a) ** -0.25
    return (q * vesc)[:, None] * _iso_dirs(rng, n)


def hernquist_positions(rng, n, a, r_cut):
    uc = r_cut ** 2 / (r_cut + a) ** 2
    s = np.sqrt(rng.uniform(0.0, uc, n))
    r = a * s / (1.0 - s)
    return r[:, None] * _iso_dirs(rng, n), r


def nfw_mass(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw_positions(rng, n, rs, r_cut):
    grid = np.concatenate([[0.0], np.geomspace(1e-6 * rs, r_cut, 20000)])
    cdf = nfw_mass(grid / rs) / nfw_mass(r_cut / rs)
    r = np.interp(rng.uniform(0.0, 1.0, n), cdf, grid)
    return r[:, None] * _iso_dirs(rng, n), r


# --------------------------------------------------------------------------
# galaxy model (Sec. 3.1, Table 2 ratios, scaled to h = M_disc = 1)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class GalaxyModel:
    n_disc: int = 2_000_000
    n_bulge: int = 500_000
    n_halo: int = 6_000_000
    M_disc: float = 1.0
    M_bulge: float = 2.14 / 4.82     # Table 2
    M_halo: float = 20.0 / 4.82      # Table 2
    h: float = 1.0
    z0: float = 0.1
    R_max: float = 10.0
    z_max: float = 1.0
    a_bulge: float = 0.2             # 0.5 kpc / 2.5 kpc
    rc_bulge: float = 2.8            # 14 a
    rs_halo: float = 6.72            # 16.8 kpc / 2.5 kpc
    rc_halo: float = 18.0
    Q: float = 2.0
    R_Q: float = 3.2                 # 8 kpc / 2.5 kpc


def _disc_mass_frac(R, h, R_max):
    f = lambda x: 1.0 - (1.0 + x / h) * np.exp(-x / h)
    return f(R) / f(R_max)


def _enclosed_mass_fn(gm: GalaxyModel):
    """Spherical approximation of the total enclosed mass M(<r)."""
    def M(r):
        r = np.asarray(r, dtype=np.float64)
        md = gm.M_disc * _disc_mass_frac(np.minimum(r, gm.R_max), gm.h, gm.R_max)
        rb = np.minimum(r, gm.rc_bulge)
        mb = gm.M_bulge * (rb / (rb + gm.a_bulge)) ** 2 / (gm.rc_bulge / (gm.rc_bulge + gm.a_bulge)) ** 2
        rh = np.minimum(r, gm.rc_halo)
        mh = gm.M_halo * nfw_mass(rh / gm.rs_halo) / nfw_mass(gm.rc_halo / gm.rs_halo)
        return md + mb + mh
    return M


def _jeans_sigma(rho_fn, Menc, r_cut, G=1.0):
    """Isotropic Jeans dispersion sigma^2(r) = (1/rho) int_r^rc rho G M / r'^2 dr'."""
    rg = np.geomspace(1e-5, r_cut, 4000)
    f = rho_fn(rg) * G * Menc(rg) / rg ** 2
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(rg)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    s2 = tail / np.maximum(rho_fn(rg), 1e-300)
    return lambda r: np.interp(r, rg, s2)


def _spherical_velocities(rng, pos, r, rho_fn, Menc, r_cut):
    s2 = _jeans_sigma(rho_fn, Menc, r_cut)(r)
    return rng.normal(size=pos.shape) * np.sqrt(np.maximum(s2, 0.0))[:, None]


def disc_particles(rng, n, gm: GalaxyModel, Menc):
    # radius: Sigma ~ exp(-R/h), cut at R_max (inverse CDF by interpolation)
    Rg = np.linspace(0.0, gm.R_max, 200001)
    cdf = _disc_mass_frac(Rg, gm.h, gm.R_max)
    R = np.interp(rng.uniform(0.0, 1.0, n), cdf, Rg)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    # height: sech^2(z/z0) cut at |z| < z_max
    t = math.tanh(gm.z_max / gm.z0)
    z = gm.z0 * np.arctanh(rng.uniform(-t, t, n))
    pos = np.stack([R * np.cos(ph), R * np.sin(ph), z], axis=1)
    # kinematics (epicycle approximation)
    Rs = np.maximum(R, 1e-3)
    Om2 = Menc(Rs) / Rs ** 3
    dR = 1e-4 * np.maximum(Rs, 1e-2)
    dOm2 = (Menc(Rs + dR) / (Rs + dR) ** 3 - Menc(Rs - dR) / (Rs - dR) ** 3) / (2 * dR)
    kap2 = np.maximum(Rs * dOm2 + 4.0 * Om2, 1e-12)
    norm = 1.0 - (1.0 + gm.R_max / gm.h) * math.exp(-gm.R_max / gm.h)
    Sig = gm.M_disc / (2.0 * np.pi * gm.h ** 2 * norm) * np.exp(-Rs / gm.h)
    RQ = gm.R_Q
    Om2Q = Menc(RQ) / RQ ** 3
    dQ = 1e-4 * RQ
    kapQ = math.sqrt(RQ * (Menc(RQ + dQ) / (RQ + dQ) ** 3 - Menc(RQ - dQ) / (RQ - dQ) ** 3) / (2 * dQ) + 4 * Om2Q)
    SigQ = gm.M_disc / (2.0 * np.pi * gm.h ** 2 * norm) * math.exp(-RQ / gm.h)
    sR0 = gm.Q * 3.36 * SigQ / kapQ * math.exp(RQ / (2 * gm.h))
    sR = sR0 * np.exp(-Rs / (2 * gm.h))
    sz = np.sqrt(np.pi * Sig * gm.z0)
    sphi = sR * np.sqrt(kap2 / (4.0 * Om2))
    vc2 = Menc(Rs) / Rs
    vphi2 = vc2 - sR ** 2 * (sphi ** 2 / sR ** 2 - 1.0 + 2.0 * Rs / gm.h)
    vphi = np.sqrt(np.maximum(vphi2, 0.0))
    vR = rng.normal(size=n) * sR
    vp = vphi + rng.normal(size=n) * sphi
    vz = rng.normal(size=n) * sz
    c, s = np.cos(ph), np.sin(ph)
    vel = np.stack([vR * c - vp * s, vR * s + vp * c, vz], axis=1)
    return pos, vel


def galaxy(workload: int, gm: GalaxyModel):
    Menc = _enclosed_mass_fn(gm)
    xs, vs, ms, cs = [], [], [], []
    if gm.n_disc:
        p, v = disc_particles(rng_for(workload, DISC), gm.n_disc, gm, Menc)
        xs.append(p); vs.append(v); ms.append(np.full(gm.n_disc, gm.M_disc / gm.n_disc)); cs.append(np.full(gm.n_disc, DISC))
    if gm.n_bulge:
        rng = rng_for(workload, BULGE)
        p, r = hernquist_positions(rng, gm.n_bulge, gm.a_bulge, gm.rc_bulge)
        rho = lambda rr: 1.0 / (rr * (rr + gm.a_bulge) ** 3) * (rr < gm.rc_bulge)
        v = _spherical_velocities(rng, p, r, rho, Menc, gm.rc_bulge)
        xs.append(p); vs.append(v); ms.append(np.full(gm.n_bulge, gm.M_bulge / gm.n_bulge)); cs.append(np.full(gm.n_bulge, BULGE))
    if gm.n_halo:
        rng = rng_for(workload, HALO)
        p, r = nfw_positions(rng, gm.n_halo, gm.rs_halo, gm.rc_halo)
        rho = lambda rr: 1.0 / ((rr / gm.rs_halo) * (1.0 + rr / gm.rs_halo) ** 2) * (rr < gm.rc_halo)
        v = _spherical_velocities(rng, p, r, rho, Menc, gm.rc_halo)
        xs.append(p); vs.append(v); ms.append(np.full(gm.n_halo, gm.M_halo / gm.n_halo)); cs.append(np.full(gm.n_halo, HALO))
    return (np.concatenate(xs), np.concatenate(vs), np.concatenate(ms),
            np.concatenate(cs).astype(np.int8), Menc)


def point_mass_orbit(M_enclosed, R_A, e, incl_deg, G=1.0):
    """Apocentre position and velocity of a two-body ellipse (Sec. 5.1 set-up):
    v_A^2 = G M (1 - e) / R_A; the orbit plane is tilted by the inclination
    about the x axis; prograde for i < 90 degrees."""
    vA = math.sqrt(G * M_enclosed * (1.0 - e) / R_A)
    i = math.radians(incl_deg)
    return np.array([R_A, 0.0, 0.0]), np.array([0.0, vA * math.cos(i), vA * math.sin(i)])


def pericentre(R_A, e):
    return R_A * (1.0 - e) / (1.0 + e)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def plummer_cube(n=100_000, N=64, workload=1):
    """Single isolated 64^3 grid of side 10a, Plummer sphere G = M = a = 1."""
    rng = rng_for(workload, SAT)
    R = 5.0
    r_t = 4.5
    pos, r = plummer_positions(rng, n, 1.0, r_t)
    vel = plummer_velocities(rng, r, 1.0, 1.0)
    m = np.full(n, 1.0 / n)
    return Workload("plummer_64", pos, vel, m, np.full(n, SAT, np.int8),
                    np.zeros(n, np.int8), [HierSpec([LevelSpec(N, R, 1.0)])], dt=0.01, steps=10)


def disc_galaxy(scale=1.0, N=128, workload=2, steps=100):
    """Disc-bulge-halo galaxy on 3 nested 128^3 grids (half-extents 1, 4, 20),
    inner two flattened to q = 1/4; particle counts times `scale`."""
    gm = GalaxyModel(n_disc=int(2_000_000 * scale), n_bulge=int(500_000 * scale),
                     n_halo=int(6_000_000 * scale))
    x, v, m, comp, _ = galaxy(workload, gm)
    h = HierSpec([LevelSpec(N, 1.0, 0.25), LevelSpec(N, 4.0, 0.25), LevelSpec(N, 20.0, 1.0)],
                 centring="com")
    return Workload("disc_galaxy_3x128", x, v, m, comp, np.zeros(x.shape[0], np.int8), [h],
                    dt=0.01, steps=steps)


def galaxy_satellite(scale=1.0, N=128, workload=3, steps=500, e=0.3, incl=10.0):
    """The disc galaxy plus a Plummer satellite (M = 0.1, a = 0.6, cut 6a) on an
    orbit with apocentre 10, eccentricity e, inclination incl (prograde)."""
    gm = GalaxyModel(n_disc=int(2_000_000 * scale), n_bulge=int(500_000 * scale),
                     n_halo=int(6_000_000 * scale))
    x, v, m, comp, Menc = galaxy(workload, gm)
    ns = int(200_000 * scale)
    rng = rng_for(workload, SAT)
    ps, rs = plummer_positions(rng, ns, 0.6, 6.0)
    vs = plummer_velocities(rng, rs, 0.1, 0.6)
    R_A = 10.0
    X0, V0 = point_mass_orbit(float(Menc(R_A)), R_A, e, incl)
    x = np.concatenate([x, ps + X0]); v = np.concatenate([v, vs + V0])
    m = np.concatenate([m, np.full(ns, 0.1 / ns)])
    comp = np.concatenate([comp, np.full(ns, SAT, np.int8)])
    gal = np.concatenate([np.zeros(x.shape[0] - ns, np.int8), np.ones(ns, np.int8)])
    hg = HierSpec([LevelSpec(N, 1.0, 0.25), LevelSpec(N, 4.0, 0.25), LevelSpec(N, 20.0, 1.0)],
                  centring="com")
    hs = HierSpec([LevelSpec(N, 1.0, 1.0), LevelSpec(N, 6.0, 1.0), LevelSpec(N, 20.0, 1.0)],
                  centring="com")
    return Workload("galaxy_satellite_2x3x128", x, v, m, comp, gal, [hg, hs], dt=0.01, steps=steps)


def random_cells(rng, N, n, lo=2, hi=None):
    """Integer cell indices inside [lo, hi] per axis (for field tests)."""
    hi = N - 3 if hi is None else hi
    return rng.integers(lo, hi + 1, size=(n, 3))


def q_for(N):
    """Smallest flattening in {1/4, 1/2, 1} admissible on 3 levels of half-extents
    1, 4, 20 with N cells (the q_crit rule of Eq. 9 is applied by the library)."""
    qc = max(1.0 / 4.0, 4.0 / (N - 4) * 20.0 / 4.0)
    for q in (0.25, 0.5, 1.0):
        if q >= qc:
            return q
    return 1.0


def ensemble(n_inst=16, workload=4, steps=200, scale=1.0, sizes=(64, 128, 256), n_range=(1e5, 2e6)):
    """Independent satellite-sinking instances of uneven size: per instance a
    grid size from `sizes`, a particle count log-uniform in n_range (times
    `scale`) split disc:bulge:halo as the disc galaxy, a satellite of mass
    uniform in [0.02, 0.2] disc masses at equal particle mass, orbit
    eccentricity uniform in [0, 0.8] and inclination uniform in [0, 180] deg."""
    rng = rng_for(workload, 99)
    out = []
    for k in range(n_inst):
        N = int(rng.choice(sizes))
        n = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))) * scale)
        msat = float(rng.uniform(0.02, 0.2))
        e = float(rng.uniform(0.0, 0.8))
        inc = float(rng.uniform(0.0, 180.0))
        # the satellite's particles weigh as much as disc particles
        n_gal = max(int(n / (1.0 + 2.0 * msat / 8.5)), 100)
        gm = GalaxyModel(n_disc=int(n_gal * 2 / 8.5), n_bulge=int(n_gal * 0.5 / 8.5),
                         n_halo=int(n_gal * 6 / 8.5))
        x, v, m, comp, Menc = galaxy(1000 * workload + k, gm)
        m_disc = gm.M_disc / max(gm.n_disc, 1)
        ns = max(int(round(msat / m_disc)), 10)
        srng = rng_for(1000 * workload + k, SAT)
        ps, rs = plummer_positions(srng, ns, 0.6, 6.0)
        vs = plummer_velocities(srng, rs, msat, 0.6)
        X0, V0 = point_mass_orbit(float(Menc(10.0)), 10.0, e, inc)
        x = np.concatenate([x, ps + X0]); v = np.concatenate([v, vs + V0])
        m = np.concatenate([m, np.full(ns, msat / ns)])
        comp = np.concatenate([comp, np.full(ns, SAT, np.int8)])
        gal = np.concatenate([np.zeros(x.shape[0] - ns, np.int8), np.ones(ns, np.int8)])
        q = q_for(N)
        hg = HierSpec([LevelSpec(N, 1.0, q), LevelSpec(N, 4.0, q), LevelSpec(N, 20.0, 1.0)],
                      centring="com")
        hs = HierSpec([LevelSpec(N, 1.0, 1.0), LevelSpec(N, 6.0, 1.0), LevelSpec(N, 20.0, 1.0)],
                      centring="com")
        out.append(Workload(f"instance{k}_N{N}", x, v, m, comp, gal, [hg, hs], dt=0.01, steps=steps))
    return out


def adjoint_segment(scale=1.0, N=256, workload=5, steps=10):
    """Differentiable segment: one fixed 256^3 grid of half-extent 12 holding
    1M disc and 1M halo particles (disc-galaxy shapes; the halo cut at 11.5 so
    that every particle starts on the grid) and a 50k-particle Plummer
    satellite (M = 0.1, a = 0.6, cut at 3 so that it fits on the grid) at
    radius 8 in the disc plane on a circular orbit; all in one galaxy, the
    satellite as its own component."""
    gm = GalaxyModel(n_disc=int(1_000_000 * scale), n_bulge=0, n_halo=int(1_000_000 * scale),
                     rc_halo=11.5)
    x, v, m, comp, Menc = galaxy(workload, gm)
    ns = int(50_000 * scale)
    rng = rng_for(workload, SAT)
    ps, rs = plummer_positions(rng, ns, 0.6, 3.0)
    vs = plummer_velocities(rng, rs, 0.1, 0.6)
    X0, V0 = point_mass_orbit(float(Menc(8.0)), 8.0, 0.0, 0.0)
    x = np.concatenate([x, ps + X0]); v = np.concatenate([v, vs + V0])
    m = np.concatenate([m, np.full(ns, 0.1 / ns)])
    comp = np.concatenate([comp, np.full(ns, SAT, np.int8)])
    h = HierSpec([LevelSpec(N, 12.0, 1.0)])
    return Workload("adjoint_segment_256", x, v, m, comp, np.zeros(x.shape[0], np.int8), [h],
                    dt=0.01, steps=steps)


def escape_segment(kind="single", n=3000, workload=6, steps=4, dt=0.02):
    """A flattened cloud on fixed grids plus four heavy particles that leave
    the outermost grid during a short segment: they start inside its usable
    cells, moving outward fast enough to cross its boundary in the drift of
    the second cycle (they take part in cycles 0 and 1 and are lost from
    cycle 2 on).  kind 'single': one 32^3 grid of half-extent 2.5; 'nested':
    three fixed 32^3 levels of half-extents 0.5, 1.5 (both q = 1/2) and 4.
    The escapers are component 1, the component the segment tests select."""
    rng = rng_for(workload, 0 if kind == "single" else 1)
    x = rng.normal(size=(n, 3)) * np.array([0.6, 0.6, 0.15])
    v = rng.normal(size=(n, 3)) * 0.3
    m = rng.uniform(0.5, 1.5, n) / n
    comp = (rng.uniform(size=n) < 0.5).astype(np.int8)
    if kind == "single":
        hs = HierSpec([LevelSpec(32, 2.5, 1.0)])
        hi, lo, speed = 2.33, -2.51, 2.5     # usable edges at +2.411 and -2.589
    else:
        hs = HierSpec([LevelSpec(32, 0.5, 0.5), LevelSpec(32, 1.5, 0.5), LevelSpec(32, 4.0, 1.0)])
        hi, lo, speed = 3.72, -4.0, 4.0      # usable edges at +3.857 and -4.143
    ex = np.array([[hi, 0.1, 0.3], [lo, -0.2, -0.25], [0.15, hi, 0.2], [-0.1, 0.2, hi]])
    ev = np.array([[speed, 0.0, 0.0], [-speed, 0.0, 0.0], [0.0, speed, 0.0], [0.0, 0.0, speed]])
    x = np.vstack([x, ex]); v = np.vstack([v, ev])
    m = np.concatenate([m, np.full(4, 0.02)])
    comp = np.concatenate([comp, np.ones(4, np.int8)])
    return Workload("escape-" + kind, x, v, m, comp, np.zeros(n + 4, np.int8), [hs], dt, steps)
