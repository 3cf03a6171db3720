"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars (stated here, derived in the design notes):
  * integers (cell indices, classes, loss flags): bit-exact;
  * FP64 form: fields within 1e-11 of max|Phi|, forces within 1e-9 of the
    rms force (reduction order and reciprocal constants only);
  * FP32 form: Green's table within 2e-7 relative, fields within 3e-6 of
    max|Phi|, forces: 99th percentile of |da| <= 1e-4 rms|a| and max <= 1e-3
    rms|a| (FP32 rounding of the FFT amplified by differencing over cells).
"""
import numpy as np
import pytest

import synth
from oracle import pm_oracle as O
from tests import common as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbx():
    from paper_1210_1736_amd import sbx as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a ROCm device"
    return t


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, 700, k]))


PRECS = [0, 1]  # SBX_FP32, SBX_FP64


# ------------------------------------------------------------ Green table ---
@pytest.mark.parametrize("N,q", [(8, 1.0), (16, 0.25), (64, 0.5), (128, 1.0)])
@pytest.mark.parametrize("prec", PRECS)
def test_green_table_matches_oracle(sbx, N, q, prec):
    R = 3.0
    p = sbx.Poisson(N, R, q, G=1.3, prec=prec)
    Hs, rel_imag = p.sbx_poisson_green()
    assert rel_imag < 1e-13
    Hh, _ = O.green_hat(O.Level(N, R, q))
    ref = 1.3 / (2 * N) ** 3 * Hh[: N + 1, : N + 1, : N + 1]
    tol = 1e-12 if prec == sbx.SBX_FP64 else 2e-7
    assert np.max(np.abs(Hs - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("h0", [0, 1, 2])
@pytest.mark.parametrize("N,q", [(16, 1.0), (64, 0.25)])
@pytest.mark.parametrize("prec", PRECS)
def test_green_table_h0_readings(sbx, N, q, h0, prec):
    """The three readings of the singular H(0,0,0) (h0_mode 0: H(1,0,0),
    1: mean of 1/r over the cell, 2: zero) against the oracle's tables."""
    R = 2.0
    p = sbx.Poisson(N, R, q, G=1.0, h0_mode=h0, prec=prec)
    Hs, rel_imag = p.sbx_poisson_green()
    assert rel_imag < 1e-13
    Hh, _ = O.green_hat(O.Level(N, R, q), h0)
    ref = Hh[: N + 1, : N + 1, : N + 1] / (2 * N) ** 3
    tol = 1e-12 if prec == sbx.SBX_FP64 else 2e-7
    assert np.max(np.abs(Hs - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("h0", [1, 2])
def test_forces_h0_readings_fp64(sbx, h0):
    """Fields and forces of the nested galaxy with the other readings of
    H(0,0,0), through sbx_create's h0_mode, against the oracle."""
    w = T.small_galaxy(scale=0.003, N=64, q=0.5)
    sysm = T.oracle_system(w, h0_mode=h0)
    lost = sysm.lost_now(w.x)
    centres = sysm.centres(w.x, w.m, w.gal, lost)
    pots = sysm.potentials(w.x, w.m, w.gal, lost, centres)
    ctx = T.make_ctx(w, sbx.SBX_FP64, h0_mode=h0)
    acc, pot = ctx.sbx_compute_forces()
    for k, ref in enumerate(_slots(pots[0]["Phi"])):
        g = ctx.sbx_get_grid(0, k, 1).transpose(2, 1, 0)
        assert np.max(np.abs(g - ref)) <= 1e-11 * np.max(np.abs(ref)), k
    a_ref, P_ref = sysm.accel(w.x, w.m, w.gal, lost, centres, pots, want_pot=True)
    assert T.rel_err_vec(acc, a_ref).max() < 1e-9
    assert np.abs(pot + P_ref).max() < 1e-11 * np.abs(P_ref).max()


# ----------------------------------------------------------- Poisson solve --
def _solve_gpu(sbx, torch, N, R, q, Ms, prec, G=1.0):
    dt = torch.float64 if prec == sbx.SBX_FP64 else torch.float32
    rho = torch.tensor(np.stack([M.transpose(2, 1, 0) for M in Ms]), dtype=dt, device="cuda").contiguous()
    phi = torch.empty_like(rho)
    p = sbx.Poisson(N, R, q, G=G, prec=prec, stream=torch.cuda.current_stream().cuda_stream)
    p.sbx_poisson_solve(len(Ms), rho.data_ptr(), phi.data_ptr())
    torch.cuda.synchronize()
    out = phi.double().cpu().numpy()
    p.close()
    return [o.transpose(2, 1, 0) for o in out]


@pytest.mark.parametrize("N,q", [(8, 1.0), (16, 0.25), (32, 1.0), (64, 0.5), (128, 0.25)])
@pytest.mark.parametrize("prec", PRECS)
def test_poisson_solve_matches_oracle(sbx, torch, N, q, prec):
    rng = _rng(N)
    R = 2.0
    L = O.Level(N, R, q)
    Ms = []
    for b in range(3):
        M = np.zeros((N, N, N))
        cells = rng.integers(0, N, size=(max(50, N * N // 4), 3))
        np.add.at(M, tuple(cells.T), rng.uniform(0.1, 1.0, cells.shape[0]))
        Ms.append(T.rounded(M, prec))
    got = _solve_gpu(sbx, torch, N, R, q, Ms, prec, G=0.7)
    Hh, _ = O.green_hat(L)
    tol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    for M, g in zip(Ms, got):
        ref = O.solve_fft(M, Hh, G=0.7)
        assert np.max(np.abs(g - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("v", [16, 32])
@pytest.mark.parametrize("N,q", [(64, 0.5), (128, 0.25)])
def test_fft_schedules_match_oracle(sbx, torch, v, N, q):
    """Each FFT line schedule pinned in turn (16 or 32 values per thread; FP32
    lines of 128 and 256 points have both, and the tuner picks per pass)
    against the oracle's FFT convolution (Eqs. 3-5), FP32 bar 3e-6 of max|Phi|."""
    rng = _rng(1000 + N + v)
    R = 2.0
    Ms = []
    for b in range(2):
        M = np.zeros((N, N, N))
        cells = rng.integers(0, N, size=(N * N // 4, 3))
        np.add.at(M, tuple(cells.T), rng.uniform(0.1, 1.0, cells.shape[0]))
        Ms.append(T.rounded(M, sbx.SBX_FP32))
    sbx.sbx_set_fft_schedule(v)
    try:
        got = _solve_gpu(sbx, torch, N, R, q, Ms, sbx.SBX_FP32, G=0.7)
    finally:
        sbx.sbx_set_fft_schedule(0)
    Hh, _ = O.green_hat(O.Level(N, R, q))
    for M, g in zip(Ms, got):
        ref = O.solve_fft(M, Hh, G=0.7)
        assert np.max(np.abs(g - ref)) <= 3e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("form", [3, 5])
@pytest.mark.parametrize("N,q,prec", [(16, 1.0, 1), (32, 0.25, 0), (32, 0.25, 1), (64, 0.5, 0),
                                      (64, 0.5, 1), (128, 0.25, 0), (128, 0.25, 1)])
def test_fft_forms_match_oracle(sbx, torch, form, N, q, prec):
    """Each form of the solve pinned in turn: three plane-fused passes (x
    and y of one plane in LDS; even and odd frequencies of each padded line
    as two half-length transforms) or five line passes, against the oracle's
    FFT convolution (Eqs. 3-5), three solves per batch (at N = 128 the
    plane forward takes the even and the odd kx columns of a plane in two
    blocks, the inverse the even and the odd rows, or in FP32 whole planes,
    as the tuner times them).  N = 16 has no plane form and runs five
    passes under either pin."""
    rng = _rng(3000 + N + form + 10 * prec)
    R = 2.0
    Ms = []
    for b in range(3):
        M = np.zeros((N, N, N))
        cells = rng.integers(0, N, size=(max(50, N * N // 4), 3))
        np.add.at(M, tuple(cells.T), rng.uniform(0.1, 1.0, cells.shape[0]))
        Ms.append(T.rounded(M, prec))
    sbx.sbx_set_fft_form(form)
    try:
        got = _solve_gpu(sbx, torch, N, R, q, Ms, prec, G=0.7)
        rep = sbx.sbx_fft_tuning_report()
    finally:
        sbx.sbx_set_fft_form(0)
    want = form if N >= 32 else 5
    esz = "fp64" if prec == sbx.SBX_FP64 else "fp32"
    assert f"{esz} N={N} x3 form={want} " in rep
    Hh, _ = O.green_hat(O.Level(N, R, q))
    tol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    for M, g in zip(Ms, got):
        ref = O.solve_fft(M, Hh, G=0.7)
        assert np.max(np.abs(g - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("nt,prec", [(256, 0), (512, 0), (1024, 0), (256, 1), (512, 1)])
def test_plane_block_sizes_match_oracle(sbx, torch, nt, prec):
    """128^3 with the plane form and each block size pinned in turn: 256
    and 512 threads run both half-plane passes (even and odd kx columns
    forward, even and odd rows y inverse; in FP64 the only plane form at
    this size), 1024 the FP32 whole-plane inverse after the half-plane
    forward (which has no 1024); three solves of different fill against
    the oracle's FFT convolution (Eqs. 3-5)."""
    N, R, q = 128, 2.0, 0.25
    rng = _rng(4100 + nt + prec)
    Ms = []
    for b in range(3):
        M = np.zeros((N, N, N))
        cells = rng.integers(0, N, size=(N * N // (2 + b), 3))
        np.add.at(M, tuple(cells.T), rng.uniform(0.1, 1.0, cells.shape[0]))
        Ms.append(T.rounded(M, prec))
    sbx.sbx_set_fft_form(3)
    sbx.sbx_set_plane_threads(nt)
    try:
        got = _solve_gpu(sbx, torch, N, R, q, Ms, prec, G=0.7)
        rep = sbx.sbx_fft_tuning_report()
    finally:
        sbx.sbx_set_fft_form(0)
        sbx.sbx_set_plane_threads(0)
    esz = "fp64" if prec == sbx.SBX_FP64 else "fp32"
    assert f"{esz} N={N} x3 form=3 plane_inv nt={nt}" in rep
    if nt != 1024:
        assert f"{esz} N={N} x3 form=3 plane_fwd nt={nt}" in rep
    Hh, _ = O.green_hat(O.Level(N, R, q))
    tol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    for M, g in zip(Ms, got):
        ref = O.solve_fft(M, Hh, G=0.7)
        assert np.max(np.abs(g - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [64, 128])
@pytest.mark.parametrize("prec", PRECS)
def test_plane_form_in_the_step(sbx, prec, N):
    """The galaxy's fields and forces with the plane-fused form pinned (its
    summed grids 2+3 and 4+5 add their second mass grid in the plane
    forward pass) against the oracle, to the bars of the five-pass form;
    at 128^3 through the half-plane passes (in FP64 the tuner would keep
    five passes for this solve count)."""
    w = T.small_galaxy(scale=0.005, N=N, q=0.5)
    sysm, x, v, m, lost, centres, pots = _state_oracle(w, prec)
    sbx.sbx_set_fft_form(3)
    try:
        ctx = T.make_ctx(w, prec)
        acc, pot = ctx.sbx_compute_forces()
        rep = sbx.sbx_fft_tuning_report()
    finally:
        sbx.sbx_set_fft_form(0)
    assert ("fp64" if prec == sbx.SBX_FP64 else "fp32") + f" N={N} x5 form=3 plane_fwd" in rep
    cg = ctx.sbx_get_centres()
    cls_ref, idx_ref = O.classify(x, sysm.h[0], cg[0])
    pots = sysm.potentials(x, m, w.gal, lost, cg)
    ftol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    for k, ref in enumerate(_slots(pots[0]["Phi"])):
        g = ctx.sbx_get_grid(0, k, 1).transpose(2, 1, 0)
        assert np.max(np.abs(g - ref)) <= ftol * np.max(np.abs(ref)), k
    a_ref, P_ref = sysm.accel(x, m, w.gal, lost, cg, pots, want_pot=True)
    e = T.rel_err_vec(acc, a_ref)
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3
    ctx.close()


@pytest.mark.parametrize("v", [16, 32])
def test_fft_schedules_max_size_sampled(sbx, torch, v):
    """N = 256 (512-point lines) with each schedule pinned: sampled cells
    against the direct sum of Eq. 1 (FP32 bar 3e-6)."""
    N, R, q = 256, 10.0, 1.0
    L = O.Level(N, R, q)
    rng = _rng(2560 + v)
    src = rng.integers(0, N, size=(2000, 3))
    mass = T.rounded(rng.uniform(0.1, 1.0, 2000), sbx.SBX_FP32)
    M = np.zeros((N, N, N))
    np.add.at(M, tuple(src.T), mass)
    sbx.sbx_set_fft_schedule(v)
    try:
        g = _solve_gpu(sbx, torch, N, R, q, [M], sbx.SBX_FP32)[0]
    finally:
        sbx.sbx_set_fft_schedule(0)
    H = O.green_table(L)
    probes = rng.integers(0, N, size=(200, 3))
    nz = np.argwhere(M != 0)
    w = M[tuple(nz.T)]
    ref = np.array([np.sum(w * H[np.abs(nz[:, 0] - a), np.abs(nz[:, 1] - b), np.abs(nz[:, 2] - c)])
                    for a, b, c in probes])
    assert np.max(np.abs(g[tuple(probes.T)] - ref)) <= 3e-6 * np.max(ref)


def test_poisson_solve_equals_direct_sum(sbx, torch):
    N, R, q = 16, 1.5, 0.5
    rng = _rng(99)
    M = np.zeros((N, N, N))
    cells = rng.integers(0, N, size=(40, 3))
    np.add.at(M, tuple(cells.T), rng.uniform(0.1, 1.0, 40))
    g = _solve_gpu(sbx, torch, N, R, q, [M], sbx.SBX_FP64)[0]
    ref = O.solve_direct(M, O.Level(N, R, q))
    assert np.max(np.abs(g - ref)) <= 1e-11 * np.max(ref)


@pytest.mark.parametrize("prec", PRECS)
def test_poisson_max_size_sampled(sbx, torch, prec):
    """N = 256 (512^3 padded): sampled cells against the direct sum."""
    N, R, q = 256, 10.0, 1.0
    L = O.Level(N, R, q)
    rng = _rng(256)
    src = rng.integers(0, N, size=(3000, 3))
    mass = T.rounded(rng.uniform(0.1, 1.0, 3000), prec)
    M = np.zeros((N, N, N))
    np.add.at(M, tuple(src.T), mass)
    g = _solve_gpu(sbx, torch, N, R, q, [M], prec)[0]
    H = O.green_table(L)
    probes = rng.integers(0, N, size=(300, 3))
    nz = np.argwhere(M != 0)
    w = M[tuple(nz.T)]
    ref = np.array([np.sum(w * H[np.abs(nz[:, 0] - a), np.abs(nz[:, 1] - b), np.abs(nz[:, 2] - c)])
                    for a, b, c in probes])
    got = g[tuple(probes.T)]
    tol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(ref)


def test_poisson_batch_is_per_grid(sbx, torch):
    """Solving grids in one batch gives exactly what solving each alone gives."""
    N = 32
    rng = _rng(5)
    Ms = [rng.uniform(size=(N, N, N)) * (rng.uniform(size=(N, N, N)) < 0.05) for _ in range(4)]
    Ms = [T.rounded(M, 0) for M in Ms]
    together = _solve_gpu(sbx, torch, N, 1.0, 1.0, Ms, sbx.SBX_FP32)
    alone = [_solve_gpu(sbx, torch, N, 1.0, 1.0, [M], sbx.SBX_FP32)[0] for M in Ms]
    for a, b in zip(together, alone):
        assert np.array_equal(a, b)


# ---------------------------------------------------------- cell indices ----
def _adversarial_positions(hs: synth.HierSpec, rng, n_rand=20000):
    """Random points plus points on cell faces (u = k + 1/2 and +-1 ulp),
    at radius exactly R, and outside the grids."""
    pts = [rng.normal(size=(n_rand, 3)) * np.array([2.0, 2.0, 0.5])]
    c = np.asarray(hs.centre)
    for L in hs.levels:
        l = (2.0 * L.R) / (L.N - 4)
        lz = L.q * l
        k = rng.integers(0, L.N, size=(400, 3)).astype(np.float64)
        u = k + 0.5
        base = c + (u - L.N / 2.0) * np.array([l, l, lz])
        pts += [base, np.nextafter(base, np.inf), np.nextafter(base, -np.inf)]
        d = rng.normal(size=(200, 3)); d /= np.linalg.norm(d, axis=1)[:, None]
        d[:, 2] *= L.q
        pts.append(c + d * L.R)
    pts.append(rng.uniform(-25, 25, size=(500, 3)))
    return np.concatenate(pts)


@pytest.mark.parametrize("prec", PRECS)
def test_indices_and_classes_bit_exact(sbx, prec):
    hs = synth.HierSpec([synth.LevelSpec(64, 1.0, 0.5), synth.LevelSpec(64, 4.0, 0.5),
                         synth.LevelSpec(64, 20.0, 1.0)], centring="fixed",
                        centre=(0.0625, -0.03125, 0.01), outer_centre=(0.5, 0.25, -0.125))
    rng = _rng(11)
    x = _adversarial_positions(hs, rng)
    n = x.shape[0]
    ctx = sbx.Context(prec=prec)
    ctx.sbx_build_grids([T.sbx_hier(hs)])
    ctx.sbx_load_particles(x, np.zeros_like(x), np.ones(n), np.zeros(n, np.int8), np.zeros(n, np.int8))
    xo = T.rounded(x, prec)
    cls_ref, idx_ref = O.classify(xo, T.oracle_hier(hs), np.asarray(hs.centre))
    for level in range(3):
        idx, cls = ctx.sbx_get_indices(0, level)
        assert np.array_equal(cls, cls_ref)
        assert np.array_equal(idx.astype(np.int64), idx_ref[level])
    assert len(set(cls_ref.tolist())) == 4


# ------------------------------------------------ grids, fields and forces --
def _state_oracle(w, prec, taylor=True):
    sysm = T.oracle_system(w, taylor=taylor)
    x, v, m = T.oracle_inputs(w, prec)
    lost = np.zeros(w.n, bool)
    lost |= sysm.lost_now(x)
    centres = sysm.centres(x, m, w.gal, lost)
    pots = sysm.potentials(x, m, w.gal, lost, centres)
    return sysm, x, v, m, lost, centres, pots


def _slots(pot):
    """Oracle grids in the library's slot order: 1, 3, 2+3, 5, 4+5."""
    if len(pot) == 1:
        return [pot[0]]
    return [pot[0], pot[2], pot[1] + pot[2], pot[4], pot[3] + pot[4]]


@pytest.mark.parametrize("prec", PRECS)
def test_galaxy_grids_fields_forces(sbx, prec):
    w = T.small_galaxy(scale=0.005, N=64, q=0.5)
    sysm, x, v, m, lost, centres, pots = _state_oracle(w, prec)
    ctx = T.make_ctx(w, prec)
    acc, pot = ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    assert np.allclose(cg[0], centres[0], rtol=0, atol=1e-13 * (1 + np.abs(centres[0]).max()))
    # integers: classes and cells of every particle, classified by the oracle
    # at the library's own centres (the two sides reduce the centre of mass
    # in different orders, so a particle on a cell face could otherwise flip)
    cls_ref, idx_ref = O.classify(x, sysm.h[0], cg[0])
    for level in range(3):
        idx, cls = ctx.sbx_get_indices(0, level)
        assert np.array_equal(cls, cls_ref)
        assert np.array_equal(idx.astype(np.int64), idx_ref[level])
    # fields
    ftol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    for k, ref in enumerate(_slots(pots[0]["Phi"])):
        g = ctx.sbx_get_grid(0, k, 1).transpose(2, 1, 0)
        assert np.max(np.abs(g - ref)) <= ftol * np.max(np.abs(ref)), k
    # forces and potentials at the particles
    a_ref, P_ref = sysm.accel(x, m, w.gal, lost, centres, pots, want_pot=True)
    e = T.rel_err_vec(acc, a_ref)
    pe = np.abs(pot - (-P_ref)) / np.max(np.abs(P_ref))
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9 and pe.max() < 1e-11
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3 and pe.max() < 3e-6
    # cell masses (re-assigned; the solve overwrote them).  FP32 sums of up to
    # ~1e5 particle masses per cell carry an error ~ eps32 * sqrt(K) of the cell.
    mtol = 1e-12 if prec == sbx.SBX_FP64 else 3e-5
    for k, ref in enumerate(_slots(pots[0]["M"])):
        g = ctx.sbx_get_grid(0, k, 0).transpose(2, 1, 0)
        assert np.max(np.abs(g - ref)) <= mtol * max(np.max(ref), 1e-30), k


@pytest.mark.parametrize("prec", PRECS)
def test_central_difference_mode(sbx, prec):
    w = T.small_galaxy(scale=0.002, N=32, q=1.0)
    w.hier = [synth.HierSpec([synth.LevelSpec(32, 1.0, 1.0), synth.LevelSpec(32, 4.0, 1.0),
                              synth.LevelSpec(32, 20.0, 1.0)], centring="com")]
    sysm, x, v, m, lost, centres, pots = _state_oracle(w, prec, taylor=False)
    ctx = T.make_ctx(w, prec, taylor=0)
    acc, _ = ctx.sbx_compute_forces()
    a_ref = sysm.accel(x, m, w.gal, lost, centres, pots)
    e = T.rel_err_vec(acc, a_ref)
    assert e.max() < (1e-9 if prec == sbx.SBX_FP64 else 1e-3)


def test_steps_match_oracle_fp64(sbx):
    w = T.small_galaxy(scale=0.003, N=64, q=0.5)
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    sysm = T.oracle_system(w)
    x, v, m = w.x.copy(), w.v.copy(), w.m.copy()
    lost = np.zeros(w.n, bool)
    for _ in range(3):
        x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt)
    ctx.sbx_step(w.dt, 3)
    xg, vg, lg = ctx.sbx_get_particles()
    assert np.array_equal(lg, lost)
    assert np.max(np.abs(xg - x)) < 1e-10
    assert np.max(np.abs(vg - v)) < 1e-8


def test_plummer_64_full_fp64(sbx):
    """The single-grid Plummer workload: one force evaluation plus 10 steps."""
    w = synth.plummer_cube()
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    sysm = T.oracle_system(w)
    acc, pot = ctx.sbx_compute_forces()
    lost = np.zeros(w.n, bool)
    a_ref, P_ref = sysm.accel(w.x, w.m, w.gal, lost, want_pot=True)
    assert T.rel_err_vec(acc, a_ref).max() < 1e-9
    x, v = w.x.copy(), w.v.copy()
    for _ in range(w.steps):
        x, v, lost, _ = sysm.step(x, v, w.m, w.gal, lost, w.dt)
    ctx.sbx_step(w.dt, w.steps)
    xg, vg, lg = ctx.sbx_get_particles()
    assert np.array_equal(lg, lost)
    assert np.max(np.abs(xg - x)) < 1e-10 and np.max(np.abs(vg - v)) < 1e-8


def test_plummer_64_fp32_error_stated(sbx):
    """FP32 form on the Plummer workload: force error against the FP64
    oracle from the same (rounded) inputs."""
    w = synth.plummer_cube()
    ctx = T.make_ctx(w, sbx.SBX_FP32)
    sysm = T.oracle_system(w)
    acc, pot = ctx.sbx_compute_forces()
    x, v, m = T.oracle_inputs(w, sbx.SBX_FP32)
    a_ref = sysm.accel(x, m, w.gal, np.zeros(w.n, bool))
    e = T.rel_err_vec(acc, a_ref)
    print(f"FP32 Plummer force error: p99 {np.percentile(e, 99):.2e} max {e.max():.2e} of rms")
    assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3


def test_loss_and_lost_particles_frozen(sbx):
    hs = synth.HierSpec([synth.LevelSpec(32, 4.0, 1.0)])
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [5.0, 0.0, 0.0], [3.95, 0.0, 0.0]])
    v = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    m = np.array([1.0, 0.0, 0.0, 0.0])
    w = synth.Workload("t", x, v, m, np.zeros(4, np.int8), np.zeros(4, np.int8), [hs], 0.1, 2)
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    ctx.sbx_step(0.1, 1)
    xg, vg, lg = ctx.sbx_get_particles()
    assert list(lg) == [False, False, True, True]
    assert np.all(xg[2] == x[2])
    ctx.sbx_step(0.1, 1)
    xg2, _, _ = ctx.sbx_get_particles()
    assert np.all(xg2[3] == xg[3])
    assert ctx.sbx_count_live() == 2


# Diagnostics bars.  FP64: the sums of the FP64 forces (1e-9 of rms) and
# potentials.  FP32 (FP32 fields and particles, FP64 reductions): E_kin, L
# and the dispersions take v + dt/2 a, where the FP32 force error (1e-4 of
# rms at most) enters multiplied by dt/2: 1e-7 relative; W sums the FP32
# potential, within 3e-6 of its largest value per particle: 1e-5 relative.
DIAG_BARS = {0: dict(ekin=1e-7, epot=1e-5, L=1e-7, sig=1e-7),
             1: dict(ekin=1e-10, epot=1e-9, L=1e-9, sig=1e-9)}


def assert_diag_close(d, ref, prec, m, x, v):
    b = DIAG_BARS[prec]
    assert np.allclose(d["ekin"], ref["ekin"], rtol=b["ekin"], atol=1e-14)
    assert np.allclose(d["epot"], ref["epot"], rtol=b["epot"], atol=1e-14)
    # angular momentum per component: within the bar of sum m |x| |v|
    for c in range(8):
        scale = np.sum(m * np.linalg.norm(x, axis=1) * np.linalg.norm(v, axis=1))
        assert np.all(np.abs(d["L"][c] - ref["L"][c]) <= b["L"] * scale + 1e-14), c
    assert d["disc_sigR"] == pytest.approx(ref["disc_sigR"], rel=b["sig"])
    assert d["disc_sigz"] == pytest.approx(ref["disc_sigz"], rel=b["sig"])
    assert d["n_lost"] == ref["n_lost"]


@pytest.mark.parametrize("prec", PRECS)
def test_diagnostics_match_oracle(sbx, prec):
    w = T.small_galaxy(scale=0.003, N=64, q=0.5)
    ctx = T.make_ctx(w, prec)
    d = ctx.sbx_diagnostics(w.dt)
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, prec)
    ref = sysm.diagnostics(x, v, m, w.comp, w.gal, np.zeros(w.n, bool), w.dt)
    assert_diag_close(d, ref, prec, m, x, v)
    # the in-step log records the same quantities at the start of a step
    ctx.sbx_step(w.dt, 1, diag_every=1)
    log = ctx.sbx_diag_log()
    assert len(log) == 1
    assert np.allclose(log[0]["ekin"], d["ekin"], rtol=1e-12)


@pytest.mark.parametrize("prec", PRECS)
def test_galaxy_and_satellite(sbx, prec):
    """Two galaxies (3 levels each, shared global grid): classes relative to
    each galaxy and summed forces."""
    w = synth.galaxy_satellite(scale=0.004, N=64)
    for h in w.hier:
        h.levels = [synth.LevelSpec(64, L.R, 0.5 if h is w.hier[0] and i < 2 else 1.0)
                    for i, L in enumerate(h.levels)]
    sysm, x, v, m, lost, centres, pots = _state_oracle(w, prec)
    ctx = T.make_ctx(w, prec)
    acc, _ = ctx.sbx_compute_forces()
    cg = ctx.sbx_get_centres()
    for g in range(2):
        assert np.allclose(cg[g], centres[g], rtol=0, atol=1e-13 * (1 + np.abs(centres[g]).max()))
        cls_ref, idx_ref = O.classify(x, sysm.h[g], cg[g])
        idx, cls = ctx.sbx_get_indices(g, 1)
        assert np.array_equal(cls, cls_ref)
        assert np.array_equal(idx.astype(np.int64), idx_ref[1])
    a_ref = sysm.accel(x, m, w.gal, lost, centres, pots)
    e = T.rel_err_vec(acc, a_ref)
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3


def test_disc_galaxy_full_size_sampled(sbx):
    """The 3 x 128^3 disc-galaxy workload at full size (8.5M particles, FP32):
    forces at 20k sampled particles against the oracle's full fields."""
    w = synth.disc_galaxy(scale=1.0)
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, sbx.SBX_FP32)
    lost = sysm.lost_now(x)
    centres = sysm.centres(x, m, w.gal, lost)
    pots = sysm.potentials(x, m, w.gal, lost, centres)
    ctx = T.make_ctx(w, sbx.SBX_FP32)
    acc, _ = ctx.sbx_compute_forces()
    rng = _rng(3)
    s = rng.choice(np.flatnonzero(~lost), 20000, replace=False)
    a_ref, _ = sysm.field_at(x[s], centres, pots)
    e = T.rel_err_vec(acc[s], a_ref)
    print(f"FP32 disc-galaxy force error: p99 {np.percentile(e, 99):.2e} max {e.max():.2e} of rms")
    assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3
    cg = ctx.sbx_get_centres()
    assert np.allclose(cg[0], centres[0], rtol=0, atol=1e-12 * (1 + np.abs(centres[0]).max()))
    cls_ref, idx_ref = O.classify(x[s], sysm.h[0], cg[0])
    for level in range(3):
        idx, cls = ctx.sbx_get_indices(0, level)
        assert np.array_equal(cls[s], cls_ref)
        assert np.array_equal(idx[s].astype(np.int64), idx_ref[level])


def test_error_paths(sbx):
    ctx = sbx.Context(prec=sbx.SBX_FP32)
    with pytest.raises(sbx.SbxError) as e:
        ctx.sbx_step(0.01, 1)
    assert e.value.status == sbx.SBX_ESTATE
    bad = sbx.make_hierarchy([(128, 1, 0.2), (128, 4, 0.2), (128, 20, 1)])
    with pytest.raises(sbx.SbxError) as e:
        ctx.sbx_build_grids([bad])
    assert e.value.status == sbx.SBX_EQCRIT
    with pytest.raises(sbx.SbxError) as e:
        ctx.sbx_load_particles(np.zeros((2, 3)), np.zeros((2, 3)), np.array([1.0, np.nan]),
                               np.zeros(2, np.int8), np.zeros(2, np.int8))
    assert e.value.status == sbx.SBX_EINVAL


def test_cell_sort_keeps_results_and_order(sbx):
    """Reordering particles by cell is invisible to the caller: steps with
    and without the sort agree to rounding, outputs come back in input order."""
    w = T.small_galaxy(scale=0.003, N=64, q=0.5)
    out = []
    for every in (0, 1, 3):
        ctx = T.make_ctx(w, sbx.SBX_FP64)
        ctx.sbx_set_sort_interval(every)
        ctx.sbx_step(w.dt, 4)
        out.append(ctx.sbx_get_particles())
        idx, cls = ctx.sbx_get_indices(0, 0)
        out[-1] = out[-1] + (idx, cls)
        ctx.close()
    for o in out[1:]:
        assert np.array_equal(o[2], out[0][2])
        assert np.max(np.abs(o[0] - out[0][0])) < 1e-12
        assert np.max(np.abs(o[1] - out[0][1])) < 1e-10
        assert np.array_equal(o[4], out[0][4])


def test_fp32_steps_track_oracle(sbx):
    """FP32 form over 5 steps stays within FP32 rounding of the FP64 oracle."""
    w = T.small_galaxy(scale=0.003, N=64, q=0.5)
    ctx = T.make_ctx(w, sbx.SBX_FP32)
    sysm = T.oracle_system(w)
    x, v, m = T.oracle_inputs(w, sbx.SBX_FP32)
    lost = np.zeros(w.n, bool)
    for _ in range(5):
        x, v, lost, _ = sysm.step(x, v, m, w.gal, lost, w.dt)
    ctx.sbx_step(w.dt, 5)
    xg, vg, lg = ctx.sbx_get_particles()
    assert np.array_equal(lg, lost)
    vr = np.sqrt(np.mean(np.sum(v * v, axis=1)))
    ev = np.linalg.norm(vg - v, axis=1) / vr
    assert np.percentile(ev, 99) < 1e-4
    assert np.max(np.abs(xg - x)) < 1e-4


def test_batch_graph_replays_match_single_contexts(sbx):
    """Instances of uneven size stepped as one batch (one launch per phase,
    one graph replay per step, with cell sorts) equal the same instances
    stepped one by one, after every replay."""
    ws = synth.ensemble(n_inst=4, scale=0.004, sizes=(32, 64))
    for w in ws:
        for h in w.hier:
            h.levels = [synth.LevelSpec(L.N, L.R, 1.0) for L in h.levels]
    sizes = sorted({w.hier[0].levels[0].N for w in ws})
    assert len(sizes) >= 2
    ref = [T.make_ctx(w, sbx.SBX_FP64) for w in ws]
    bat = [T.make_ctx(w, sbx.SBX_FP64) for w in ws]
    for c in ref + bat:
        c.sbx_set_sort_interval(3)
    b = sbx.Batch(bat)
    for step in range(7):
        for c, w in zip(ref, ws):
            c.sbx_step(w.dt, 1)
        b.sbx_batch_step([w.dt for w in ws], 1)
        b.sbx_batch_sync()
        for c, d in zip(ref, bat):
            xr, vr, lr = c.sbx_get_particles()
            xb, vb, lb = d.sbx_get_particles()
            assert np.array_equal(lr, lb)
            assert np.max(np.abs(xr - xb)) < 1e-11, step
            assert np.max(np.abs(vr - vb)) < 1e-9, step
    with pytest.raises(sbx.SbxError):
        bat[0].sbx_step(0.01, 1)
    b.close()
    bat[0].sbx_step(ws[0].dt, 1)  # released contexts step alone again


@pytest.mark.parametrize("every", [1, 2, 3])
def test_reorder_steps_match_oracle_fp64(sbx, every):
    """Steps that reorder the particles by cell every `every` steps (the mass
    assignment's wave sums then see runs of equal cells, broken up again as
    the particles drift) against the oracle's steps: positions within 1e-10,
    velocities within 1e-8, loss flags exact, after each of 7 steps; the
    reorder is invisible in the caller's order."""
    w = T.small_galaxy(scale=0.003, N=64, q=0.5)
    sysm = T.oracle_system(w)
    x, v, lost = w.x.copy(), w.v.copy(), np.zeros(w.n, bool)
    ctx = T.make_ctx(w, sbx.SBX_FP64)
    ctx.sbx_set_sort_interval(every)
    for k in range(7):
        x, v, lost, _ = sysm.step(x, v, w.m, w.gal, lost, w.dt)
        ctx.sbx_step(w.dt, 1, 3)
        xg, vg, lg = ctx.sbx_get_particles()
        assert np.array_equal(lg, lost), k
        assert np.max(np.abs(xg - x)) < 1e-10, k
        assert np.max(np.abs(vg - v)) < 1e-8, k
    assert len(ctx.sbx_diag_log()) == 3


def test_reorder_steps_fp32_match_unsorted(sbx):
    """FP32: stepping with reorders every 2 steps against the same context
    never reordered (only the summation order differs): loss flags equal,
    positions within 1e-5, velocities within 1e-4 of the rms velocity at the
    99th percentile, after 9 steps."""
    w = T.small_galaxy(scale=0.004, N=64, q=0.5)
    a = T.make_ctx(w, sbx.SBX_FP32)
    b = T.make_ctx(w, sbx.SBX_FP32)
    a.sbx_set_sort_interval(2)
    b.sbx_set_sort_interval(0)
    a.sbx_step(w.dt, 9, 4)
    b.sbx_step(w.dt, 9, 4)
    xa, va, la = a.sbx_get_particles()
    xb, vb, lb = b.sbx_get_particles()
    assert np.array_equal(la, lb)
    vr = np.sqrt(np.mean(np.sum(vb * vb, axis=1)))
    assert np.max(np.abs(xa - xb)) < 1e-5
    assert np.percentile(np.linalg.norm(va - vb, axis=1) / vr, 99) < 1e-4
    da, db = a.sbx_diag_log(), b.sbx_diag_log()
    assert np.allclose(da[-1]["ekin"], db[-1]["ekin"], rtol=1e-6)


@pytest.mark.parametrize("merge", [0, 1])
@pytest.mark.parametrize("prec", PRECS)
def test_sorted_mass_assignment_after_drift(sbx, prec, merge):
    """The mass assignment on particles reordered by cell that have drifted
    since (4 steps with large dt after the reorder; with merge, a satellite's
    outer masses land in the first galaxy's grid 5): the fields of every slot
    against the oracle's at the library's own positions and centres (FP64
    1e-11, FP32 3e-6 of max|Phi|), and the forces."""
    w = synth.galaxy_satellite(scale=0.004, N=64)
    for h in w.hier:
        h.levels = [synth.LevelSpec(64, L.R, 0.5 if h is w.hier[0] and i < 2 else 1.0)
                    for i, L in enumerate(h.levels)]
    ctx = sbx.Context(prec=prec, G=w.G)
    ctx.sbx_set_outer_merge(merge)
    ctx.sbx_set_sort_interval(8)
    ctx.sbx_build_grids([T.sbx_hier(h) for h in w.hier])
    ctx.sbx_load_particles(w.x, w.v, w.m, w.comp, w.gal)
    ctx.sbx_step(0.05, 5)
    acc, _ = ctx.sbx_compute_forces()
    xg, vg, lg = ctx.sbx_get_particles()
    cg = ctx.sbx_get_centres()
    sysm = T.oracle_system(w)
    m = T.rounded(w.m, prec)
    lost = lg.astype(bool)
    pots = sysm.potentials(xg, m, w.gal, lost, list(cg))
    ftol = 1e-11 if prec == sbx.SBX_FP64 else 3e-6
    for g in range(2):
        ref = _slots(pots[g]["Phi"])
        if merge:
            ref[3] = None if g else pots[0]["Phi"][4] + pots[1]["Phi"][4]
            ref[4] = pots[g]["Phi"][3]
        for k, r in enumerate(ref):
            if r is None:
                continue
            gg = ctx.sbx_get_grid(g, k, 1).transpose(2, 1, 0)
            assert np.max(np.abs(gg - r)) <= ftol * np.max(np.abs(r)), (g, k)
    a_ref = sysm.accel(xg, m, w.gal, lost, list(cg), pots)
    e = T.rel_err_vec(acc, a_ref)
    if prec == sbx.SBX_FP64:
        assert e.max() < 1e-9
    else:
        assert np.percentile(e, 99) < 1e-4 and e.max() < 1e-3
