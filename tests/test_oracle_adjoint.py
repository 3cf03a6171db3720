"""Pins of the oracle's segment adjoint: transposes by dot products, and the
gradients of the loss against central finite differences of the forward."""
import numpy as np
import pytest

from oracle import pm_oracle as O


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, 950, k]))


@pytest.mark.parametrize("taylor", [True, False])
def test_scatter_is_transpose_of_gather(taylor):
    """<A Phi, mu> = <Phi, A^T mu> for the Eq. 8 gather."""
    N = 16
    L = O.Level(N, 2.0, 0.5)
    rng = _rng(1)
    Phi = rng.normal(size=(N, N, N))
    n = 300
    idx = rng.integers(2, N - 2, size=(n, 3))
    dl = rng.uniform(-0.5, 0.5, size=(n, 3)) * L.lengths
    mu = rng.normal(size=(n, 3))
    a = O.eq8_accel(Phi, idx, dl, L.lengths, taylor)
    B = np.zeros_like(Phi)
    O.eq8_scatter_transpose(B, idx, dl, L.lengths, mu, taylor)
    assert np.sum(a * mu) == pytest.approx(np.sum(Phi * B), rel=1e-12)


def test_jacobian_is_derivative_of_gather():
    """Eq. 8 is linear in the in-cell offset: a(D + h e_b) - a(D) = h J e_b."""
    N = 16
    L = O.Level(N, 2.0, 0.25)
    rng = _rng(2)
    Phi = rng.normal(size=(N, N, N))
    idx = rng.integers(2, N - 2, size=(50, 3))
    dl = rng.uniform(-0.3, 0.3, size=(50, 3)) * L.lengths
    J = O.eq8_jacobian(Phi, idx, L.lengths)
    for b in range(3):
        h = np.zeros(3); h[b] = 1e-3 * L.lengths[b]
        da = O.eq8_accel(Phi, idx, dl + h, L.lengths) - O.eq8_accel(Phi, idx, dl, L.lengths)
        assert np.allclose(da, J[:, :, b] * h[b], rtol=1e-9, atol=1e-12 * np.abs(da).max())
    assert np.allclose(J, np.transpose(J, (0, 2, 1)))


def test_solve_is_symmetric():
    """<K A, B> = <A, K B> for the isolated convolution (H even)."""
    N = 16
    L = O.Level(N, 2.0, 0.5)
    Hh, _ = O.green_hat(L)
    rng = _rng(3)
    A = rng.normal(size=(N, N, N)); B = rng.normal(size=(N, N, N))
    assert np.sum(O.solve_fft(A, Hh) * B) == pytest.approx(np.sum(A * O.solve_fft(B, Hh)), rel=1e-12)


def _small_system(levels):
    rng = _rng(4)
    n = 600
    x = rng.normal(size=(n, 3)) * np.array([0.6, 0.6, 0.15])
    v = rng.normal(size=(n, 3)) * 0.3
    m = rng.uniform(0.5, 1.5, n) / n
    comp = (rng.uniform(size=n) < 0.5).astype(np.int8)
    gal = np.zeros(n, np.int8)
    sysm = O.System([O.Hierarchy(levels)])
    return sysm, x, v, m, comp, gal


@pytest.mark.parametrize("kind", ["single", "nested"])
def test_segment_gradients_match_finite_differences(kind):
    """dL/dm, dL/dx0, dL/dv0 of the reverse mode against central differences
    of the forward loss (step sizes small enough that no cell changes)."""
    if kind == "single":
        levels = [O.Level(32, 2.5)]
    else:
        levels = [O.Level(32, 0.5, 0.5), O.Level(32, 1.5, 0.5), O.Level(32, 4.0)]
    sysm, x, v, m, comp, gal = _small_system(levels)
    dt, K = 0.02, 4
    Lval, gm, gx, gv = O.segment_loss_and_grads(sysm, x, v, m, comp, gal, dt, K, 1, 0)

    def loss(x_, v_, m_):
        return _fwd(sysm, x_, v_, m_, comp, gal, dt, K)

    rng = _rng(5)
    for q in rng.choice(x.shape[0], 8, replace=False):
        eps = 1e-4 * m[q]
        mp = m.copy(); mp[q] += eps
        mm = m.copy(); mm[q] -= eps
        fd = (loss(x, v, mp) - loss(x, v, mm)) / (2 * eps)
        assert fd == pytest.approx(gm[q], rel=2e-5, abs=1e-9 * abs(gm).max())
        a = int(rng.integers(0, 3))
        h = 1e-7
        vp = v.copy(); vp[q, a] += h
        vm = v.copy(); vm[q, a] -= h
        fd = (loss(x, vp, m) - loss(x, vm, m)) / (2 * h)
        assert fd == pytest.approx(gv[q, a], rel=1e-4, abs=1e-6 * abs(gv).max())
        xp = x.copy(); xp[q, a] += h
        xm = x.copy(); xm[q, a] -= h
        fd = (loss(xp, v, m) - loss(xm, v, m)) / (2 * h)
        assert fd == pytest.approx(gx[q, a], rel=1e-4, abs=1e-6 * abs(gx).max())


def _fwd(sysm, x, v, m, comp, gal, dt, K):
    lost = np.zeros(x.shape[0], bool)
    for _ in range(K):
        x, v, lost, _ = sysm.step(x, v, m, gal, lost, dt)
    sel = (comp == 1) & (gal == 0) & ~lost
    return 0.5 * np.sum(m[sel] * v[sel, 2] ** 2)


@pytest.mark.parametrize("kind", ["single", "nested"])
def test_segment_gradients_with_particles_lost_mid_segment(kind):
    """Four heavy particles take part in cycles 0 and 1 of a 4-cycle segment
    and leave the outermost grid in the drift of cycle 1 (Sec. 2.1 particle
    loss).  Their masses shaped the fields of cycles 0 and 1, so dL/dm of each
    is nonzero and equals the central difference of the forward loss; they
    are not in the loss and their cells are piecewise constant, so dL/dx and
    dL/dv vanish.  Cloud particles are checked as in the plain segment."""
    import synth
    w = synth.escape_segment(kind)
    from tests import common as T
    sysm = T.oracle_system(w)
    esc = np.arange(w.n - 4, w.n)
    # the set-up: escapers live in cycles 0 and 1, lost from cycle 2 on
    x, v, lost = w.x.copy(), w.v.copy(), np.zeros(w.n, bool)
    for k in range(w.steps):
        live = ~(lost | sysm.lost_now(x))
        assert bool(live[esc].all()) == (k < 2) and bool(live[esc].any()) == (k < 2)
        x, v, lost, _ = sysm.step(x, v, w.m, w.gal, lost, w.dt)
    assert lost[esc].all() and lost.sum() == 4
    L, gm, gx, gv = O.segment_loss_and_grads(sysm, w.x, w.v, w.m, w.comp, w.gal, w.dt, w.steps, 1, 0)
    assert L == pytest.approx(_fwd(sysm, w.x, w.v, w.m, w.comp, w.gal, w.dt, w.steps), rel=1e-14)

    def loss(x_, v_, m_):
        return _fwd(sysm, x_, v_, m_, w.comp, w.gal, w.dt, w.steps)

    for q in esc:
        eps = 1e-4 * w.m[q]
        mp = w.m.copy(); mp[q] += eps
        mm = w.m.copy(); mm[q] -= eps
        fd = (loss(w.x, w.v, mp) - loss(w.x, w.v, mm)) / (2 * eps)
        assert abs(gm[q]) > 1e-6 * abs(gm).max()
        assert fd == pytest.approx(gm[q], rel=2e-5)
        assert not gx[q].any() and not gv[q].any()
    rng = _rng(6)
    for q in rng.choice(w.n - 4, 4, replace=False):
        eps = 1e-4 * w.m[q]
        mp = w.m.copy(); mp[q] += eps
        mm = w.m.copy(); mm[q] -= eps
        fd = (loss(w.x, w.v, mp) - loss(w.x, w.v, mm)) / (2 * eps)
        assert fd == pytest.approx(gm[q], rel=2e-5, abs=1e-9 * abs(gm).max())
        a = int(rng.integers(0, 3))
        h = 1e-7
        vp = w.v.copy(); vp[q, a] += h
        vm = w.v.copy(); vm[q, a] -= h
        fd = (loss(w.x, vp, w.m) - loss(w.x, vm, w.m)) / (2 * h)
        assert fd == pytest.approx(gv[q, a], rel=1e-4, abs=1e-6 * abs(gv).max())
