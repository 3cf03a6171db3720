"""CPU checks of the identities the plane-fused solve form is built on,
with numpy's FFT as the reference (no GPU, no oracle): a zero-padded
length-2N transform of N inputs as two length-N transforms, the first N
outputs of a length-2N inverse from its two halves, two real rows packed
as one complex line and separated by symmetry, the padded 2D/3D
convolution assembled from these pieces in the kernels' layouts, and the
two splits of a plane over two blocks (forward by kx parity, inverse by
row parity)."""
import numpy as np


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1210, 1736, 900, k]))


def test_padded_transform_as_two_halves():
    rng = _rng(0)
    for N in (16, 32, 128):
        f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        w = np.exp(-2j * np.pi * np.arange(N) / (2 * N))
        F = np.fft.fft(np.concatenate([f, np.zeros(N)]))
        assert np.allclose(F[0::2], np.fft.fft(f), atol=1e-12)
        assert np.allclose(F[1::2], np.fft.fft(f * w), atol=1e-12)
        # first N outputs of the unnormalised inverse from the two halves
        G = rng.standard_normal(2 * N) + 1j * rng.standard_normal(2 * N)
        g = np.fft.ifft(G) * 2 * N
        ge = np.fft.ifft(G[0::2]) * N
        go = np.fft.ifft(G[1::2]) * N
        assert np.allclose(g[:N], ge + np.conj(w) * go, atol=1e-10)


def test_two_real_rows_and_column_zero_separation():
    """Z = F(a + i b) gives F(a) = (Z(k) + conj Z(-k)) / 2 and
    F(b) = -i (Z(k) - conj Z(-k)) / 2; X(0) and X(N) of a real row are real,
    so a column of X(0) + i X(N) separates the same way after its transform."""
    rng = _rng(1)
    N = 32
    a, b = rng.standard_normal((2, 2 * N))
    Z = np.fft.fft(a + 1j * b)
    Zm = np.conj(np.roll(Z[::-1], 1))  # conj Z(-k)
    assert np.allclose((Z + Zm) / 2, np.fft.fft(a), atol=1e-12)
    assert np.allclose(-1j * (Z - Zm) / 2, np.fft.fft(b), atol=1e-12)
    A = np.fft.fft(np.concatenate([a[:N], np.zeros(N)]))
    assert abs(A[0].imag) < 1e-12 and abs(A[N].imag) < 1e-12


def test_plane_pipeline_equals_padded_convolution():
    """The three passes in the kernels' order and layouts (rows packed two
    to a line, even and odd halves of every padded line, column 0 packed as
    X(0) + i X(N), spectra as P[kx][z][ky']) against the zero-padded 3D
    convolution with an even kernel table."""
    rng = _rng(2)
    N, L = 8, 16
    rho = rng.standard_normal((N, N, N))            # [z][y][x]
    Hh = rng.standard_normal((N + 1, N + 1, N + 1))  # folded even table [kx][ky][kz]
    fold = lambda k: k if k <= N else L - k          # noqa: E731
    Hfull = Hh[np.ix_([fold(k) for k in range(L)], [fold(k) for k in range(L)], [fold(k) for k in range(L)])]
    pad = np.zeros((L, L, L)); pad[:N, :N, :N] = rho
    ref = (np.fft.ifftn(np.fft.fftn(pad) * Hfull.transpose(2, 1, 0)) * L ** 3).real[:N, :N, :N]
    w = np.exp(-2j * np.pi * np.arange(N) / L)
    P = np.zeros((N + 1, N, L), complex)            # [kx][z][ky']
    for z in range(N):
        S = np.zeros((N, N), complex)               # plane, column-major [kx][y]
        for j in range(N // 2):
            line = rho[z, 2 * j] + 1j * rho[z, 2 * j + 1]
            Ze, Zo = np.fft.fft(line), np.fft.fft(line * w)
            zat = lambda k: Ze[k >> 1] if k % 2 == 0 else Zo[k >> 1]  # noqa: E731
            for kx in range(N):
                Zk, R = zat(kx), zat(N if kx == 0 else L - kx)
                if kx == 0:
                    S[0, 2 * j], S[0, 2 * j + 1] = Zk.real + 1j * R.real, Zk.imag + 1j * R.imag
                else:
                    S[kx, 2 * j] = (Zk + np.conj(R)) / 2
                    S[kx, 2 * j + 1] = -1j * (Zk - np.conj(R)) / 2
        for kx in range(N):
            V = np.concatenate([np.fft.fft(S[kx]), np.fft.fft(S[kx] * w)])
            if kx:
                P[kx, z] = V
            else:
                for h in range(2):
                    for m in range(N):
                        mm = (N - 1 - m) if h else ((N - m) % N)
                        A, B = V[h * N + m], V[h * N + mm]
                        P[0, z, h * N + m] = (A + np.conj(B)) / 2
                        P[N, z, h * N + m] = -1j * (A - np.conj(B)) / 2
    kyof = np.array([2 * k if k < N else 2 * (k - N) + 1 for k in range(L)])
    Q = np.zeros_like(P)
    for kx in range(N + 1):
        for kp in range(L):
            line = np.concatenate([P[kx, :, kp], np.zeros(N)])
            Q[kx, :, kp] = (np.fft.ifft(np.fft.fft(line) * Hfull[kx, kyof[kp], :]) * L)[:N]
    out = np.zeros((N, N, N))
    for z in range(N):
        S = np.zeros((N, N), complex)
        for kx in range(N):
            e = Q[0, z] + 1j * Q[N, z] if kx == 0 else Q[kx, z]
            S[kx] = np.fft.ifft(e[:N]) * N + np.conj(w) * np.fft.ifft(e[N:]) * N
        xat = lambda y, k: S[0, y].real if k == 0 else (S[0, y].imag if k == N else S[k, y])  # noqa: E731
        for j in range(N // 2):
            Zs = np.array([xat(2 * j, k) + 1j * xat(2 * j + 1, k) if k <= N
                           else np.conj(xat(2 * j, L - k)) + 1j * np.conj(xat(2 * j + 1, L - k))
                           for k in range(L)])
            zz = np.fft.ifft(Zs[0::2]) * N + np.conj(w) * np.fft.ifft(Zs[1::2]) * N
            out[z, 2 * j], out[z, 2 * j + 1] = zz.real, zz.imag
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_half_plane_forward_by_kx_parity():
    """Columns kx of one parity take their row spectra from one of the two
    length-N transforms of each packed row pair only: for kx = 2m + h the
    padded row spectrum is that transform's output m (times w^n before it
    for h = 1), and so is the mirror 2N - kx (same parity), so the
    separation of the packed rows needs nothing from the other parity."""
    rng = _rng(3)
    N = 32
    L = 2 * N
    w = np.exp(-2j * np.pi * np.arange(N) / L)
    a, b = rng.standard_normal(N), rng.standard_normal(N)
    Fa = np.fft.fft(np.concatenate([a, np.zeros(N)]))
    Fb = np.fft.fft(np.concatenate([b, np.zeros(N)]))
    z = a + 1j * b
    for h in (0, 1):
        Zh = np.fft.fft(z * w ** h)          # the outputs m of parity h
        for kx in range(h, N, 2):
            Z = Zh[kx >> 1]
            R = Zh[(N if kx == 0 else L - kx) >> 1]
            if kx == 0:                      # X(0) + i X(N) of each row
                assert np.isclose(Z.real, Fa[0].real) and np.isclose(R.real, Fa[N].real)
                assert np.isclose(Z.imag, Fb[0].real) and np.isclose(R.imag, Fb[N].real)
            else:
                assert np.isclose((Z + np.conj(R)) / 2, Fa[kx])
                assert np.isclose(-1j * (Z - np.conj(R)) / 2, Fb[kx])


def test_half_plane_inverse_by_row_parity():
    """Rows y = 2p + hp of the first N outputs of a length-2N inverse come
    from two length-N/2 inverses of folded halves: with E and O the even
    and odd inputs and s = (-1)^hp, a = IDFT((E(m) + s E(m + N/2))
    e^{2 pi i m hp / N}), b the same of O, and row 2p + hp is
    a(p) + w^-(2p+hp) b(p)."""
    rng = _rng(4)
    for N in (16, 128):
        L, H = 2 * N, N // 2
        w = np.exp(-2j * np.pi * np.arange(N) / L)
        Q = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        full = (np.fft.ifft(Q) * L)[:N]
        E, O = Q[0::2], Q[1::2]
        for hp in (0, 1):
            s = -1.0 if hp else 1.0
            t = np.exp(2j * np.pi * np.arange(H) * hp / N)
            a = np.fft.ifft((E[:H] + s * E[H:]) * t) * H
            bb = np.fft.ifft((O[:H] + s * O[H:]) * t) * H
            y = 2 * np.arange(H) + hp
            assert np.allclose(a + np.conj(w[y]) * bb, full[y], atol=1e-9)
