"""Pins of the oracle's own FFT and tensor algebra (no GPU).

The oracle's naive mixed-radix FFT is pinned against the O(n^2) definition of
the DFT written with numpy, and the discrete convolution of eq. DiscConv
computed through that FFT is pinned against the direct O(N^2d) sum.
"""
import numpy as np
import pytest

from oracle import oracle as O


def dft_matrix(n, sign):
    j = np.arange(n)
    # reduce j k mod n first so the matrix entries are exact to rounding
    return np.exp(sign * 2j * np.pi * (np.outer(j, j) % n) / n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 24, 30, 48, 64, 96, 97, 128, 192, 384])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_matches_dft_definition(n, sign):
    rng = np.random.default_rng(n * 7 + (sign > 0))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = dft_matrix(n, sign) @ x
    got = O.fft1d(x, sign)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_fft1d_roundtrip_and_impulse():
    n = 48
    e = np.zeros(n, complex)
    e[5] = 1.0
    got = O.fft1d(e, -1)
    assert np.allclose(got, np.exp(-2j * np.pi * 5 * np.arange(n) / n), atol=1e-15)
    x = np.random.default_rng(0).standard_normal(n) + 0j
    back = O.fft1d(O.fft1d(x, -1), +1) / n
    assert np.max(np.abs(back - x)) < 1e-14


@pytest.mark.parametrize("shape", [(6, 10, 8), (16, 12), (4, 4, 4), (24, 20)])
def test_fftnd_is_separable_dft(shape):
    rng = np.random.default_rng(len(shape))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = a.copy()
    for ax, n in enumerate(shape):
        ref = np.moveaxis(np.tensordot(dft_matrix(n, -1), np.moveaxis(ref, ax, 0), axes=1), 0, ax)
    got = O.fftnd(a, -1)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def brute_conv(T, rho):
    """eq. DiscConv written out: Phi_i = sum_{i'} T_{(i - i') mod P} rho_{i'}."""
    N = rho.shape
    P = T.shape
    phi = np.zeros(N)
    for i in np.ndindex(*N):
        acc = 0.0
        for ip in np.ndindex(*N):
            m = tuple((a - b) % p for a, b, p in zip(i, ip, P))
            acc += T[m] * rho[ip]
        phi[i] = acc
    return phi


def test_direct_sum_matches_brute_force_tiny():
    rng = np.random.default_rng(3)
    N = (4, 6)
    T = rng.standard_normal((8, 12))
    rho = rng.standard_normal(N)
    assert np.allclose(O.conv_direct(T, rho), brute_conv(T, rho), rtol=0, atol=1e-13)
    N3 = (2, 4, 2)
    T3 = rng.standard_normal((4, 8, 4))
    rho3 = rng.standard_normal(N3)
    assert np.allclose(O.conv_direct(T3, rho3), brute_conv(T3, rho3), rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind,L,N", [
    ("coulomb3d", (8.0, 8.0, 8.0), (8, 8, 8)),
    ("coulomb3d", (3.0, 5.0, 4.0), (12, 10, 16)),
    ("yukawa3d", (4.0, 4.0, 4.0), (16, 16, 16)),
    ("log2d", (6.0, 4.0), (24, 20)),
    ("log2d", (8.0, 8.0), (64, 64)),
    ("coulomb2d", (5.0, 7.0), (18, 30)),
    ("biharmonic3d", (4.0, 4.0, 4.0), (10, 12, 8)),
    ("biharmonic2d", (4.0, 6.0), (16, 14)),
])
def test_fft_route_equals_direct_sum(kind, L, N):
    rng = np.random.default_rng(sum(N))
    rho = rng.standard_normal(N)
    eps = 2.0 * min(L) / 8.0
    T = O.build_tensor(kind, L, N, eps, lam=1.0 if kind == "yukawa3d" else 0.0)
    a = O.conv_fft(T, rho)
    b = O.conv_direct(T, rho)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_direct_points_match_full_direct():
    rng = np.random.default_rng(11)
    N = (10, 8, 12)
    T = O.build_tensor("coulomb3d", (4.0, 4.0, 4.0), N, 1.0)
    rho = rng.standard_normal(N)
    full = O.conv_direct(T, rho)
    idx = rng.choice(full.size, 37, replace=False)
    assert np.allclose(O.conv_direct_points(T, rho, idx), full.ravel()[idx], rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind,L,N", [
    ("coulomb3d", (8.0, 8.0, 8.0), (16, 16, 16)),
    ("log2d", (8.0, 6.0), (32, 24)),
    ("yukawa3d", (6.0, 6.0, 6.0), (12, 16, 12)),
])
def test_tensor_real_and_even(kind, L, N):
    """T(2) = IDFT(W) of a real even W is real; T is even on every axis (Sec. 2.3)."""
    eps = 2.0 * min(L) / 8.0
    T, T1, T2, imax = O.build_tensor(kind, L, N, eps, lam=0.5, parts=True)
    assert imax <= 1e-15 * np.max(np.abs(T2)) * 10
    for ax in range(T.ndim):
        P = T.shape[ax]
        flipped = np.take(T, (-np.arange(P)) % P, axis=ax)
        assert np.max(np.abs(flipped - T)) <= 1e-15 * np.max(np.abs(T)) * 10
    assert np.allclose(T, T1 + T2, rtol=0, atol=0)


def test_impulse_response_is_the_tensor():
    """Applying the solver to a unit impulse at grid index c returns T_{i - c}."""
    L, N = (6.0, 6.0, 6.0), (12, 12, 12)
    T = O.build_tensor("coulomb3d", L, N, 1.5)
    c = (6, 3, 9)
    rho = np.zeros(N)
    rho[c] = 1.0
    phi = O.conv_fft(T, rho)
    idx = np.meshgrid(*[(np.arange(n) - cc) % (2 * n) for n, cc in zip(N, c)], indexing="ij")
    assert np.max(np.abs(phi - T[tuple(idx)])) <= 1e-14 * np.max(np.abs(T))


def test_linearity():
    rng = np.random.default_rng(5)
    L, N = (5.0, 5.0), (20, 20)
    T = O.build_tensor("log2d", L, N, 1.25)
    r1, r2 = rng.standard_normal(N), rng.standard_normal(N)
    lhs = O.conv_fft(T, 2.5 * r1 - 0.75 * r2)
    rhs = 2.5 * O.conv_fft(T, r1) - 0.75 * O.conv_fft(T, r2)
    assert np.linalg.norm(lhs - rhs) <= 1e-14 * np.linalg.norm(rhs)


def test_rejects_bad_geometry():
    with pytest.raises(ValueError):
        O.build_tensor("coulomb3d", (1.0, 1.0, 1.0), (7, 8, 8), 0.2)
    with pytest.raises(ValueError):
        O.build_tensor("coulomb3d", (1.0, 1.0), (8, 8), 0.2)
    with pytest.raises(ValueError):
        O.build_tensor("log2d", (1.0, -1.0), (8, 8), 0.2)


def test_direct_sum_is_compensated():
    """Same-signed terms: the direct sum matches a long-double sum to a few ulps."""
    rng = np.random.default_rng(21)
    N = (40, 40, 40)
    T = rng.uniform(0.5, 1.5, size=(80, 80, 80))
    rho = rng.uniform(0.5, 1.5, size=N)
    idx = rng.choice(rho.size, 6, replace=False)
    got = O.conv_direct_points(T, rho, idx)
    for v, i in zip(got, idx):
        i0, i1, i2 = np.unravel_index(i, N)
        sub = T[np.ix_((i0 - np.arange(40)) % 80, (i1 - np.arange(40)) % 80,
                       (i2 - np.arange(40)) % 80)]
        ref = np.sum((sub * rho).astype(np.longdouble), dtype=np.longdouble)
        assert abs(v - float(ref)) <= 4e-16 * abs(float(ref))
