"""The oracle against the paper's printed results and exact potentials (no GPU).

A match of the coarse-grid errors to the printed significant digits pins the
grid convention (eq. UniformMesh), T(1) (eq. Tensor1), W and k_p (eq. FouTran,
Table 1), T(2) (eq. Tensor2), the r = 0 value and the crop all at once.  The
planted-mistake tests show that each plausible slip fails one of the pins.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import reference as R
from paper_2504_19410_amd import synth


def iso_setup(d, L, N, sigma2):
    axes = O.grid_axes([L] * d, [N] * d)
    X = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(sum(x * x for x in X))
    return r, np.exp(-r * r / sigma2)


def iso_exact(kind, r, sigma2, lam=0.0):
    s = np.sqrt(sigma2)
    if kind == "coulomb3d":
        return R.coulomb3d_iso(r, 1.0, s)
    if kind == "log2d":
        return R.log2d_iso(r, 1.0, s)
    if kind == "yukawa3d":
        return R.yukawa3d_iso(r, 1.0, s, lam)
    raise ValueError(kind)


def sig2(v):
    """Rounded to two significant digits: the precision the pins hold the printed values to."""
    return float(f"{v:.1e}")


@pytest.mark.parametrize("key,kind,d,cases", [
    ("coulomb3d_iso", "coulomb3d", 3, [0, 1]),
    ("log2d_iso", "log2d", 2, [0, 1, 2]),
])
def test_printed_coarse_errors(golden, key, kind, d, cases):
    g = golden[key]
    for c in cases:
        h = g["h"][c]
        N = int(round(2 * g["L"] / h))
        r, rho = iso_setup(d, g["L"], N, g["sigma2"])
        phi = O.solve(kind, [g["L"]] * d, [N] * d, rho, eps=g["eps"])
        err = R.rel_max_err(phi, iso_exact(kind, r, g["sigma2"]))
        # the oracle reproduces four significant digits; assert the printed value to 1e-3 relative
        assert abs(err - g["err"][c]) <= 1e-3 * g["err"][c], (key, h, err, g["err"][c])


def test_printed_coulomb2d_errors(golden):
    g = golden["coulomb2d_iso"]
    s = np.sqrt(g["sigma2"])
    for c, printed in [(0, g["err"][0]), (1, 2.9648e-06)]:  # h=1/2 exponent read as -06
        N = int(round(2 * g["L"] / g["h"][c]))
        _, rho = iso_setup(2, g["L"], N, g["sigma2"])
        phi = O.solve("coulomb2d", [g["L"]] * 2, [N] * 2, rho, eps=g["eps"])
        ex = R.gaussian_sum_potential("coulomb2d", [(1.0, [0, 0], [s, s])], [g["L"]] * 2, [N] * 2)
        err = R.rel_max_err(phi, ex)
        assert abs(err - printed) <= 1e-3 * printed, (c, err)


def biharmonic3d_exact(r, sigma2):
    """Phi(r) = (1/4) int_0^inf rho(s) s [(r+s)^3 - |r-s|^3] / (3r) ds for the
    radial density rho = exp(-s^2/sigma2) and U = |x|/(8 pi) (angular integral
    done in closed form); Gauss-Legendre on [0, 40] split at r."""
    from numpy.polynomial.legendre import leggauss
    xg, wg = leggauss(200)
    out = np.empty_like(r)
    ur, inv = np.unique(np.round(r, 12), return_inverse=True)
    vals = np.empty_like(ur)
    for i, rv in enumerate(ur):
        tot = 0.0
        for a, b in ([(0.0, rv), (rv, 40.0)] if rv > 0 else [(0.0, 40.0)]):
            s = 0.5 * (b - a) * xg + 0.5 * (a + b)
            w = 0.5 * (b - a) * wg
            rho = np.exp(-s * s / sigma2)
            if rv == 0:
                f = rho * s * s * s * 0.5  # 4 pi s^2 * s/(8 pi)
            else:
                f = 0.25 * rho * s * ((rv + s) ** 3 - np.abs(rv - s) ** 3) / (3 * rv)
            tot += np.sum(w * f)
        vals[i] = tot
    out[...] = vals[inv].reshape(r.shape)
    return out


def test_printed_biharmonic3d_errors(golden):
    g = golden["biharmonic3d_iso"]
    for c in (0, 1, 2):
        N = int(round(2 * g["L"] / g["h"][c]))
        r, rho = iso_setup(3, g["L"], N, g["sigma2"])
        phi = O.solve("biharmonic3d", [g["L"]] * 3, [N] * 3, rho, eps=g["eps"])
        err = R.rel_max_err(phi, biharmonic3d_exact(r, g["sigma2"]))
        assert abs(err - g["err"][c]) <= 1e-3 * g["err"][c], (c, err)


def biharmonic2d_exact(r, sigma2):
    """Phi(r) = -(1/4) int_0^inf rho(s) s [(A^2 + B^2)(ln A - 1) + B^2] ds,
    A = max(r, s), B = min(r, s), for rho = exp(-s^2/sigma2) and
    U = -|x|^2 (ln|x| - 1)/(8 pi): the circle average of q^2 ln q^2 over
    |y| = s is 2(A^2 + B^2) ln A + 2 B^2 (Fourier series of ln|1 - z e^{it}|);
    40-point Gauss-Legendre on panels of width 1/2 over [0, 8], where the
    density lives (e^{-64/1.2} beyond), split at r.  Each distinct r is integrated as it is: grouping radii rounded
    to 12 decimals moved the far-corner values by ~5e-12 (dPhi/dr ~ 10 there),
    which an mpmath evaluation of the same integral at 40 digits showed to be
    the whole of the 6.5e-14 relative error this test used to see.
    The sums run in extended precision (x87 long double), and the rule is
    short-panelled, since 200-point nodes left ~3e-13 at the corners."""
    from numpy.polynomial.legendre import leggauss
    ld = np.longdouble
    xg, wg = leggauss(40)
    xg, wg = xg.astype(ld), wg.astype(ld)
    out = np.empty_like(r)
    ur, inv = np.unique(r, return_inverse=True)
    vals = np.empty_like(ur)
    base = {ld(0.5 * k) for k in range(17)}
    for i, rv in enumerate(ur):
        tot = ld(0.0)
        rv = ld(rv)
        cuts = sorted(base | ({rv} if 0.0 < rv < 8.0 else set()))
        for a, b in zip(cuts[:-1], cuts[1:]):
            s = (b - a) / 2 * xg + (a + b) / 2
            w = (b - a) / 2 * wg
            A, B = np.maximum(rv, s), np.minimum(rv, s)
            f = np.exp(-s * s / ld(sigma2)) * s * ((A * A + B * B) * (np.log(A) - 1) + B * B)
            tot += np.sum(w * f)
        vals[i] = float(-tot / 4)
    out[...] = vals[inv].reshape(r.shape)
    return out


def test_biharmonic2d_reference_against_mpmath(golden):
    """The quadrature reference of the 2D biharmonic potential agrees with a
    40-digit mpmath evaluation of the same radial integral to 2e-16 of the
    potential's maximum on the grid (its far-corner value, the scale of the
    relative max error), at the centre and at far-corner radii of Table 5's
    h = 1/4 grid, so it cannot hide an oracle error at the printed level."""
    mp = pytest.importorskip("mpmath")
    g = golden["biharmonic2d_iso"]
    s2 = g["sigma2"]
    radii = np.array([0.0, 5.0, 15.388713396512394, 16.97056274847714])
    ref = biharmonic2d_exact(radii, s2)
    mp.mp.dps = 40
    S2 = mp.mpf(s2)
    exact = []
    for rv in radii:
        R = mp.mpf(rv)

        def f(s):
            A, B = (R, s) if R > s else (s, R)
            la = mp.log(A) if A > 0 else mp.mpf(0)
            return mp.exp(-s * s / S2) * s * ((A * A + B * B) * (la - 1) + B * B)
        pts = sorted({mp.mpf(0), mp.mpf(4), mp.mpf(8), mp.mpf(40)} | ({R} if 0 < R < 40 else set()))
        exact.append(-mp.quad(f, pts) / 4)
    scale = float(max(abs(e) for e in exact))
    for rv, got, ex in zip(radii, ref, exact):
        assert abs(mp.mpf(got) - ex) <= 2e-16 * scale, (rv, got, ex)


def test_printed_biharmonic2d_errors(golden):
    g = golden["biharmonic2d_iso"]
    for c in range(4):
        N = int(round(2 * g["L"] / g["h"][c]))
        r, rho = iso_setup(2, g["L"], N, g["sigma2"])
        phi = O.solve("biharmonic2d", [g["L"]] * 2, [N] * 2, rho, eps=g["eps"])
        err = R.rel_max_err(phi, biharmonic2d_exact(r, g["sigma2"]))
        if c < 3:
            assert abs(err - g["err"][c]) <= 1e-3 * g["err"][c], (c, err)
        else:
            # printed 1.29e-15; against this reference (within 1.5e-16 of a
            # 40-digit mpmath evaluation at the corners) the oracle reaches
            # 2.0e-15, at the far corner where U grows like r^2 ln r: the
            # round-off of the FFT convolution
            assert err <= 3e-15, err


def ddi_setup(g, h):
    N = int(round(2 * g["L"] / h))
    axes = O.grid_axes([g["L"]] * 3, [N] * 3)
    X = np.meshgrid(*axes, indexing="ij")
    rho = np.exp(-sum(x * x for x in X) / g["sigma2"])
    return N, X, rho


def test_printed_ddi3d_errors(golden):
    """Table 5's 3D DDI row against the exact potential -(m.n) rho - 3 d_nm Phi_C."""
    g = golden["ddi3d_iso"]
    s = np.sqrt(g["sigma2"])
    for c in range(4):
        N, X, rho = ddi_setup(g, g["h"][c])
        phi = O.solve_ddi([g["L"]] * 3, [N] * 3, rho, g["eps"], g["n"], g["m"])
        err = R.rel_max_err(phi, R.ddi3d_iso(X, 1.0, s, g["n"], g["m"]))
        if c < 3:
            assert abs(err - g["err"][c]) <= 1e-3 * g["err"][c], (c, err)
        else:
            assert err <= 1e-13, err   # printed 7.57e-15: round-off level


def test_ddi_readings_that_miss_the_printed_row(golden):
    """The printed DDI errors pin the derivative step: the derivative taken on
    the 2N-padded grid (the Coulomb convolution's own grid), or the exact
    derivative of the Gaussian sampled on the grid, give other values at h = 1
    and h = 1/2 (computed here with numpy, on the CPU)."""
    g = golden["ddi3d_iso"]
    s = np.sqrt(g["sigma2"])
    n, m = np.array(g["n"]), np.array(g["m"])
    for c in (1, 2):
        N, X, rho = ddi_setup(g, g["h"][c])
        L = g["L"]
        exact = R.ddi3d_iso(X, 1.0, s, n, m)
        T = O.build_tensor("coulomb3d", [L] * 3, [N] * 3, g["eps"])
        # (a) spectral derivative on the padded grid
        P = 2 * N
        pad = np.zeros((P,) * 3)
        pad[:N, :N, :N] = rho
        k = np.pi * np.fft.fftfreq(P, 1.0 / P) / (2 * L)
        K = np.meshgrid(k, k, k, indexing="ij")
        kn = sum(K[i] * n[i] for i in range(3))
        km = sum(K[i] * m[i] for i in range(3))
        Da = np.real(np.fft.ifftn(-kn * km * np.fft.fftn(pad)))[:N, :N, :N]
        # (b) exact derivative of the Gaussian, sampled
        xn = sum(X[i] * n[i] for i in range(3))
        xm = sum(X[i] * m[i] for i in range(3))
        Db = (4 * xn * xm / g["sigma2"] ** 2 - 2 * float(n @ m) / g["sigma2"]) * rho
        for D in (Da, Db):
            err = R.rel_max_err(-float(n @ m) * rho - 3 * O.conv_fft(T, D), exact)
            assert sig2(err) != sig2(g["err"][c]), (c, err)


def test_yukawa_h_half_entry(golden):
    """The only Yukawa entry the unstated split does not decide (see fixture reading)."""
    g = golden["yukawa3d_iso"]
    N = int(round(2 * g["L"] / 0.5))
    r, rho = iso_setup(3, g["L"], N, g["sigma2"])
    phi = O.solve("yukawa3d", [g["L"]] * 3, [N] * 3, rho, eps=g["eps"], lam=2.0)
    err = R.rel_max_err(phi, iso_exact("yukawa3d", r, g["sigma2"], lam=2.0))
    assert sig2(err) == sig2(g["err"][2])


@pytest.mark.parametrize("kind,d,lam", [("coulomb3d", 3, 0.0), ("log2d", 2, 0.0), ("yukawa3d", 3, 1.0)])
def test_machine_precision_when_resolved(kind, d, lam):
    """Spectral accuracy: the fine-grid rows of Tables 2, 4, 5 are at round-off."""
    L, sigma2 = 8.0, 1.2
    N = 64 if d == 3 else 128
    r, rho = iso_setup(d, L, N, sigma2)
    phi = O.solve(kind, [L] * d, [N] * d, rho, eps=1.0, lam=lam)
    assert R.rel_max_err(phi, iso_exact(kind, r, sigma2, lam)) <= 2e-14


def test_spectral_convergence_log2d():
    L, sigma2 = 8.0, 1.2
    errs = []
    for N in (8, 16, 32, 64):
        r, rho = iso_setup(2, L, N, sigma2)
        phi = O.solve("log2d", [L, L], [N, N], rho, eps=1.0)
        errs.append(R.rel_max_err(phi, iso_exact("log2d", r, sigma2)))
    # error ~ exp(-c/h^2): each halving of h at least squares the improvement
    assert errs[1] < errs[0] / 100 and errs[2] < errs[1] / 1e4 and errs[3] < 1e-14


@pytest.mark.parametrize("gamma3", [1.0, 0.5, 0.25])
def test_anisotropic_case1_coulomb3d(golden, gamma3):
    """Table 2 anisotropic Case I: L=8, sigma^2=1.2, eps=0.5, h=gamma/4 (N=64)."""
    g = golden["coulomb3d_aniso_case1"]
    L = [g["L"], g["L"], g["L"] * gamma3]
    N = [64, 64, 64]
    s = np.sqrt(g["sigma2"])
    widths = [s, s, s * gamma3]
    rho = synth.eval_gaussians([synth.Gaussian(1.0, (0, 0, 0), tuple(widths))], L, N)
    phi = O.solve("coulomb3d", L, N, rho, eps=g["eps"])
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([rng.choice(phi.size, 600, replace=False),
                                    np.ravel_multi_index((32, 32, np.arange(64)), N),
                                    np.ravel_multi_index((np.arange(64), 32, 32), N)]))
    ex = R.gaussian_sum_potential("coulomb3d", [(1.0, [0, 0, 0], widths)], L, N, points=idx)
    err = np.max(np.abs(phi.ravel()[idx] - ex)) / np.max(np.abs(ex))
    assert err <= 2e-14


@pytest.mark.parametrize("gamma2", [1.0, 0.5, 0.25, 0.125])
def test_anisotropic_case2_log2d(golden, gamma2):
    """Table 4 anisotropic row: L=10, sigma=1.2, eps=0.4, h=(1,gamma2)/8, rho=-Laplace(Phi)."""
    g = golden["log2d_aniso_case2"]
    L = [g["L"], g["L"] * gamma2]
    N = [160, 160]
    rho = synth.case2_density(L, N, g["sigma"], [1.0, gamma2])
    phi = O.solve("log2d", L, N, rho, eps=g["eps"])
    ex = R.case2_phi0(L, N, g["sigma"], [1.0, gamma2])
    assert R.rel_max_err(phi, ex) <= 1e-14


def test_case2_shifted_coulomb3d():
    """Case II with a shifted copy (Sec. 5.1): Phi = Phi0(x) + Phi0(x - x0), with the
    paper's eps = 0.4 and h = 1/8 on a reduced box [-8,8]^2 x [-4,4] (gamma3 = 1/2)."""
    L = [8.0, 8.0, 4.0]
    N = [128, 128, 64]
    sigma = np.sqrt(0.8)
    rho = synth.case2_density(L, N, sigma, [1, 1, 0.5], x0=(1.0, 1.0, 0.0))
    phi = O.solve("coulomb3d", L, N, rho, eps=0.4)
    ex = R.case2_phi0(L, N, sigma, [1, 1, 0.5], x0=(1.0, 1.0, 0.0))
    assert R.rel_max_err(phi, ex) <= 1e-13


@pytest.mark.parametrize("kind,lam", [("coulomb3d", 0.0), ("yukawa3d", 0.7), ("biharmonic3d", 0.0),
                                      ("log2d", 0.0), ("coulomb2d", 0.0), ("biharmonic2d", 0.0)])
def test_eps_independence(kind, lam):
    """Theorem 1: once eps meets condition (b) of eq. ApproxProp and the grid
    resolves U^eps, the result does not depend on eps.  U^eps enters through
    T(1) and W through T(2), so a slip in either (a dropped term, a wrong
    sign or scale) leaves an eps-dependent residue: this pins the pair for
    every kernel, including those with no printed error table."""
    d = O.KIND_DIM[kind]
    n = 48 if d == 3 else 64
    L, N = [8.0] * d, [n] * d
    r, rho = iso_setup(d, 8.0, n, 2.0)
    a = O.solve(kind, L, N, rho, eps=16.0 / 8.0, lam=lam)
    b = O.solve(kind, L, N, rho, eps=16.0 / 6.0, lam=lam)
    assert R.rel_l2_err(a, b) <= 1e-13


@pytest.mark.parametrize("kind,lam", [("yukawa3d", 0.7), ("coulomb2d", 0.0), ("biharmonic2d", 0.0)])
def test_eps_independence_detects_a_planted_w_error(kind, lam):
    """The pin above is sensitive: W scaled by 1.01 (planted in T(2), on the
    CPU) moves the two eps results apart by many orders above 1e-13."""
    d = O.KIND_DIM[kind]
    n = 48 if d == 3 else 64
    L, N = [8.0] * d, [n] * d
    r, rho = iso_setup(d, 8.0, n, 2.0)
    out = []
    for eps in (16.0 / 8.0, 16.0 / 6.0):
        _, t1, t2, _ = O.build_tensor(kind, L, N, eps, lam=lam, parts=True)
        out.append(O.conv_fft(t1 + 1.01 * t2, rho))
    assert R.rel_l2_err(out[0], out[1]) > 1e-6


def test_isotropic_coulomb_32_against_closed_form():
    """The 32^3 three-Gaussian workload (h = 1/2, widths >= 0.8): the oracle's
    error against the closed form is 4.3e-9 for this seed."""
    p = synth.isotropic_coulomb_32()
    rho = synth.eval_gaussians(p.gaussians, p.L, p.N)
    phi = O.solve("coulomb3d", p.L, p.N, rho, eps=2.0)
    ex = R.gaussian_sum_potential("coulomb3d", [(g.amp, g.center, g.width) for g in p.gaussians],
                                  p.L, p.N)
    err = R.rel_max_err(phi, ex)
    assert err <= 1e-8


# ----------------------------------------------------------------------------
# Planted mistakes: each plausible slip in the discretisation breaks a pin.
# ----------------------------------------------------------------------------

def _coulomb32_error(T):
    r, rho = iso_setup(3, 8.0, 32, 0.8)
    return R.rel_max_err(O.conv_fft(T, rho), iso_exact("coulomb3d", r, 0.8))


def test_planted_mistakes_fail_the_pin(golden):
    printed = golden["coulomb3d_iso"]["err"][1]
    L, N = [8.0] * 3, [32] * 3
    T, T1, T2, _ = O.build_tensor("coulomb3d", L, N, 1.0, parts=True)
    assert abs(_coulomb32_error(T) - printed) <= 1e-3 * printed
    # dropped singular part
    assert _coulomb32_error(T1) > 1e-2
    # wrong sign of the singular part
    assert _coulomb32_error(T1 - T2) > 1e-2
    # wrong Fourier grid scale k = pi p / L instead of pi p / (2L)
    P = 64
    p = np.arange(P)
    p = np.where(p < 32, p, p - P)
    K = np.meshgrid(*([np.pi * p / 8.0] * 3), indexing="ij")
    W = O.what("coulomb3d", np.sqrt(sum(k * k for k in K)), 1.0)
    T2_bad = np.real(O.fftnd(W, +1)) / P ** 3
    assert _coulomb32_error(T1 + T2_bad) > 1e-3
    # dropped h^d factor on T(1)
    assert _coulomb32_error(T1 / 0.125 + T2) > 1e-1
    # grid shifted by one cell (x = -L + (i+1) h) against the exact potential
    axes = [(-8.0 + (np.arange(32) + 1) * 0.5)] * 3
    X = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(sum(x * x for x in X))
    _, rho = iso_setup(3, 8.0, 32, 0.8)
    assert R.rel_max_err(O.conv_fft(T, rho), iso_exact("coulomb3d", r, 0.8)) > 1e-2
