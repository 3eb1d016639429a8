"""The oracle's general construction (Sec. 4, eq. GeneralApprox1 with W by
quadrature of eq. Fourier-Symmetric) against what fixes it (no GPU).

* its Bessel functions K0 and J0 against a library routine;
* its quadrature W against the closed forms of Table 1, for the kernels whose
  U erf(r/eps) is smooth (window xi = 0, so U^eps is Table 1's);
* its windowed W against an independent quadrature written here with scipy;
* the potentials against the printed Table 5 rows (2D and 3D Yukawa,
  quasi-2D DDI) and against exact potentials of Gaussians at round-off;
* eps-independence (Theorem 1) and agreement with the closed-form route.
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import oracle as O
from oracle import reference as R


def iso_grid(d, L, N, sigma2):
    axes = O.grid_axes([L] * d, [N] * d)
    X = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(sum(x * x for x in X))
    return X, r, np.exp(-r * r / sigma2)


def yukawa_exact(d, X, sigma2, lam):
    s = np.sqrt(sigma2)
    if d == 3:
        return R.yukawa3d_iso(np.sqrt(sum(x * x for x in X)), 1.0, s, lam)
    return R.gaussian_sum_potential("yukawa2d", [(1.0, [0.0, 0.0], [s, s])],
                                    [float(-X[0][0, 0])] * 2, list(X[0].shape), lam=lam)


# ---------------------------------------------------------------------------
# Special functions
# ---------------------------------------------------------------------------

def test_k0_against_library():
    x = np.geomspace(1e-10, 300.0, 2000)
    assert np.max(np.abs(O.k0(x) / special.k0(x) - 1.0)) <= 2e-14
    x = np.geomspace(1e-10, 5000.0, 2000)
    assert np.max(np.abs(O.k0e(x) / special.k0e(x) - 1.0)) <= 2e-14


def test_j0_against_library():
    # both branches (Bessel's integral below 25, Hankel's expansion above)
    x = np.concatenate([np.linspace(0.0, 40.0, 4001), np.geomspace(40.0, 3000.0, 2000)])
    assert np.max(np.abs(O.j0(x) - special.j0(x))) <= 5e-15
    # both sides of the branch point
    x = 25.0 + np.array([-1e-9, -1e-12, 0.0, 1e-12, 1e-9])
    assert np.max(np.abs(O.j0(x) - special.j0(x))) <= 5e-15


# ---------------------------------------------------------------------------
# W by quadrature
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["coulomb3d", "coulomb2d", "biharmonic3d"])
@pytest.mark.parametrize("eps", [0.5, 1.0, 2.0])
def test_quadrature_w_equals_table1(kind, eps):
    """For these kernels U erf(r/eps) is smooth, the window is off, U^eps is
    Table 1's, and the quadrature of eq. Fourier-Symmetric must reproduce
    Table 1's closed-form transform."""
    assert not O.windowed(kind)
    k = np.concatenate([[0.0], np.geomspace(1e-3, 120.0, 60)])
    wq = O.what_general(kind, k, eps)
    wc = O.what(kind, k, eps)
    assert np.max(np.abs(wq - wc)) <= 2e-15 * abs(wc[0])
    r = np.linspace(0.0, 20.0, 201)
    assert np.allclose(O.ueps_general(kind, r, eps), O.ueps(kind, r, eps), rtol=1e-15, atol=0)


def _u_scipy(kind, r, lam, eta):
    if kind == "yukawa2d":
        return special.k0(lam * r) / (2 * np.pi)
    if kind == "yukawa3d":
        return np.exp(-lam * r) / (4 * np.pi * r)
    if kind == "log2d":
        return -np.log(r) / (2 * np.pi)
    if kind == "biharmonic2d":
        return -r * r * (np.log(r) - 1.0) / (8 * np.pi)
    if kind == "quasi2d_ddi":
        return special.k0e(r * r / (4 * eta * eta)) / ((2 * np.pi) ** 1.5 * eta)
    raise ValueError(kind)


def _what_scipy(kind, k, eps, lam=0.0, eta=None):
    """eq. Fourier-Symmetric for U - U^eps = U [erfc(r/eps) + erf(r/eps) xi(r)],
    xi(r) = erfc((r - 6 eps)/eps)/2, written independently with scipy."""
    d = O.KIND_DIM[kind]

    def f(r):
        rem = _u_scipy(kind, r, lam, eta) * (special.erfc(r / eps) + special.erf(r / eps)
                                            * 0.5 * special.erfc((r - 6 * eps) / eps))
        if d == 2:
            return 2 * np.pi * rem * special.j0(k * r) * r
        return 4 * np.pi * rem * np.sinc(k * r / np.pi) * r * r

    brk = [0.0, 1e-8, 1e-5, 1e-3, 0.03, 0.2] + list(np.arange(0.5, 13.0 * eps + 0.25, 0.25 * eps))
    brk = sorted(b for b in set(brk) if b <= 13.0 * eps)
    tot = 0.0
    for a, b in zip(brk[:-1], brk[1:]):
        v, _ = integrate.quad(f, a, b, epsabs=1e-19, epsrel=1e-13, limit=500)
        tot += v
    return tot


@pytest.mark.parametrize("kind,lam,eta", [("yukawa2d", 2.0, None), ("yukawa3d", 2.0, None),
                                          ("log2d", 0.0, None), ("biharmonic2d", 0.0, None),
                                          ("quasi2d_ddi", 0.0, 1 / np.sqrt(32))])
def test_windowed_w_against_independent_quadrature(kind, lam, eta):
    assert O.windowed(kind)
    eps = 1.0
    ks = np.array([0.0, 0.3, 1.0, 2.5, 6.0, 11.0])
    wq = O.what_general(kind, ks, eps, lam=lam, eta=eta)
    ws = np.array([_what_scipy(kind, k, eps, lam, eta) for k in ks])
    assert np.max(np.abs(wq - ws)) <= 1e-13 * np.max(np.abs(ws)), (wq, ws)


def test_window_limits():
    """U^eps vanishes at r = 0 to the window's 1e-17 and equals U erf(r/eps)
    beyond 12 eps (the window has decayed), which is all condition (b) of
    eq. ApproxProp needs when eps <= R0/12."""
    eps, lam = 0.8, 2.0
    assert O.ueps_general("yukawa2d", [0.0], eps, lam=lam)[0] == 0.0
    assert abs(O.ueps_general("yukawa3d", [0.0], eps, lam=lam)[0]) <= 2e-18
    r = np.linspace(12.0 * eps, 30.0, 50)
    u = O.u_any("yukawa2d", r, lam=lam) * special.erf(r / eps)
    assert np.allclose(O.ueps_general("yukawa2d", r, eps, lam=lam), u, rtol=1e-16, atol=0)
    # smooth transition in between: no point where U^eps exceeds U
    r = np.linspace(1e-3, 12.0 * eps, 500)
    assert np.all(np.abs(O.ueps_general("yukawa2d", r, eps, lam=lam))
                  <= np.abs(O.u_any("yukawa2d", r, lam=lam)) * (1 + 1e-15))


# ---------------------------------------------------------------------------
# Printed Table 5 rows
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("key,d", [("yukawa2d_iso", 2), ("yukawa3d_iso", 3)])
def test_printed_yukawa_rows(golden, key, d):
    """With lambda = 2 the general construction reproduces the h = 2, 1, 1/2
    entries of both Yukawa rows to all printed digits."""
    g = golden[key]
    for c in range(3):
        N = int(round(2 * g["L"] / g["h"][c]))
        X, r, rho = iso_grid(d, g["L"], N, g["sigma2"])
        phi = O.solve("yukawa2d" if d == 2 else "yukawa3d", [g["L"]] * d, [N] * d, rho,
                      eps=g["eps"], lam=2.0, general=True)
        err = R.rel_max_err(phi, yukawa_exact(d, X, g["sigma2"], 2.0))
        assert abs(err - g["err"][c]) <= 2e-4 * g["err"][c], (key, c, err)


def test_printed_yukawa2d_finest_entry(golden):
    """h = 1/4 (printed 5.2e-16): round-off of the FP64 FFT convolution."""
    g = golden["yukawa2d_iso"]
    N = int(round(2 * g["L"] / g["h"][3]))
    X, r, rho = iso_grid(2, g["L"], N, g["sigma2"])
    phi = O.solve("yukawa2d", [g["L"]] * 2, [N] * 2, rho, eps=g["eps"], lam=2.0)
    assert R.rel_max_err(phi, yukawa_exact(2, X, g["sigma2"], 2.0)) <= 1e-13


def test_printed_quasi2d_row(golden):
    g = golden["quasi2d_ddi_iso"]
    s = np.sqrt(g["sigma2"])
    N = int(round(2 * g["L"] / g["h"][2]))
    X, r, rho = iso_grid(2, g["L"], N, g["sigma2"])
    phi = O.solve_q2d([g["L"]] * 2, [N] * 2, rho, g["eps"], g["eta"], g["n"])
    err = R.rel_max_err(phi, R.quasi2d_ddi_iso(X, 1.0, s, g["eta"], g["n"]))
    assert abs(err - g["err"][2]) <= 1e-4 * g["err"][2], err


@pytest.mark.parametrize("n", [[0.0, 0.0, 1.0], [0.3, 0.5, np.sqrt(0.66)]])
def test_quasi2d_exact_when_resolved(n):
    """Every dipole orientation at h = 1/4 (a smaller box than Table 5's, so
    the test stays short): the spectral derivative, the kernel's window
    construction and the convolution together reach round-off."""
    L, N, sigma2, eta = 8.0, 64, 1.2, 1 / np.sqrt(32)
    X, r, rho = iso_grid(2, L, N, sigma2)
    phi = O.solve_q2d([L] * 2, [N] * 2, rho, 1.0, eta, n)
    assert R.rel_max_err(phi, R.quasi2d_ddi_iso(X, 1.0, np.sqrt(sigma2), eta, n)) <= 1e-13


# ---------------------------------------------------------------------------
# Invariants of the construction
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,lam,eta", [("yukawa2d", 1.5, None), ("log2d", 0.0, None),
                                          ("biharmonic2d", 0.0, None),
                                          ("quasi2d_ddi", 0.0, 0.3)])
def test_general_eps_independence(kind, lam, eta):
    """Theorem 1 for the general construction: two admissible eps (both
    <= R0/12) give the same potential once the grid resolves U^eps."""
    L, N = 8.0, 64
    X, r, rho = iso_grid(2, L, N, 2.0)
    a = O.solve(kind, [L] * 2, [N] * 2, rho, eps=1.0, lam=lam, general=True, eta=eta)
    b = O.solve(kind, [L] * 2, [N] * 2, rho, eps=1.3, lam=lam, general=True, eta=eta)
    assert R.rel_l2_err(a, b) <= 1e-13


def test_general_eps_independence_detects_a_planted_w_error():
    """The pin above is sensitive: W scaled by 1.001 (planted in T(2), on the
    CPU) moves the two eps results apart far above 1e-13."""
    L, N = [8.0] * 2, [32] * 2
    X, r, rho = iso_grid(2, 8.0, 32, 2.0)
    out = []
    for eps in (1.0, 1.3):
        _, t1, t2, _ = O.build_tensor("yukawa2d", L, N, eps, lam=1.5, parts=True)
        out.append(O.conv_fft(t1 + 1.001 * t2, rho))
    assert R.rel_l2_err(out[0], out[1]) > 1e-7


@pytest.mark.parametrize("kind,lam", [("log2d", 0.0), ("yukawa3d", 1.0), ("biharmonic2d", 0.0)])
def test_general_and_closed_routes_agree(kind, lam):
    """Two admissible far-field approximations of one kernel converge to the
    same discretisation once resolved."""
    d = O.KIND_DIM[kind]
    n = 48 if d == 3 else 64
    X, r, rho = iso_grid(d, 8.0, n, 2.0)
    a = O.solve(kind, [8.0] * d, [n] * d, rho, eps=1.0, lam=lam)
    b = O.solve(kind, [8.0] * d, [n] * d, rho, eps=1.0, lam=lam, general=True)
    assert R.rel_l2_err(a, b) <= 1e-13


def test_general_route_identical_tensor_without_window():
    """Coulomb: the general route only swaps the closed-form W for its
    quadrature, so the tensors agree to round-off on a coarse grid too."""
    L, N = [8.0] * 3, [16] * 3
    a = O.build_tensor("coulomb3d", L, N, 1.0)
    b = O.build_tensor("coulomb3d", L, N, 1.0, general=True)
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(a))
