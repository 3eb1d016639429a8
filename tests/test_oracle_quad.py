"""The quadruple-precision oracle of the extended-precision mode
(`oracle/fsa_oracle_q.c`, Coulomb kernels) against what fixes it (no GPU):
its FFT against the DFT definition evaluated with mpmath, the printed quad row
of Table 2, the 2D Coulomb row, and agreement with the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import reference as R
from paper_2504_19410_amd import synth


def test_quad_fft_matches_dft_definition():
    import mpmath as mp
    rng = np.random.default_rng(5)
    for n, sign in ((8, -1), (12, -1), (16, +1)):
        x = np.empty((n, 4))
        x[:, 0] = rng.standard_normal(n)
        x[:, 2] = rng.standard_normal(n)
        x[:, 1] = x[:, 0] * 1e-17 * rng.standard_normal(n)
        x[:, 3] = x[:, 2] * 1e-17 * rng.standard_normal(n)
        got = O.fft1d_quad(x, sign)
        with mp.workdps(45):
            xs = [mp.mpc(mp.mpf(a) + mp.mpf(b), mp.mpf(c) + mp.mpf(e)) for a, b, c, e in x]
            worst = 0
            scale = max(abs(v) for v in xs) * n
            for k in range(n):
                ref = sum(xs[j] * mp.expj(sign * 2 * mp.pi * j * k / n) for j in range(n))
                g = mp.mpc(mp.mpf(got[k, 0]) + mp.mpf(got[k, 1]), mp.mpf(got[k, 2]) + mp.mpf(got[k, 3]))
                worst = max(worst, float(abs(g - ref) / scale))
        assert worst <= 1e-32, (n, worst)


@pytest.mark.parametrize("c", [0, 1, 2])
def test_printed_quad_row(golden, c):
    """Table 2's 3D quad row at h = 1, 1/2, 1/4 (the last, 4.8161e-18, only
    appears in quadruple precision: the double row stops at 5.6e-16)."""
    g = golden["coulomb3d_iso_quad"]
    N = int(round(2 * g["L"] / g["h"][c]))
    L = [g["L"]] * 3
    rho = synth.gaussian_dd(L, [N] * 3, g["sigma2"])
    phi = O.solve_quad("coulomb3d", L, [N] * 3, rho, g["eps"])
    err = R.dd_rel_max_err(phi, R.coulomb3d_iso_dd(L, [N] * 3, g["sigma2"]))
    assert abs(err - g["err"][c]) <= 1e-3 * g["err"][c], (c, err)


def test_quad_2d_coulomb_row(golden):
    """The 2D Coulomb row of Table 2 (h = 1, 1/2 with R10's exponent reading)
    in quad, and the resolved h = 1/8 grid at quad round-off."""
    g = golden["coulomb2d_iso"]
    L = [g["L"]] * 2
    for h, printed in ((1.0, g["err"][0]), (0.5, 2.9648e-06)):
        N = int(round(2 * g["L"] / h))
        rho = synth.gaussian_dd(L, [N] * 2, g["sigma2"])
        phi = O.solve_quad("coulomb2d", L, [N] * 2, rho, g["eps"])
        err = R.dd_rel_max_err(phi, R.coulomb2d_iso_dd(L, [N] * 2, g["sigma2"]))
        assert abs(err - printed) <= 1e-3 * printed, (h, err)
    N = int(round(2 * g["L"] / 0.125))
    rho = synth.gaussian_dd(L, [N] * 2, g["sigma2"])
    phi = O.solve_quad("coulomb2d", L, [N] * 2, rho, g["eps"])
    assert R.dd_rel_max_err(phi, R.coulomb2d_iso_dd(L, [N] * 2, g["sigma2"])) <= 1e-31


@pytest.mark.parametrize("kind,L,N", [("coulomb3d", (3.0, 5.0, 4.0), (8, 16, 8)),
                                      ("coulomb2d", (8.0, 6.0), (32, 16))])
def test_quad_agrees_with_fp64_oracle(kind, L, N):
    """Same discretisation: the quad result rounded to double equals the FP64
    oracle's to FP64 rounding."""
    rng = np.random.default_rng(3)
    rho = np.zeros(tuple(N) + (2,))
    rho[..., 0] = rng.standard_normal(N)
    q = O.solve_quad(kind, L, N, rho, 1.0)
    f = O.solve(kind, L, N, rho[..., 0], eps=1.0)
    assert np.linalg.norm(q[..., 0] - f) <= 1e-14 * np.linalg.norm(f)


def test_gaussian_dd_density():
    """The double-double density carries exp(-r^2/sigma^2) with sigma^2 the
    decimal 0.8, not the nearest double."""
    import mpmath as mp
    L, N = [8.0] * 2, [16, 16]
    rho = synth.gaussian_dd(L, N, 0.8)
    X = np.meshgrid(*O.grid_axes(L, N), indexing="ij")
    with mp.workdps(40):
        for i, j in ((3, 5), (8, 8), (0, 15)):
            r2 = mp.mpf(float(X[0][i, j])) ** 2 + mp.mpf(float(X[1][i, j])) ** 2
            ref = mp.exp(-r2 / mp.mpf("0.8"))
            got = mp.mpf(rho[i, j, 0]) + mp.mpf(rho[i, j, 1])
            assert abs(got - ref) <= 1e-31 * ref
