"""Exact potentials of Gaussian densities (test infrastructure only).

These are the analytic references the paper measures its error against
(Sec. 5: "the potential can be computed analytically"); the paper does not
print them, so they are derived here from the heat-kernel representation of
each kernel and checked in the tests against brute-force quadrature.

For rho(x) = a exp(-sum_j (x_j - c_j)^2 / s_j^2), y = x - c and

    G(t) = prod_j s_j (s_j^2 + 4t)^{-1/2} exp(-y_j^2 / (s_j^2 + 4t)),

* 3D Coulomb 1/(4 pi r):     Phi = a int_0^inf G(t) dt
* 3D Yukawa e^{-lam r}/(4 pi r): Phi = a int_0^inf e^{-lam^2 t} G(t) dt
* 2D Yukawa K0(lam r)/(2 pi):    the same integral with the 2D G(t)
* 2D log -(1/2pi) ln r:      Phi = a int_0^inf [G(t) - s_0 s_1 e^{-1/(4t)}/(4t)] dt
* 2D Coulomb 1/(2 pi r):     Phi = a/sqrt(pi) int_0^inf t^{-1/2} G(t) dt

Isotropic closed forms (s_j = s, r = |y|):
* Coulomb 3D: a sqrt(pi) s^3 erf(r/s) / (4 r), Phi(0) = a s^2 / 2
* log 2D:     -(a s^2/4) [ln r^2 + E1(r^2/s^2)], Phi(0) = -(a s^2/4)(2 ln s - gamma)
* Yukawa 3D:  a pi^{3/2} s^3 e^{lam^2 s^2/4} / (8 pi r)
                 [e^{-lam r} erfc(lam s/2 - r/s) - e^{lam r} erfc(lam s/2 + r/s)]

Case II densities rho = -Laplace(Phi0) (Sec. 5, Example 1 and Example 3) have
Phi = Phi0 exactly for the 3D Coulomb and 2D log kernels.
"""
from __future__ import annotations

import numpy as np
from scipy import special

EULER_GAMMA = 0.57721566490153286060651209008240243


def _grid(L, N):
    return np.meshgrid(*[(-float(l) + np.arange(int(n)) * (2.0 * float(l) / int(n)))
                         for l, n in zip(L, N)], indexing="ij")


# --------------------------------------------------------------------------- #
# Isotropic closed forms                                                      #
# --------------------------------------------------------------------------- #

def coulomb3d_iso(r, a, s):
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-8 * s
    rr = np.where(small, 1.0, r)
    out[...] = a * np.sqrt(np.pi) * s ** 3 * special.erf(rr / s) / (4.0 * rr)
    out[small] = a * s * s / 2.0
    return out


def log2d_iso(r, a, s):
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r == 0.0
    rr = np.where(small, 1.0, r)
    out[...] = -(a * s * s / 4.0) * (np.log(rr * rr) + special.exp1(rr * rr / (s * s)))
    out[small] = -(a * s * s / 4.0) * (2.0 * np.log(s) - EULER_GAMMA)
    return out


def yukawa3d_iso(r, a, s, lam):
    """Closed form; the two erfc terms are written with erfcx to avoid overflow."""
    r = np.asarray(r, dtype=np.float64)
    b = lam * s / 2.0
    pref = a * np.pi ** 1.5 * s ** 3 / (8.0 * np.pi)
    out = np.empty_like(r)
    small = r < 1e-6 * s
    rr = np.where(small, 1.0, r)
    u1 = b - rr / s
    u2 = b + rr / s
    # e^{b^2} e^{-lam r} erfc(u1) = e^{-r^2/s^2} erfcx(u1)  (b^2 - lam r = u1^2 - r^2/s^2)
    # e^{b^2} e^{+lam r} erfc(u2) = e^{-r^2/s^2} erfcx(u2)  (b^2 + lam r = u2^2 - r^2/s^2)
    g = np.exp(-(rr / s) ** 2)
    t1 = np.where(u1 >= 0,
                  g * special.erfcx(np.maximum(u1, 0.0)),
                  np.exp(b * b - lam * rr) * special.erfc(u1))
    t2 = g * special.erfcx(u2)
    out[...] = pref * (t1 - t2) / rr
    # r -> 0: d/dr of the bracket at 0 -> Phi(0) = pref * 2 [ (2/(s sqrt(pi))) - b e^{b^2} erfc(b) * (2/s) / 2 ... ]
    if np.any(small):
        # derivative of e^{b^2}[e^{-lam r} erfc(b - r/s) - e^{lam r} erfc(b + r/s)] at r = 0
        d = 2.0 * (-lam * special.erfcx(b) + 2.0 / (s * np.sqrt(np.pi)))
        out[small] = pref * d
    return out


# --------------------------------------------------------------------------- #
# 1-D heat-kernel integrals for anisotropic Gaussians                         #
# --------------------------------------------------------------------------- #

def _gauss_legendre(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def heat_integral(kind, y, s, lam=0.0, n_nodes=400, panels=8):
    """int_0^inf of the kernel's heat-kernel integrand for one Gaussian.

    ``y`` has shape (d, M) (offsets from the centre), ``s`` shape (d,).  The
    substitution t = (s*^2/4)(u^-2 - 1), u in (0, 1], s* = min s_j, maps the
    half line to the unit interval; composite Gauss-Legendre on ``panels``
    geometric panels in u resolves the u -> 0 end.
    """
    y = np.asarray(y, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    d = s.size
    sstar = float(np.min(s))
    # panels in u: [u_k, u_{k+1}] with geometric spacing towards 0
    edges = np.concatenate([[0.0], np.geomspace(1e-6, 1.0, panels)])
    xg, wg = _gauss_legendre(n_nodes)
    us = []
    ws = []
    for a0, a1 in zip(edges[:-1], edges[1:]):
        us.append(a0 + (a1 - a0) * xg)
        ws.append((a1 - a0) * wg)
    u = np.concatenate(us)
    wu = np.concatenate(ws)
    if kind == "coulomb2d":
        # t^{-1/2} is singular at t = 0: integrate in v = sqrt(t) instead,
        # v = (s*/2)(1/u - 1), so that int t^{-1/2} G dt = int 2 G(v^2) dv.
        v = 0.5 * sstar * (1.0 / u - 1.0)
        t = v * v
        dt_du = 0.5 * sstar / (u * u)
    else:
        t = 0.25 * sstar * sstar * (u ** -2 - 1.0)
        dt_du = 0.5 * sstar * sstar * u ** -3
    total = np.zeros(y.shape[1])
    chunk = max(1, 4_000_000 // max(1, u.size))
    for c0 in range(0, y.shape[1], chunk):
        yy = y[:, c0:c0 + chunk]
        g = np.ones((u.size, yy.shape[1]))
        for j in range(d):
            q = s[j] * s[j] + 4.0 * t
            g *= (s[j] / np.sqrt(q))[:, None] * np.exp(-(yy[j][None, :] ** 2) / q[:, None])
        if kind == "coulomb3d":
            f = g
        elif kind in ("yukawa3d", "yukawa2d"):
            f = g * np.exp(-lam * lam * t)[:, None]
        elif kind == "log2d":
            f = g - (np.prod(s) * np.exp(-0.25 / t) / (4.0 * t))[:, None]
        elif kind == "coulomb2d":
            f = g * (2.0 / np.sqrt(np.pi))
        else:
            raise ValueError(kind)
        total[c0:c0 + chunk] = np.einsum("u,um->m", wu * dt_du, f)
    return total


def gaussian_sum_potential(kind, gaussians, L, N, lam=0.0, points=None, iso_closed_form=True):
    """Exact potential of sum_i a_i exp(-sum_j (x_j - c_ij)^2 / s_ij^2) on the grid.

    ``gaussians`` is a list of (a, c[d], s[d]).  ``points`` optionally selects
    flat grid indices.  Isotropic Gaussians use the closed form where one
    exists; the rest use the 1-D integral.
    """
    X = _grid(L, N)
    d = len(X)
    if points is None:
        coords = np.stack([x.ravel() for x in X])
    else:
        idx = np.asarray(points, dtype=np.int64)
        coords = np.stack([x.ravel()[idx] for x in X])
    out = np.zeros(coords.shape[1])
    for a, c, s in gaussians:
        c = np.asarray(c, dtype=np.float64).reshape(d, 1)
        s = np.asarray(s, dtype=np.float64).reshape(d)
        y = coords - c
        iso = bool(np.all(s == s[0]))
        if iso and iso_closed_form and kind in ("coulomb3d", "log2d", "yukawa3d"):
            r = np.sqrt(np.sum(y * y, axis=0))
            if kind == "coulomb3d":
                out += coulomb3d_iso(r, a, s[0])
            elif kind == "log2d":
                out += log2d_iso(r, a, s[0])
            else:
                out += yukawa3d_iso(r, a, s[0], lam)
        else:
            out += a * heat_integral(kind, y, s, lam=lam)
    if points is None:
        return out.reshape(tuple(int(n) for n in N))
    return out


def case2_phi0(L, N, sigma, gammas, x0=None):
    """Phi0(x) = exp(-sum_j x_j^2/(gamma_j^2 sigma^2)) (+ shifted copy at x0)."""
    X = _grid(L, N)
    g = np.asarray(gammas, dtype=np.float64)

    def one(shift):
        e = np.zeros_like(X[0])
        for j, x in enumerate(X):
            e += (x - shift[j]) ** 2 / (g[j] ** 2 * sigma ** 2)
        return np.exp(-e)

    phi = one(np.zeros(len(X)))
    if x0 is not None:
        phi = phi + one(np.asarray(x0, dtype=np.float64))
    return phi


def rel_max_err(phi_num, phi_exact):
    """The paper's error norm: max|Phi - Phi_h| / max|Phi| on the grid (Sec. 5)."""
    return float(np.max(np.abs(phi_num - phi_exact)) / np.max(np.abs(phi_exact)))


def rel_l2_err(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def ddi3d_iso(X, a, s, n, m):
    """3D dipole-dipole potential of a * exp(-|x|^2/s^2), exactly:
    -(m.n) rho - 3 d_nm Phi_C with Phi_C = a sqrt(pi) s^3 erf(r/s)/(4 r) the
    Coulomb potential (Sec. 5.3); the Hessian of a radial f is
    f'' xh xh^T + f'/r (I - xh xh^T), and at r = 0 it is f''(0) I, f''(0) = -a/3."""
    n = np.asarray(n, dtype=float)
    m = np.asarray(m, dtype=float)
    r = np.sqrt(sum(x * x for x in X))
    z = r == 0.0
    rr = np.where(z, 1.0, r)
    g = np.exp(-rr * rr / (s * s))
    ef = special.erf(rr / s)
    c = a * np.sqrt(np.pi) * s ** 3 / 4.0
    two = 2.0 / (np.sqrt(np.pi) * s)
    fp = c * (two * g / rr - ef / rr ** 2)
    fpp = c * (-2.0 * two * g / (s * s) - 2.0 * two * g / rr ** 2 + 2.0 * ef / rr ** 3)
    xn = sum(X[i] * n[i] for i in range(3)) / rr
    xm = sum(X[i] * m[i] for i in range(3)) / rr
    nm = float(n @ m)
    hess = fpp * xn * xm + fp / rr * (nm - xn * xm)
    hess = np.where(z, -a * nm / 3.0, hess)
    rho = a * np.exp(-r * r / (s * s))
    return -nm * rho - 3.0 * hess


def quasi2d_ddi_iso(X, a, s, eta, n, panels=60, n_nodes=24):
    """Quasi-2D dipole-dipole potential of a * exp(-|x|^2/s^2) (Sec. 5.3):
    Phi = -(3/2) (d_{n_perp n_perp} - n_3^2 Lap) F with F = U~ conv rho.

    U~ has the 2D transform erfcx(k eta / sqrt 2) / k (its s-integral done in
    closed form), so the radial F and its derivatives are Hankel integrals
      F   =  (a s^2/2) int g(k) J0(kr) dk,
      F'  = -(a s^2/2) int g(k) k J1(kr) dk,
      F'' =  (a s^2/2) int g(k) k^2 (J1(kr)/(kr) - J0(kr)) dk,
    g(k) = erfcx(k eta/sqrt 2) e^{-k^2 s^2/4}, by composite Gauss-Legendre on
    [0, K], e^{-K^2 s^2/4} = e^{-46}.  The Hessian of a radial F is
    F'' xh xh^T + F'/r (I - xh xh^T), and F''(0) I at r = 0."""
    n = np.asarray(n, dtype=float)
    x0, x1 = np.asarray(X[0], dtype=float), np.asarray(X[1], dtype=float)
    r = np.sqrt(x0 * x0 + x1 * x1)
    K = 2.0 * np.sqrt(46.0) / s
    xg, wg = _gauss_legendre(n_nodes)
    edges = np.linspace(0.0, K, panels + 1)
    k = np.concatenate([a0 + (a1 - a0) * xg for a0, a1 in zip(edges[:-1], edges[1:])])
    wk = np.concatenate([(a1 - a0) * wg for a0, a1 in zip(edges[:-1], edges[1:])])
    g = special.erfcx(k * eta / np.sqrt(2.0)) * np.exp(-k * k * s * s / 4.0) * wk
    c = a * s * s / 2.0
    rf = r.ravel()
    fp = np.empty_like(rf)
    fpp = np.empty_like(rf)
    for i0 in range(0, rf.size, 4096):
        rr = rf[i0:i0 + 4096]
        kr = np.outer(rr, k)
        j0 = special.j0(kr)
        j1 = special.j1(kr)
        with np.errstate(divide="ignore", invalid="ignore"):
            j1_over = np.where(kr > 0, j1 / np.where(kr > 0, kr, 1.0), 0.5)
        fp[i0:i0 + 4096] = -c * (j1 * k) @ g
        fpp[i0:i0 + 4096] = c * ((j1_over - j0) * k * k) @ g
    fp = fp.reshape(r.shape)
    fpp = fpp.reshape(r.shape)
    z = r == 0.0
    rr = np.where(z, 1.0, r)
    fp_over_r = np.where(z, fpp, fp / rr)
    xn = np.where(z, 0.0, (x0 * n[0] + x1 * n[1]) / rr)
    nperp2 = n[0] * n[0] + n[1] * n[1]
    d_nn = fpp * xn * xn + fp_over_r * (nperp2 - xn * xn)
    lap = fpp + fp_over_r
    return -1.5 * (d_nn - n[2] * n[2] * lap)


def coulomb3d_iso_dd(L, N, s2):
    """The closed-form 3D Coulomb potential of exp(-r^2/s^2) on the grid
    (a = 1), sqrt(pi) s^3 erf(r/s) / (4 r), as double-double pairs (shape
    N + (2,)), evaluated with mpmath at 40 digits once per distinct r^2;
    s^2 is the decimal its repr shows."""
    import mpmath as mp
    X = _grid(L, N)
    r2 = sum(x * x for x in X)
    u, inv = np.unique(r2.ravel(), return_inverse=True)
    hi = np.empty(u.size)
    lo = np.empty(u.size)
    with mp.workdps(40):
        s = mp.sqrt(mp.mpf(repr(float(s2))))
        for i, v in enumerate(u):
            if v == 0.0:
                e = s * s / 2
            else:
                r = mp.sqrt(mp.mpf(float(v)))
                e = mp.sqrt(mp.pi) * s ** 3 * mp.erf(r / s) / (4 * r)
            hi[i] = float(e)
            lo[i] = float(e - mp.mpf(hi[i]))
    out = np.empty(r2.shape + (2,))
    out[..., 0] = hi[inv].reshape(r2.shape)
    out[..., 1] = lo[inv].reshape(r2.shape)
    return out


def dd_rel_max_err(a, b):
    """max |a - b| / max |b| for double-double arrays (last axis (hi, lo)):
    the difference is formed pairwise, exact while a and b are close."""
    d = (a[..., 0] - b[..., 0]) + (a[..., 1] - b[..., 1])
    return float(np.max(np.abs(d)) / np.max(np.abs(b[..., 0])))


def dd_rel_l2_err(a, b):
    d = (a[..., 0] - b[..., 0]) + (a[..., 1] - b[..., 1])
    return float(np.linalg.norm(d.ravel()) / np.linalg.norm(b[..., 0].ravel()))


def coulomb2d_iso_dd(L, N, s2):
    """The closed-form 2D Coulomb (1/(2 pi r)) potential of exp(-r^2/s^2)
    (a = 1): (sqrt(pi) s / 2) e^{-r^2/(2 s^2)} I0(r^2/(2 s^2)), from the
    Hankel integral (s^2/2) int_0^inf e^{-k^2 s^2/4} J0(k r) dk; double-double
    pairs as coulomb3d_iso_dd."""
    import mpmath as mp
    X = _grid(L, N)
    r2 = sum(x * x for x in X)
    u, inv = np.unique(r2.ravel(), return_inverse=True)
    hi = np.empty(u.size)
    lo = np.empty(u.size)
    with mp.workdps(40):
        ss = mp.mpf(repr(float(s2)))
        s = mp.sqrt(ss)
        for i, v in enumerate(u):
            z = mp.mpf(float(v)) / (2 * ss)
            e = mp.sqrt(mp.pi) * s / 2 * mp.exp(-z) * mp.besseli(0, z)
            hi[i] = float(e)
            lo[i] = float(e - mp.mpf(hi[i]))
    out = np.empty(r2.shape + (2,))
    out[..., 0] = hi[inv].reshape(r2.shape)
    out[..., 1] = lo[inv].reshape(r2.shape)
    return out
