"""The general construction on the GPU (Sec. 4, eq. GeneralApprox1; W by
quadrature of eq. Fourier-Symmetric) against the FP64 CPU oracle, and the
kernels that need it: 2D Yukawa and the quasi-2D dipole-dipole interaction
(Sec. 5.3).  Needs an MI355X.

Tolerances as everywhere (relative L2 and relative max over the grid against
the oracle on the same input values): 1e-12 in FP64, 5e-6 in FP32.  At full sizes, where the
oracle's quadrature tensor is out of reach, the GPU result is checked against
exact potentials of Gaussian densities at sampled points and against the
closed-form route (properties that hold at any size).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import reference as R
from paper_2504_19410_amd import synth
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19410_amd import fsa
    return fsa


def density(L, N, seed):
    rng = synth.SplitMix64(seed)
    gs = synth.draw_gaussians(rng, len(N), 3, [-l / 4 for l in L], [l / 4 for l in L],
                              [l / 5 for l in L], [l / 3 for l in L], isotropic=False)
    return synth.eval_gaussians(gs, L, N)


def to_dev(F, a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(F.DTYPES[prec]).cuda()


GENERAL = [
    # kind, L, N, lam, eps (None: the plan's default)
    ("yukawa2d", (12.0, 12.0), (96, 96), 2.0, 1.0),     # Table 5's box at h = 1/4
    ("yukawa2d", (6.0, 9.0), (48, 128), 0.7, None),     # anisotropic, default eps
    ("yukawa2d", (4.0, 4.0), (24, 16), 3.0, None),
    ("yukawa3d", (8.0, 8.0, 8.0), (16, 24, 32), 2.0, None),
    ("coulomb3d", (3.0, 5.0, 4.0), (24, 16, 48), None, None),
    ("biharmonic3d", (4.0, 4.0, 4.0), (16, 16, 16), None, None),
    ("log2d", (8.0, 6.0), (48, 96), None, None),
    ("coulomb2d", (6.0, 6.0), (24, 32), None, None),
    ("biharmonic2d", (5.0, 7.0), (32, 48), None, None),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,L,N,lam,eps", GENERAL)
def test_parity_general(F, kind, L, N, lam, eps, prec):
    rho64 = density(L, N, seed=sum(N) + 3)
    plan = F.Plan(kind, L, N, prec, eps=eps, lam=lam, general=True).build()
    rho = to_dev(F, rho64, prec)
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    ref = O.solve(kind, L, N, rho.double().cpu().numpy(), eps=plan.eps, lam=lam or 0.0,
                  general=True)
    check(phi.double().cpu().numpy(), ref, prec, f"general {kind} {N} {prec} eps={plan.eps:.4g}")


@pytest.mark.parametrize("kind,L,N,lam", [("yukawa2d", (6.0, 9.0), (48, 64), 0.7),
                                           ("yukawa3d", (4.0, 4.0, 4.0), (16, 16, 16), 2.0),
                                           ("coulomb2d", (3.0, 4.0), (16, 24), None)])
def test_general_tensor_matches_oracle_dft(F, kind, L, N, lam):
    """The GPU spectral octant (Chebyshev-interpolated quadrature W) equals
    DFT(T(1) + T(2)) / prod P of the oracle (W by adaptive quadrature at each
    lattice |k|)."""
    plan = F.Plan(kind, L, N, "f64", lam=lam, general=True).build()
    got = plan.tensor().numpy()
    T = O.build_tensor(kind, L, N, plan.eps, lam=lam or 0.0, general=True)
    That = O.fftnd(T, -1) / T.size
    octant = That.real[tuple(slice(0, n + 1) for n in N)]
    ref = np.transpose(octant, tuple(reversed(range(len(N)))))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


Q2D_ETA = 1 / np.sqrt(32)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L,N,n,eta,eps", [
    ((12.0, 12.0), (96, 96), (0.0, 0.0, 1.0), Q2D_ETA, 1.0),      # Table 5's setup, h = 1/4
    ((6.0, 8.0), (64, 48), (0.3, 0.5, np.sqrt(0.66)), 0.3, None),
    ((4.0, 4.0), (32, 24), (0.8, -0.6, 0.0), 0.25, None),           # in-plane dipoles
])
def test_parity_quasi2d_ddi(F, L, N, n, eta, eps, prec):
    """Quasi-2D DDI: three derivative launches for the source, then the 2D
    convolution with the quasi-2D kernel in the general construction."""
    rho64 = density(L, N, seed=sum(N) + 5)
    plan = F.Plan("quasi2d_ddi", L, N, prec, eps=eps, n=n, eta=eta).build()
    assert plan.launches() == ["spectral"] * 3 + ["r2c", "conv", "c2r"]
    rho = to_dev(F, rho64, prec)
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    ref = O.solve_q2d(L, N, rho.double().cpu().numpy(), plan.eps, eta, n)
    check(phi.double().cpu().numpy(), ref, prec, f"quasi2d {N} {prec}")
    rho2 = rho.clone()
    plan.apply(rho2, out=rho2)
    torch.cuda.synchronize()
    assert torch.equal(rho2, phi)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_parity_ddi3d_general(F, prec):
    """The 3D DDI's Coulomb convolution with the quadrature W."""
    L, N = (6.0, 6.0, 3.0), (32, 48, 16)
    n, m = (0.82778, 0.41505, -0.37751), (0.3118, 0.9378, -0.15214)
    rho64 = density(L, N, seed=91)
    plan = F.Plan("ddi3d", L, N, prec, n=n, m=m, general=True).build()
    rho = to_dev(F, rho64, prec)
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    ref = O.solve_ddi(L, N, rho.double().cpu().numpy(), plan.eps, n, m, general=True)
    check(phi.double().cpu().numpy(), ref, prec, f"ddi3d general {N} {prec}")


def test_quasi2d_not_batched_or_served(F):
    plan = F.Plan("quasi2d_ddi", (8.0, 8.0), (16, 16), "f32", n=(0, 0, 1), eta=0.3).build()
    r = torch.zeros(16, 16, device="cuda")
    with pytest.raises(F.FsaError, match="EUNSUPPORTED"):
        F.apply_batched([plan], [r])
    srv = F.Server(1 << 30)
    try:
        import ctypes
        k = F._kernel("quasi2d_ddi", None, None, (0, 0, 1), None, 0.3)
        t = ctypes.c_uint64()
        Ls = (ctypes.c_double * 2)(8.0, 8.0)
        Ns = (ctypes.c_int64 * 2)(16, 16)
        st = F.lib().fsa_server_submit(srv._h, ctypes.byref(k), 2, Ls, Ns, 0,
                                       ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(r.data_ptr()), ctypes.byref(t))
        assert F.STATUS[st] == "FSA_EUNSUPPORTED"
    finally:
        srv.close()


def test_general_plans_batch_and_serve(F):
    """General-construction plans go through the batched graph (bitwise equal
    to their single evaluations) and the server (tensor cached per key,
    including the construction)."""
    specs = [("yukawa2d", (6.0, 6.0), (64, 32), 1.5), ("log2d", (5.0, 4.0), (32, 48), None)]
    plans, rhos, singles = [], [], []
    for i, (kind, L, N, lam) in enumerate(specs):
        p = F.Plan(kind, L, N, "f32", lam=lam, general=True).build()
        r = to_dev(F, density(L, N, seed=40 + i), "f32")
        plans.append(p)
        rhos.append(r)
        singles.append(p.apply(r))
    outs = F.apply_batched(plans, rhos)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)
    srv = F.Server(1 << 30)
    try:
        kind, L, N, lam = specs[0]
        phi = torch.empty_like(rhos[0])
        t = srv.submit(kind, L, N, rhos[0], phi, lam=lam, general=True)
        srv.wait(t)
        assert torch.equal(phi, singles[0])
        # the closed-form log kernel and its general construction are cached
        # apart (two tensor builds), each reused by a repeat
        kind, L, N, _ = specs[1]
        phi_c = torch.empty_like(rhos[1])
        phi_g = torch.empty_like(rhos[1])
        misses = srv.stats()["cache_misses"]
        srv.wait(srv.submit(kind, L, N, rhos[1], phi_c))
        srv.wait(srv.submit(kind, L, N, rhos[1], phi_g, general=True))
        assert srv.stats()["cache_misses"] == misses + 2
        srv.wait(srv.submit(kind, L, N, rhos[1], phi_g, general=True))
        srv.wait(srv.submit(kind, L, N, rhos[1], phi_c))
        assert srv.stats()["cache_misses"] == misses + 2
        assert torch.equal(phi_g, singles[1])
    finally:
        srv.close()


def test_rejects_invalid_general_plans(F):
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.Plan("yukawa2d", (8.0, 8.0), (32, 32), lam=0.0)          # needs lambda > 0
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.Plan("quasi2d_ddi", (8.0, 8.0), (32, 32), n=(0, 0, 1))   # needs eta > 0
    with pytest.raises(F.FsaError, match="EINVAL"):
        F.Plan("quasi2d_ddi", (8.0, 8.0), (32, 32), n=(0, 0, 0), eta=0.3)
    with pytest.raises(F.FsaError, match="EINVAL"):                # window needs eps <= R0/12
        F.Plan("yukawa2d", (8.0, 8.0), (32, 32), lam=1.0, eps=1.5)
    p = F.Plan("yukawa2d", (8.0, 8.0), (32, 32), lam=1.0)
    assert abs(p.eps - 16.0 / 16.0) < 1e-15                        # default R0/16


# ---------------------------------------------------------------------------
# Full sizes: exact potentials at sampled points, and the closed-form route
# ---------------------------------------------------------------------------

def _sample_idx(shape, n, seed):
    rng = np.random.default_rng(seed)
    size = int(np.prod(shape))
    return np.unique(np.concatenate([rng.choice(size, n, replace=False), [0, size - 1]]))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 5e-6)])
def test_yukawa2d_largest_grid_against_exact(F, prec, tol):
    """2048 x 2048 (the largest grid) on [-12, 12]^2, three Gaussians: the
    GPU potential against the exact one (1-D heat-kernel integral) at sampled
    points, relative to the potential's maximum."""
    L, N, lam = (12.0, 12.0), (2048, 2048), 2.0
    gs = [(1.0, [0.5, -1.0], [1.2, 0.9]), (0.7, [-2.0, 1.5], [0.8, 1.4]),
          (-0.4, [1.0, 2.5], [1.0, 1.0])]
    axes = O.grid_axes(L, N)
    X = np.meshgrid(*axes, indexing="ij")
    rho64 = sum(a * np.exp(-((X[0] - c[0]) / s[0]) ** 2 - ((X[1] - c[1]) / s[1]) ** 2)
                for a, c, s in gs)
    plan = F.Plan("yukawa2d", L, N, prec, lam=lam).build()
    phi = plan.apply(to_dev(F, rho64, prec))
    torch.cuda.synchronize()
    phi = phi.double().cpu().numpy()
    idx = _sample_idx(N, 48, 1)
    idx = np.append(idx, int(np.argmax(np.abs(phi))))
    ex = R.gaussian_sum_potential("yukawa2d", gs, L, N, lam=lam, points=idx)
    err = float(np.max(np.abs(phi.ravel()[idx] - ex)) / np.max(np.abs(ex)))
    print(f"yukawa2d 2048^2 {prec}: sampled rel max err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 5e-6)])
def test_yukawa3d_256_general_against_closed_route(F, prec, tol):
    """256^3 on [-8, 8]^3, eps = 1: the general construction (window +
    quadrature W) and the closed-form Gaussian-screened split are two
    discretisations of one potential; resolved, both reach the exact one."""
    L, N, lam = (8.0,) * 3, (256,) * 3, 2.0
    rho64 = density(L, N, seed=256)
    rho = to_dev(F, rho64, prec)
    a = F.Plan("yukawa3d", L, N, prec, lam=lam, eps=1.0, general=True).build().apply(rho)
    b = F.Plan("yukawa3d", L, N, prec, lam=lam, eps=1.0).build().apply(rho)
    torch.cuda.synchronize()
    err = float((a.double() - b.double()).norm() / b.double().norm())
    print(f"yukawa3d 256^3 {prec}: general vs closed rel L2 {err:.3e}")
    assert err <= tol
