"""Parity of the HIP path with the FP64 CPU oracle (needs an MI355X).

Tolerances (relative L2 and relative max over the points compared, against
the oracle on the same input values): 1e-12 in FP64 mode, 5e-6 in FP32 mode.
Every call goes through the C ABI of include/fsa.h via the ctypes binding.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import reference as R
from paper_2504_19410_amd import synth
from parity import check, sample_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19410_amd import fsa
    return fsa


def density(kind, L, N, seed, noise=False):
    rng = synth.SplitMix64(seed)
    d = len(N)
    gs = synth.draw_gaussians(rng, d, 3, [-l / 4 for l in L], [l / 4 for l in L],
                              [l / 5 for l in L], [l / 3 for l in L], isotropic=False)
    rho = synth.eval_gaussians(gs, L, N)
    if noise:
        rho = rho + 0.1 * np.random.default_rng(seed).standard_normal(rho.shape)
    return rho


def run_gpu(F, kind, L, N, prec, rho64, eps=None, lam=None):
    plan = F.Plan(kind, L, N, prec, eps=eps, lam=lam).build()
    rho = torch.from_numpy(rho64).to(F.DTYPES[prec]).cuda()
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    return plan, rho.double().cpu().numpy(), phi.double().cpu().numpy()


SMALL = [
    ("coulomb3d", (8.0, 8.0, 8.0), (32, 32, 32), None),
    ("coulomb3d", (3.0, 5.0, 4.0), (24, 16, 48), None),
    ("coulomb3d", (6.0, 6.0, 6.0), (12, 8, 16), None),
    ("yukawa3d", (8.0, 8.0, 8.0), (16, 24, 32), 1.0),
    ("biharmonic3d", (4.0, 4.0, 4.0), (16, 16, 16), None),
    ("log2d", (8.0, 6.0), (48, 96), None),
    ("log2d", (10.0, 5.0), (256, 128), None),
    ("log2d", (4.0, 16.0), (96, 24), None),
    ("coulomb2d", (6.0, 6.0), (24, 32), None),
    ("biharmonic2d", (5.0, 7.0), (32, 48), None),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,L,N,lam", SMALL)
def test_parity_small(F, kind, L, N, lam, prec):
    rho64 = density(kind, L, N, seed=sum(N))
    plan, rho_used, phi = run_gpu(F, kind, L, N, prec, rho64, lam=lam)
    ref = O.solve(kind, L, N, rho_used, eps=plan.eps, lam=lam or 0.0)
    check(phi, ref, prec, f"{kind} {N} {prec}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,L,N", [("coulomb3d", (4.0, 4.0, 4.0), (16, 24, 32)),
                                       ("log2d", (5.0, 5.0), (64, 48))])
def test_parity_rough_density(F, kind, L, N, prec):
    """A density with white noise: every frequency of the padded grid is excited."""
    rho64 = density(kind, L, N, seed=7, noise=True)
    plan, rho_used, phi = run_gpu(F, kind, L, N, prec, rho64)
    ref = O.solve(kind, L, N, rho_used, eps=plan.eps)
    check(phi, ref, prec, f"rough {kind} {N} {prec}")


@pytest.mark.parametrize("kind,L,N,lam", [("coulomb3d", (3.0, 5.0, 4.0), (24, 16, 32), None),
                                           ("yukawa3d", (4.0, 4.0, 4.0), (16, 16, 16), 2.0),
                                           ("yukawa3d", (4.0, 4.0, 4.0), (16, 24, 32), 1.0),
                                           ("coulomb3d", (4.0, 6.0, 4.0), (16, 96, 24), None),
                                           ("log2d", (8.0, 6.0), (48, 32), None),
                                           ("biharmonic2d", (3.0, 4.0), (16, 24), None)])
def test_tensor_matches_oracle_dft(F, kind, L, N, lam):
    """The GPU spectral octant equals DFT(T(1) + T(2)) / prod P of the oracle.
    The 3D Yukawa boxes are cubes, so W comes from the radial table and the
    last axis takes its rows ordered by a1^2 + a2^2 (a square and a
    rectangular set of rows); the 16 x 96 x 24 Coulomb grid transforms its
    middle axis at length 192 (3 * 2^6)."""
    plan = F.Plan(kind, L, N, "f64", lam=lam).build()
    got = plan.tensor().numpy()
    T = O.build_tensor(kind, L, N, plan.eps, lam=lam or 0.0)
    That = O.fftnd(T, -1) / T.size
    assert np.max(np.abs(That.imag)) <= 1e-14 * np.max(np.abs(That.real))
    octant = That.real[tuple(slice(0, n + 1) for n in N)]
    ref = np.transpose(octant, tuple(reversed(range(len(N)))))
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [(16, 24, 32), (48, 48, 48)])
def test_tensor_rebuild_is_bitwise_identical(F, N):
    """A rebuild (which reuses the line order the first build of a cubic box
    computed) writes the same tensor, bit for bit, as the first build and as
    a fresh plan's first build."""
    L = (4.0, 4.0, 4.0)
    plan = F.Plan("yukawa3d", L, N, "f64", lam=1.0).build()
    first = plan.tensor().clone()
    plan.build()
    again = plan.tensor().clone()
    fresh = F.Plan("yukawa3d", L, N, "f64", lam=1.0).build().tensor().clone()
    torch.cuda.synchronize()
    assert torch.equal(first, again)
    assert torch.equal(first, fresh)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_deterministic_and_in_place(F, prec):
    kind, L, N = "coulomb3d", (8.0, 8.0, 8.0), (32, 48, 24)
    plan = F.Plan(kind, L, N, prec).build()
    rho = torch.from_numpy(density(kind, L, N, 3)).to(F.DTYPES[prec]).cuda()
    a = plan.apply(rho)
    b = plan.apply(rho)
    c = rho.clone()
    plan.apply(c, out=c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, c)


def test_zero_density_gives_zero(F):
    plan = F.Plan("log2d", (4.0, 4.0), (64, 64), "f64").build()
    phi = plan.apply(torch.zeros(64, 64, dtype=torch.float64, device="cuda"))
    assert float(phi.abs().max()) == 0.0


def sampled_parity(F, kind, L, N, prec, rho64, lam=None, eps=None, npts=320, seed=0):
    """Full-size run; the oracle's direct sum of eq. DiscConv at ``npts``
    seeded points, the maximum of |phi|, and every corner and face centre."""
    plan, rho_used, phi = run_gpu(F, kind, L, N, prec, rho64, eps=eps, lam=lam)
    T = O.build_tensor(kind, L, N, plan.eps, lam=lam or 0.0)
    idx = sample_points(phi.shape, phi, npts, seed)
    ref = O.conv_direct_points(T, rho_used, idx)
    return check(phi.ravel()[idx], ref, prec, f"{kind} {N} {prec} sampled")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("gamma", [4.0, 16.0])
@pytest.mark.parametrize("orientation", ["pancake", "cigar"])
def test_parity_anisotropic_full_size(F, orientation, gamma, prec):
    """The cigar and pancake workload at its full size (256x256x64 /
    64x64x256 Coulomb, h = 1/16, Sec. 1), anisotropy 4 and 16: every grid
    point against the oracle's FFT route on the same input values."""
    p = synth.anisotropic_coulomb(orientation, gamma, prec)
    rho64 = synth.eval_gaussians(p.gaussians, p.L, p.N)
    plan, rho_used, phi = run_gpu(F, p.kernel, p.L, p.N, prec, rho64)
    ref = O.solve(p.kernel, p.L, p.N, rho_used, eps=plan.eps)
    check(phi, ref, prec, f"{orientation} gamma {gamma:g} {prec}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_parity_yukawa_256(F, prec):
    """3D Yukawa, lam = 1, eps = 2, 256^3 on [-8,8]^3, 8 Gaussians (the
    benchmark workload): every grid point against the oracle's FFT route."""
    p = synth.yukawa_problem(1.0, 256, prec)
    rho64 = synth.eval_gaussians(p.gaussians, p.L, p.N)
    plan, rho_used, phi = run_gpu(F, p.kernel, p.L, p.N, prec, rho64, eps=p.eps, lam=p.lam)
    ref = O.solve(p.kernel, p.L, p.N, rho_used, eps=plan.eps, lam=p.lam)
    check(phi, ref, prec, f"yukawa 256^3 lam 1 {prec}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("lam", [0.5, 4.0])
def test_parity_yukawa_lambda_128_full(F, lam, prec):
    """3D Yukawa with the other screening lengths of the workload (Sec. 5.3
    Example 4: lam 0.5 and 4; eps = 2, 8 Gaussians, [-8,8]^3) at 128^3: every
    grid point against the oracle.  At lam = 4 the device's U^eps takes a
    scaled-erfc form and the oracle exp * erfc, so the two sides evaluate the
    tensor by different formulas."""
    p = synth.yukawa_problem(lam, 128, prec)
    rho64 = synth.eval_gaussians(p.gaussians, p.L, p.N)
    plan, rho_used, phi = run_gpu(F, p.kernel, p.L, p.N, prec, rho64, eps=p.eps, lam=p.lam)
    ref = O.solve(p.kernel, p.L, p.N, rho_used, eps=plan.eps, lam=p.lam)
    check(phi, ref, prec, f"yukawa 128^3 lam {lam:g} {prec}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("lam", [0.5, 4.0])
def test_parity_yukawa_lambda_256_sampled(F, lam, prec):
    """The same screening lengths at 256^3: a few hundred sampled outputs
    against the oracle's direct sum."""
    p = synth.yukawa_problem(lam, 256, prec)
    rho64 = synth.eval_gaussians(p.gaussians, p.L, p.N)
    sampled_parity(F, p.kernel, p.L, p.N, prec, rho64, lam=p.lam, eps=p.eps, seed=int(lam * 8))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_config_coulomb32_three_gaussians(F, prec):
    """The plain method on the smallest workload (Sec. 5.1 Example 1 shape):
    3D Coulomb on [-8,8]^3 at 32^3, eps = R0/8 = 2, three isotropic Gaussians
    (seed 1000: centres U[-2,2]^3, widths U[0.8,1.5], amplitudes U[0.5,2]).
    Every grid point against the oracle, and against the closed-form erf
    potential of the Gaussians: the discretisation error at h = 1/2 for
    widths down to 1.6 h (the oracle's own error there is 4.3e-9; the
    workload's bar is 1e-4, FP64 is held to the oracle's level and FP32 to
    its own round-off)."""
    p = synth.isotropic_coulomb_32()
    rho64 = synth.eval_gaussians(p.gaussians, p.L, p.N)
    plan, rho_used, phi = run_gpu(F, p.kernel, p.L, p.N, prec, rho64)
    assert plan.eps == 2.0
    ref = O.solve(p.kernel, p.L, p.N, rho_used, eps=plan.eps)
    check(phi, ref, prec, f"coulomb 32^3 three Gaussians {prec}")
    gs = [(g.amp, g.center, g.width) for g in p.gaussians]
    exact = R.gaussian_sum_potential(p.kernel, gs, p.L, p.N)
    err = R.rel_max_err(phi, exact)
    print(f"coulomb 32^3 {prec}: rel max error against the closed form {err:.3e}")
    assert err <= 1e-4
    assert err <= (1e-8 if prec == "f64" else 2e-6)


DDI_N = (0.82778, 0.41505, -0.37751)
DDI_M = (0.3118, 0.9378, -0.15214)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L,N", [((8.0, 8.0, 8.0), (32, 32, 32)),
                                 ((3.0, 5.0, 4.0), (24, 16, 48)),
                                 ((6.0, 6.0, 3.0), (64, 48, 32))])
def test_parity_ddi(F, L, N, prec):
    """3D dipole-dipole: -(m.n) rho - 3 Coulomb(d_nm rho), the derivative on
    the GPU (five spectral launches) and the Coulomb convolution (five passes,
    the identity term added by pass E), against the oracle."""
    rho64 = density("coulomb3d", L, N, seed=sum(N) + 7)
    plan = F.Plan("ddi3d", L, N, prec, n=DDI_N, m=DDI_M).build()
    launches = plan.launches()
    assert launches[:5] == ["spectral"] * 5 and launches[5:] == ["r2c", "fwd_t", "conv",
                                                                  "inv_t", "c2r"]
    rho = torch.from_numpy(rho64).to(F.DTYPES[prec]).cuda()
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    ref = O.solve_ddi(L, N, rho.double().cpu().numpy(), plan.eps, DDI_N, DDI_M)
    check(phi.double().cpu().numpy(), ref, prec, f"ddi {N} {prec}")
    # in place (phi aliases rho): pass E reads each rho value before writing it
    rho2 = rho.clone()
    plan.apply(rho2, out=rho2)
    torch.cuda.synchronize()
    assert torch.equal(rho2, phi)


def test_ddi_not_batched_or_served(F):
    plan = F.Plan("ddi3d", (8.0,) * 3, (16,) * 3, "f32", n=DDI_N, m=DDI_M).build()
    r = torch.zeros(16, 16, 16, device="cuda")
    with pytest.raises(F.FsaError, match="EUNSUPPORTED"):
        F.apply_batched([plan], [r])
    srv = F.Server(1 << 30)
    try:
        k = F._kernel("ddi3d", None, None, DDI_N, DDI_M)
        import ctypes
        t = ctypes.c_uint64()
        Ls = (ctypes.c_double * 3)(8.0, 8.0, 8.0)
        Ns = (ctypes.c_int64 * 3)(16, 16, 16)
        st = F.lib().fsa_server_submit(srv._h, ctypes.byref(k), 3, Ls, Ns, 0,
                                       ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(r.data_ptr()), ctypes.byref(t))
        assert F.STATUS[st] == "FSA_EUNSUPPORTED"
    finally:
        srv.close()


_LARGEST_REF = {}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,L,N", [
    ("log2d", (12.0, 10.0), (2048, 2048)),          # the largest grid length on both axes
    ("coulomb2d", (9.0, 4.0), (1536, 96)),          # 3 * 2^9 padded to 3072
    ("coulomb3d", (8.0, 2.0, 2.0), (2048, 16, 8)),  # longest pencils of the fused pass
    ("coulomb3d", (2.0, 2.0, 8.0), (8, 16, 2048)),  # longest rows of the real passes
    ("coulomb3d", (2.0, 8.0, 2.0), (8, 2048, 16)),  # longest transposed lines
])
def test_parity_largest_lengths(F, kind, L, N, prec):
    """Grid lengths at the 2048 maximum on each axis (and a 3 * 2^a one):
    transform lengths 2048 (real passes) and 4096 (complex passes), whole-grid
    relative L2 against the oracle's FFT route."""
    rho64 = density(kind, L, N, seed=sum(N) + 11)
    plan, rho_used, phi = run_gpu(F, kind, L, N, prec, rho64)
    key = (kind, L, N)
    if key not in _LARGEST_REF:   # one oracle solve per grid (the FP64 density;
        _LARGEST_REF[key] = O.solve(kind, L, N, rho64, eps=plan.eps)  # FP32 rounding of
    check(phi, _LARGEST_REF[key], prec, f"{kind} {N} {prec}")  # rho is ~1e-7)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_table3_workload_192(F, golden, prec):
    """Table 3's timing workload: 3D Coulomb at 192^3 on [-12,12]^3 (h = 1/8),
    eps = 0.4, the Case II density (a Laplacian-of-Gaussian pair, sigma^2 =
    0.8, x0 = (1,1,0)) whose potential is Phi0.  Pass A runs length-192 rows,
    whose first radix-8 stage has 24 butterflies over 16 threads (the
    prefetch must skip the missing ones, or the last row reads past rho).
    FP64 reaches round-off against Phi0, as the paper's row does
    (3.3394e-16); FP32 its own round-off."""
    g = golden["fsa_timing_192"]
    n = g["N"]
    L, N, sigma, x0 = (12.0,) * 3, (n,) * 3, np.sqrt(0.8), (1.0, 1.0, 0.0)
    rho = synth.case2_density(L, N, sigma, (1.0, 1.0, 1.0), x0=x0)
    plan = F.Plan("coulomb3d", L, N, prec, eps=0.4).build()
    phi = plan.apply(torch.from_numpy(rho).to(F.DTYPES[prec]).cuda())
    torch.cuda.synchronize()
    ex = R.case2_phi0(L, N, sigma, (1.0, 1.0, 1.0), x0=x0)
    err = R.rel_max_err(phi.double().cpu().numpy(), ex)
    print(f"Table 3 workload {prec}: rel max err {err:.3e} (paper, FP64: {g['err']:.4e})")
    assert err <= (2e-15 if prec == "f64" else 2e-6)


def test_rejects_lengths_beyond_the_maximum(F):
    with pytest.raises(F.FsaError, match="EUNSUPPORTED"):
        F.Plan("coulomb3d", (8.0,) * 3, (4096, 8, 8))
    with pytest.raises(F.FsaError, match="EUNSUPPORTED"):
        F.Plan("log2d", (8.0, 8.0), (40, 40))    # 5 * 8: radix 5 not supported
