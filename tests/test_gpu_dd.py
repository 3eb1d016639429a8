"""The extended-precision (double-double) mode on the GPU against the
quadruple-precision oracle and the paper's quad row (Table 2).  Needs an
MI355X.

Tolerance: relative L2 1e-30 against the quad oracle on the same
double-double input (double-double rounds at ~1.2e-32; the FFTs and the
tensor's special functions add a few tens of roundings: 4e-32 to 8e-32 are
typical).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import reference as R
from paper_2504_19410_amd import synth

pytestmark = pytest.mark.gpu

TOL_DD = 1e-30


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19410_amd import fsa
    return fsa


def rand_dd(N, seed):
    rng = np.random.default_rng(seed)
    a = np.empty(tuple(N) + (2,))
    a[..., 0] = rng.standard_normal(N)
    a[..., 1] = a[..., 0] * 2.0 ** -53 * rng.uniform(-1, 1, N)
    return a


def run_dd(F, kind, L, N, rho_dd, eps=None):
    plan = F.Plan(kind, L, N, "dd", eps=eps).build()
    rho = torch.from_numpy(rho_dd).cuda()
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    return plan, phi.cpu().numpy()


@pytest.mark.parametrize("kind,L,N", [
    ("coulomb3d", (8.0, 8.0, 8.0), (16, 16, 16)),
    ("coulomb3d", (3.0, 5.0, 4.0), (8, 16, 32)),
    ("coulomb3d", (4.0, 4.0, 2.0), (32, 8, 8)),
    ("coulomb2d", (8.0, 6.0), (32, 64)),
    ("coulomb2d", (5.0, 9.0), (128, 16)),
])
def test_parity_dd(F, kind, L, N):
    rho = rand_dd(N, sum(N))
    plan, phi = run_dd(F, kind, L, N, rho)
    ref = O.solve_quad(kind, L, N, rho, plan.eps)
    err = R.dd_rel_l2_err(phi, ref)
    print(f"dd {kind} {N}: rel L2 {err:.3e}")
    assert err <= TOL_DD
    assert plan.launches() == (["r2c", "fwd_t", "conv", "inv_t", "c2r"] if len(N) == 3
                               else ["r2c", "conv", "c2r"])


@pytest.mark.parametrize("kind,L,N", [
    ("coulomb2d", (9.0, 2.0), (1024, 16)),        # the longest lines: P = 2048 along axis 0
    ("coulomb2d", (2.0, 9.0), (16, 1024)),        # ... and along the contiguous axis
    ("coulomb3d", (2.0, 2.0, 9.0), (8, 8, 1024)),
    ("coulomb2d", (8.0, 8.0), (512, 512)),
])
def test_parity_dd_largest_lengths(F, kind, L, N):
    rho = rand_dd(N, sum(N) + 1)
    plan, phi = run_dd(F, kind, L, N, rho)
    ref = O.solve_quad(kind, L, N, rho, plan.eps)
    err = R.dd_rel_l2_err(phi, ref)
    print(f"dd {kind} {N}: rel L2 {err:.3e}")
    assert err <= TOL_DD


def test_dd_tensor_matches_quad(F):
    """The double-double octant against the quad oracle's tensor, built the
    paper's way (T(1) + IDFT(W), then its DFT), through a delta density: the
    potential of a unit impulse at the origin is the tensor's row T[i, 0, 0]."""
    L, N = (4.0, 4.0, 4.0), (16, 16, 16)
    rho = np.zeros(N + (2,))
    rho[0, 0, 0, 0] = 1.0
    plan, phi = run_dd(F, "coulomb3d", L, N, rho)
    ref = O.solve_quad("coulomb3d", L, N, rho, plan.eps)
    assert R.dd_rel_max_err(phi, ref) <= 1e-30


def test_dd_in_place_and_deterministic(F):
    L, N = (8.0, 8.0), (64, 32)
    plan = F.Plan("coulomb2d", L, N, "dd").build()
    rho = torch.from_numpy(rand_dd(N, 9)).cuda()
    a = plan.apply(rho)
    b = plan.apply(rho)
    c = rho.clone()
    plan.apply(c, out=c)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_dd_agrees_with_fp64_plan(F):
    """The same discretisation in FP64: the double-double result's high parts
    equal the FP64 path's to FP64 rounding."""
    L, N = (8.0, 8.0, 8.0), (32, 32, 32)
    rho = rand_dd(N, 4)
    rho[..., 1] = 0.0
    _, phi_dd = run_dd(F, "coulomb3d", L, N, rho)
    p64 = F.Plan("coulomb3d", L, N, "f64").build()
    phi64 = p64.apply(torch.from_numpy(rho[..., 0].copy()).cuda()).cpu().numpy()
    assert np.linalg.norm(phi_dd[..., 0] - phi64) <= 1e-13 * np.linalg.norm(phi64)


@pytest.mark.parametrize("c", [2, 3])
def test_dd_table2_quad_row(F, golden, c):
    """Table 2's 3D quad row on the GPU: h = 1/4 reproduces 4.8161e-18 (the
    discretisation error, below FP64 round-off); h = 1/8 (128^3, printed
    2.4e-34) reaches double-double round-off against the exact potential."""
    g = golden["coulomb3d_iso_quad"]
    n = int(round(2 * g["L"] / g["h"][c]))
    L, N = (g["L"],) * 3, (n,) * 3
    rho = synth.gaussian_dd(L, N, g["sigma2"])
    _, phi = run_dd(F, "coulomb3d", L, N, rho, eps=g["eps"])
    err = R.dd_rel_max_err(phi, R.coulomb3d_iso_dd(L, N, g["sigma2"]))
    print(f"dd coulomb3d h={g['h'][c]}: rel max err {err:.4e} (printed {g['err'][c]:.4e})")
    if c == 2:
        assert abs(err - g["err"][c]) <= 1e-3 * g["err"][c]
    else:
        assert err <= 1e-30


def test_dd_2d_round_off(F, golden):
    g = golden["coulomb2d_iso"]
    L, N = (g["L"],) * 2, (128, 128)
    rho = synth.gaussian_dd(L, N, g["sigma2"])
    _, phi = run_dd(F, "coulomb2d", L, N, rho, eps=g["eps"])
    assert R.dd_rel_max_err(phi, R.coulomb2d_iso_dd(L, N, g["sigma2"])) <= 1e-30


def test_dd_not_batched_served_or_tuned(F):
    plan = F.Plan("coulomb3d", (8.0,) * 3, (16,) * 3, "dd").build()
    r = torch.zeros(16, 16, 16, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FsaError, match="EUNSUPPORTED"):
        F.apply_batched([plan], [r])
    with pytest.raises(F.FsaError, match="EUNSUPPORTED"):
        plan.autotune(r)
    srv = F.Server(1 << 30)
    try:
        import ctypes
        k = F._kernel("coulomb3d", None, None)
        t = ctypes.c_uint64()
        Ls = (ctypes.c_double * 3)(8.0, 8.0, 8.0)
        Ns = (ctypes.c_int64 * 3)(16, 16, 16)
        st = F.lib().fsa_server_submit(srv._h, ctypes.byref(k), 3, Ls, Ns, 2,
                                       ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(r.data_ptr()), ctypes.byref(t))
        assert F.STATUS[st] == "FSA_EUNSUPPORTED"
    finally:
        srv.close()
