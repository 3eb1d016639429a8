"""Error measures and the parity bar shared by the GPU tests.

Relative L2 = ||got - ref||_2 / ||ref||_2 and relative max =
max|got - ref| / max|ref| (the measure of the paper's tables, Sec. 5), both
over the points compared.  The bar is the same for both: 1e-12 for an FP64
plan and 5e-6 for an FP32 plan, against the FP64 oracle on the same input
values.
"""
import numpy as np

TOL = {"f64": 1e-12, "f32": 5e-6}


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check(got, ref, prec, label=""):
    """Assert relative L2 and relative max within the bar of ``prec`` (a
    precision name or a number); returns both."""
    tol = TOL[prec] if isinstance(prec, str) else float(prec)
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (label, got.shape, ref.shape)
    l2, mx = rel_l2(got, ref), rel_max(got, ref)
    print(f"{label}: rel L2 {l2:.3e}, rel max {mx:.3e} ({got.size} points)")
    assert l2 <= tol, (label, "rel L2", l2, tol)
    assert mx <= tol, (label, "rel max", mx, tol)
    return l2, mx


def sample_points(shape, phi, npts, seed):
    """Flat indices of ``npts`` seeded random grid points, plus the maximum of
    |phi|, and every corner and face centre of the grid (the first and last
    rows, pencils and tiles of every pass)."""
    size = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    pts = [rng.choice(size, min(npts, size), replace=False), [int(np.argmax(np.abs(phi)))]]
    d = len(shape)
    extra = []
    for m in range(3 ** d):
        idx, q = [], m
        for n in shape:
            idx.append((0, n // 2, n - 1)[q % 3])
            q //= 3
        extra.append(int(np.ravel_multi_index(idx, shape)))
    pts.append(extra)
    return np.unique(np.concatenate([np.asarray(p, dtype=np.int64) for p in pts]))
