"""The autotuner and every compiled launch variant on the GPU.

Each variant (default; alternate radix family; half-size workgroups) and a
reduced occupancy must reach the same parity with the FP64 oracle as the
default path (relative L2 and relative max <= 1e-12 FP64, <= 5e-6 FP32); after fsa_autotune the
tuned path must still match, the batched path must stay bitwise equal to the
solo path, and a saved table must load back on the same device.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_19410_amd import synth
from parity import check, sample_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19410_amd import fsa
    return fsa


@pytest.fixture(autouse=True)
def clean_table(F):
    F.tune_reset()
    yield
    F.tune_reset()


def density(L, N, seed):
    rng = synth.SplitMix64(seed)
    gs = synth.draw_gaussians(rng, len(N), 3, [-l / 4 for l in L], [l / 4 for l in L],
                              [l / 5 for l in L], [l / 3 for l in L], isotropic=False)
    return synth.eval_gaussians(gs, L, N)


# shapes whose pass lengths have alternate-radix and half-workgroup variants
SHAPES = [
    ("coulomb3d", (6.0, 8.0, 8.0), (32, 64, 128)),
    ("yukawa3d", (8.0, 8.0, 4.0), (64, 128, 64)),
    ("log2d", (10.0, 6.0), (512, 256)),
    ("log2d", (12.0, 8.0), (1024, 512)),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,L,N", SHAPES)
def test_every_variant_matches_the_oracle(F, kind, L, N, prec):
    lam = 1.0 if kind == "yukawa3d" else None
    plan = F.Plan(kind, L, N, prec, lam=lam).build()
    rho = torch.from_numpy(density(L, N, sum(N))).to(F.DTYPES[prec]).cuda()
    ref = O.solve(kind, L, N, rho.double().cpu().numpy(), eps=plan.eps, lam=lam or 0.0)
    tried = set()
    for var in range(F.NUM_VARIANTS):
        for occ in (0, 1):
            F.tune_reset()
            used = []
            for name, n in plan.passes():
                v = var if var in F.tune_variants(prec, name, n) else 0
                F.tune_set(prec, name, n, v, occ)
                used.append(v)
            if (tuple(used), occ) in tried:
                continue
            tried.add((tuple(used), occ))
            phi = plan.apply(rho)
            torch.cuda.synchronize()
            check(phi.double().cpu().numpy(), ref, prec,
                  f"{kind} {N} {prec} variants {used} occ {occ}")
    assert len(tried) >= 4   # the shapes above exercise non-default variants


# every grid length the passes support (2^a and 3 * 2^a, 8 ... 2048): as the
# long axis of a 2D grid it sets the fused pass's length 2N (axis 0) or the
# real passes' length N (axis 1); the short axis (12) leaves a partial tile
LENGTHS = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("axis", [0, 1, "3d"])
@pytest.mark.parametrize("n", LENGTHS)
def test_every_length_and_variant_matches_the_oracle(F, n, axis, prec):
    """Every supported transform length, in every compiled launch variant, at
    full and reduced occupancy: the lengths 3 * 2^a whose first stage leaves
    some lanes without a butterfly, the tile edges of the transposing passes
    (a short axis of 12: not a multiple of the tile widths), and the longest
    rows and pencils.  axis "3d": a 3D grid (8, n, 12) whose axis 1 sets the
    transposing passes B and D to length 2n."""
    kind = "coulomb3d" if axis == "3d" else "log2d"
    N = (8, n, 12) if axis == "3d" else (n, 12) if axis == 0 else (12, n)
    L = tuple(0.25 * m for m in N)   # h = 1/2 on every axis
    plan = F.Plan(kind, L, N, prec, eps=1.0).build()
    rho = torch.from_numpy(density(L, N, 3 * n + len(N))).to(F.DTYPES[prec]).cuda()
    ref = O.solve(kind, L, N, rho.double().cpu().numpy(), eps=plan.eps)
    seen = set()
    for var in range(F.NUM_VARIANTS):
        for occ in (0, 1):
            F.tune_reset()
            used = []
            for name, m in plan.passes():
                v = var if var in F.tune_variants(prec, name, m) else 0
                F.tune_set(prec, name, m, v, occ)
                used.append(v)
            if (tuple(used), occ) in seen:
                continue
            seen.add((tuple(used), occ))
            phi = plan.apply(rho)
            torch.cuda.synchronize()
            check(phi.double().cpu().numpy(), ref, prec, f"{N} variants {used} occ {occ}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autotune_keeps_parity_and_batch_bitwise(F, prec, tmp_path):
    kind, L, N = "coulomb3d", (6.0, 8.0, 8.0), (32, 64, 128)
    plan = F.Plan(kind, L, N, prec).build()
    rho = torch.from_numpy(density(L, N, 7)).to(F.DTYPES[prec]).cuda()
    table = plan.autotune(rho, reps=3)
    slabs, slab_us = table.pop(("slabs", 0))
    assert slabs in (1, 2, 4, 8, 16) and slab_us > 0.0
    assert set(table) == set(plan.passes())
    for (name, n), (v, occ, us) in table.items():
        assert v in F.tune_variants(prec, name, n)
        assert us > 0.0
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    ref = O.solve(kind, L, N, rho.double().cpu().numpy(), eps=plan.eps)
    check(phi.double().cpu().numpy(), ref, prec, f"tuned {N} {prec}")
    # batched path with the tuned choices: bitwise equal to the solo path
    plan2 = F.Plan("log2d", (8.0, 8.0), (256, 512), prec).build()
    rho2 = torch.from_numpy(density((8.0, 8.0), (256, 512), 8)).to(F.DTYPES[prec]).cuda()
    plan2.autotune(rho2, reps=3)
    solo = [plan.apply(rho), plan2.apply(rho2)]
    outs = F.apply_batched([plan, plan2], [rho, rho2])
    torch.cuda.synchronize()
    for a, b in zip(solo, outs):
        assert torch.equal(a, b)
    # the table survives a save / reset / load on this device
    path = tmp_path / "tune.json"
    F.tune_save(str(path))
    before = {k: F.tune_get(prec, *k)[:2] for k in plan.passes()}
    F.tune_reset()
    F.tune_load(str(path))
    assert {k: F.tune_get(prec, *k)[:2] for k in plan.passes()} == before
    assert F.tune_get_slabs(prec, N)[0] == slabs


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batched_plans_at_lengths_3_2a(F, prec, variant):
    """Transforms of lengths 3 * 2^a from 192 in the batched (job table)
    kernels, every such launch on one radix family (0: the mid-3 palindrome
    on the wider team, 1: on the narrower one): each result bitwise equal to
    its solo run and within the oracle tolerance."""
    shapes = [((8.0, 6.0), (192, 96)), ((6.0, 8.0), (96, 192))]
    plans, rhos, forced = [], [], 0
    for i, (L, N) in enumerate(shapes):
        p = F.Plan("log2d", L, N, prec).build()
        for (name, n), lines in zip(p.passes(), p.pass_lines()):
            if n % 3 == 0 and n >= 192 and variant in F.tune_variants(prec, name, n):
                F.tune_set(prec, name, n, variant, 0, lines)
                forced += 1
        plans.append(p)
        rhos.append(torch.from_numpy(density(L, N, 40 + i)).to(F.DTYPES[prec]).cuda())
    assert forced >= 4   # conv 384; r2c, conv and c2r at 192
    solo = [p.apply(r) for p, r in zip(plans, rhos)]
    outs = F.apply_batched(plans, rhos)
    torch.cuda.synchronize()
    for p, r, a, b in zip(plans, rhos, solo, outs):
        assert torch.equal(a, b)
        ref = O.solve("log2d", p.L, p.N, r.double().cpu().numpy(), eps=p.eps)
        check(b.double().cpu().numpy(), ref, prec, f"batched v{variant} {p.N} {prec}")


def test_autotune_batched_tunes_the_batch_size_classes(F):
    """fsa_autotune_batched stores a choice for every launch of the batch
    among the batched entries, under the launch's own size class (many
    problems' transforms together), and leaves the single-evaluation entries
    alone; the tuned batch matches the oracle and its replays are bitwise
    equal to the outputs the tuner left."""
    shapes = [((10.0, 6.0), (256, 512)), ((12.0, 8.0), (1024, 256)), ((8.0, 8.0), (512, 512))]
    cases = [shapes[i % 3] for i in range(9)]
    plans = [F.Plan("log2d", L, N, "f32").build() for L, N in cases]
    rhos = [torch.from_numpy(density(L, N, 20 + i)).float().cuda()
            for i, (L, N) in enumerate(cases)]
    ws = torch.empty(F.batch_workspace_bytes(plans) + 256, dtype=torch.uint8, device="cuda")
    tuned = F.autotune_batched(plans, rhos, workspace=ws, reps=2)
    torch.cuda.synchronize()
    groups = {}
    for _, (N0, N1) in cases:
        for key, lines in ((("r2c", N1), N0), (("conv", 2 * N0), N1 + 1), (("c2r", N1), N0)):
            groups[key] = groups.get(key, 0) + lines
    for (name, n), lines in groups.items():
        v, occ, us = F.tune_get("f32", "batched_" + name, n, lines)
        assert v in F.tune_variants("f32", name, n) and us > 0.0, (name, n, lines)
        # the single-evaluation entries are left alone
        assert F.tune_get("f32", name, n, lines) == (0, 0, 0.0)
    for i in (0, 1, 2):
        L, N = cases[i]
        ref = O.solve("log2d", L, N, rhos[i].double().cpu().numpy(), eps=plans[i].eps)
        check(tuned[i].double().cpu().numpy(), ref, "f32", f"tuned batch problem {i} {N}")
    again = F.apply_batched(plans, rhos, workspace=ws)
    torch.cuda.synchronize()
    for a, b in zip(tuned, again):
        assert torch.equal(a, b)


def test_autotune_batched_mixed_kinds_and_precisions(F):
    """A batch of 3D and 2D problems in both precisions: the fused pass of the
    3D problems takes its input from pass B, which the tuner re-runs before
    each timed candidate; every tuned output still matches the oracle."""
    cases = [("coulomb3d", (6.0, 8.0, 8.0), (32, 64, 128), "f32", None),
             ("yukawa3d", (8.0, 8.0, 4.0), (64, 32, 32), "f64", 0.8),
             ("log2d", (10.0, 6.0), (256, 512), "f64", None),
             ("coulomb3d", (8.0, 8.0, 8.0), (32, 32, 32), "f32", None)]
    plans = [F.Plan(k, L, N, pr, lam=lam).build() for k, L, N, pr, lam in cases]
    rhos = [torch.from_numpy(density(L, N, 40 + i)).to(F.DTYPES[pr]).cuda()
            for i, (k, L, N, pr, lam) in enumerate(cases)]
    outs = F.autotune_batched(plans, rhos, reps=2)
    torch.cuda.synchronize()
    for (k, L, N, pr, lam), pl, r, o in zip(cases, plans, rhos, outs):
        ref = O.solve(k, L, N, r.double().cpu().numpy(), eps=pl.eps, lam=lam or 0.0)
        check(o.double().cpu().numpy(), ref, pr, f"tuned mixed batch {k} {N} {pr}")
    # e.g. the 2D FP64 problem's fused pass (length 512 over 513 pencils)
    assert F.tune_get("f64", "batched_conv", 512, 513)[2] > 0.0


def test_batch_recaptures_after_a_table_change(F):
    plan = F.Plan("log2d", (8.0, 8.0), (128, 256), "f32").build()
    rho = torch.from_numpy(density((8.0, 8.0), (128, 256), 9)).float().cuda()
    ws = torch.empty(F.batch_workspace_bytes([plan]) + 256, dtype=torch.uint8, device="cuda")
    outs = [torch.empty_like(rho)]
    a = F.apply_batched([plan], [rho], outs=outs, workspace=ws)[0].clone()
    # same plans, buffers and workspace: only the table generation changes,
    # and the replayed graph must follow it
    F.tune_set("f32", "conv", 256, 1, 0)      # radices 16.16 instead of 8.4.8
    b = F.apply_batched([plan], [rho], outs=outs, workspace=ws)[0]
    c = plan.apply(rho)
    torch.cuda.synchronize()
    assert torch.equal(b, c)
    assert not torch.equal(a, b)   # another radix split rounds differently
    ref = O.solve("log2d", (8.0, 8.0), (128, 256), rho.double().cpu().numpy(), eps=plan.eps)
    check(a.double().cpu().numpy(), ref, "f32", "before the table change")
    check(b.double().cpu().numpy(), ref, "f32", "after the table change")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_slab_schedules_are_bitwise_equal(F, prec):
    """Passes B, C, D in slabs of bins: the same kernels on the same pencils,
    so every slab count gives the same bits, and the oracle's result."""
    kind, L, N = "yukawa3d", (8.0, 6.0, 8.0), (48, 32, 64)
    plan = F.Plan(kind, L, N, prec, lam=0.5).build()
    rho = torch.from_numpy(density(L, N, 11)).to(F.DTYPES[prec]).cuda()
    base = plan.apply(rho)
    torch.cuda.synchronize()
    for slabs in (2, 3, 5, 16):
        F.tune_set_slabs(prec, N, slabs)
        assert F.tune_get_slabs(prec, N)[0] == slabs
        launches = plan.launches()
        assert len(launches) == 2 + 3 * slabs
        assert launches[0] == "r2c" and launches[-1] == "c2r"
        phi = plan.apply(rho)
        torch.cuda.synchronize()
        assert torch.equal(phi, base), slabs
    ref = O.solve(kind, L, N, rho.double().cpu().numpy(), eps=plan.eps, lam=0.5)
    check(base.double().cpu().numpy(), ref, prec, f"slabs {N} {prec}")


def test_apply_events_follow_the_schedule(F):
    plan = F.Plan("coulomb3d", (8.0, 8.0, 8.0), (32, 32, 32), "f32").build()
    rho = torch.from_numpy(density((8.0,) * 3, (32,) * 3, 12)).float().cuda()
    F.tune_set_slabs("f32", (32, 32, 32), 4)
    n = len(plan.launches())
    assert n == 14
    lib = ctypes.CDLL("libamdhip64.so")
    evs = []
    for _ in range(2 * n):
        e = ctypes.c_void_p()
        assert lib.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e.value)
    out = torch.empty_like(rho)
    with pytest.raises(F.FsaError, match="EINVAL"):
        plan.apply_events(rho, out, evs[:-1])          # one event short
    plan.apply_events(rho, out, evs)
    torch.cuda.synchronize()
    ref = plan.apply(rho)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # every launch's pair brackets it: positive durations that follow each
    # other in stream order
    f = ctypes.c_float()
    for i in range(n):
        assert lib.hipEventElapsedTime(ctypes.byref(f), ctypes.c_void_p(evs[2 * i]),
                                       ctypes.c_void_p(evs[2 * i + 1])) == 0
        assert f.value > 0.0
        if i:
            assert lib.hipEventElapsedTime(ctypes.byref(f), ctypes.c_void_p(evs[2 * i - 1]),
                                           ctypes.c_void_p(evs[2 * i])) == 0
            assert f.value >= 0.0
    # a null pair leaves its launch untimed; one null event of a pair is EINVAL
    part = [e if i // 2 == 2 else None for i, e in enumerate(evs)]
    plan.apply_events(rho, out, part)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    with pytest.raises(F.FsaError, match="one null event"):
        plan.apply_events(rho, out, [e if i != 3 else None for i, e in enumerate(evs)])
    for e in evs:
        lib.hipEventDestroy(ctypes.c_void_p(e))


SHIPPED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2504_19410_amd", "tune", "gfx950.json")


def sampled_check(kind, L, N, eps, lam, rho_used, phi, prec, label, npts=320, seed=0):
    """The oracle's direct sum of eq. DiscConv at ``npts`` seeded points, the
    maximum of |phi| and every corner and face centre of the grid."""
    T = O.build_tensor(kind, L, N, eps, lam=lam or 0.0)
    idx = sample_points(phi.shape, phi, npts, seed)
    ref = O.conv_direct_points(T, rho_used, idx)
    return check(phi.ravel()[idx], ref, prec, label)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_bench_configuration_parity(F, prec):
    """The 256^3 Yukawa evaluation in the launch configuration bench.py times:
    the shipped tuning table (variants, occupancy, slab schedule) loaded,
    every grid point against the oracle's FFT route."""
    if not os.path.exists(SHIPPED):
        pytest.skip("no shipped table")
    F.tune_load(SHIPPED)
    p = synth.yukawa_problem(1.0, 256, prec)
    plan = F.Plan(p.kernel, p.L, p.N, prec, eps=p.eps, lam=p.lam).build()
    rho = torch.from_numpy(synth.eval_gaussians(p.gaussians, p.L, p.N)).to(F.DTYPES[prec]).cuda()
    phi = plan.apply(rho)
    torch.cuda.synchronize()
    ref = O.solve(p.kernel, p.L, p.N, rho.double().cpu().numpy(), eps=plan.eps, lam=p.lam)
    check(phi.double().cpu().numpy(), ref, prec,
          f"bench configuration {prec}, launches {plan.launches()}")


def test_bench_batch_configuration_parity(F):
    """The 256-problem 2D log batch as bench.py runs it (shipped table, one
    captured graph): one problem of every grid shape checked on sampled
    outputs against the oracle's direct sum."""
    if not os.path.exists(SHIPPED):
        pytest.skip("no shipped table")
    F.tune_load(SHIPPED)
    probs = synth.log2d_batch(256)
    plans = [F.Plan(q.kernel, q.L, q.N, "f32") for q in probs]
    for pl in plans:
        pl.build()
    rhos = [torch.from_numpy(synth.eval_gaussians(q.gaussians, q.L, q.N, dtype=np.float32)).cuda()
            for q in probs]
    outs = F.apply_batched(plans, rhos)
    torch.cuda.synchronize()
    seen = {}
    for i, q in enumerate(probs):
        if q.N not in seen:
            seen[q.N] = i
    assert len(seen) == len(synth.LOG2D_SHAPES)
    for N, i in seen.items():
        q = probs[i]
        sampled_check(q.kernel, q.L, q.N, plans[i].eps, None, rhos[i].double().cpu().numpy(),
                      outs[i].double().cpu().numpy(), "f32", f"batch problem {i} {N}",
                      npts=200, seed=i)
