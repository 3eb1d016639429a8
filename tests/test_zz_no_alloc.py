"""fsa_apply_noalloc: the evaluation without a caller workspace, for callers
that cannot allocate device memory.

Through the C ABI, two calls in a row (the second on a smaller grid) must give
the bits of fsa_apply with a caller workspace (same kernels, same launch
choices), which the parity tests hold to the oracle; a plan whose workspace
exceeds the static scratch is rejected before any launch.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
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


CASES = [
    # the first call fills most of the 128 MiB scratch, the second is smaller
    ("yukawa3d", (8.0, 8.0, 8.0), (128, 128, 128), "f64", 1.0),
    ("coulomb3d", (6.0, 4.0, 5.0), (24, 16, 32), "f32", None),
    ("log2d", (8.0, 6.0), (96, 48), "f64", None),
]


def test_noalloc_equals_apply_on_consecutive_calls(F):
    F.tune_reset()
    plans, rhos, outs = [], [], []
    for i, (kind, L, N, prec, lam) in enumerate(CASES):
        plan = F.Plan(kind, L, N, prec, lam=lam).build()
        assert plan.workspace_bytes <= F.NOALLOC_SCRATCH_BYTES
        plans.append(plan)
        rhos.append(torch.from_numpy(density(L, N, 50 + i)).to(F.DTYPES[prec]).cuda())
        outs.append(torch.full_like(rhos[-1], float("nan")))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    for plan, rho, out in zip(plans, rhos, outs):   # back to back on one stream
        plan.apply_noalloc(rho, out)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    for (kind, L, N, prec, lam), plan, rho, out in zip(CASES, plans, rhos, outs):
        ref = plan.apply(rho)          # caller workspace
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (kind, N, prec)
        if np.prod(N) <= 64 ** 3:
            oracle = O.solve(kind, L, N, rho.double().cpu().numpy(), eps=plan.eps,
                             lam=lam or 0.0)
            check(out.double().cpu().numpy(), oracle, prec, f"noalloc {kind} {N} {prec}")
    # again, after the larger call left its data in the scratch, in place
    again = rhos[1].clone()
    plans[1].apply_noalloc(again, again)
    torch.cuda.synchronize()
    assert torch.equal(again, outs[1])


def test_noalloc_rejects_plans_beyond_the_scratch(F):
    plan = F.Plan("coulomb3d", (8.0,) * 3, (256, 256, 256), "f32")   # 405 MB workspace
    assert plan.workspace_bytes > F.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(8, device="cuda")
    st = F.lib().fsa_apply_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(x.data_ptr()), None)
    assert F.STATUS[st] == "FSA_EINVAL"
    assert b"static scratch" in F.lib().fsa_last_error()
    plan.close()
