"""Writes the shipped tuning table for this GPU: runs fsa_autotune on every
grid shape of the standard workloads (3D Coulomb/Yukawa grids of the single
evaluation and served workloads, the 2D log-kernel batch shapes) in FP32 and
FP64, and saves the table next to this script as <arch>.json (the arch name
reported by the device, e.g. gfx950).  Load it with fsa.tune_load(path) or by
pointing FSA_TUNE_CACHE at it.

Usage (on the GPU): python -m paper_2504_19410_amd.tune.make_table [--reps 7]
With --add, the shipped table is loaded first and only the extra 2D shapes
(FP64 log-kernel batch shapes, 2048^2 and 1024^2 grids) are tuned into it.
The batched launches of the 256-density 2D log-kernel batch are tuned last
(fsa_autotune_batched, entries kept apart from the single-evaluation ones);
with --batch, the shipped table is loaded and only they are tuned; with
--table3, only the 192^3 grid of the paper's timing workload.
"""
import argparse
import os

import numpy as np
import torch

from paper_2504_19410_amd import fsa as F
from paper_2504_19410_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))

SHAPES_3D = [
    ("yukawa3d", (8.0, 8.0, 8.0), (256, 256, 256), 1.0),
    ("coulomb3d", (8.0, 8.0, 8.0), (128, 128, 128), None),
    ("coulomb3d", (8.0, 8.0, 8.0), (64, 64, 64), None),
    ("coulomb3d", (8.0, 1.0, 1.0), (512, 64, 64), None),
    ("coulomb3d", (1.0, 1.0, 8.0), (64, 64, 512), None),
    ("coulomb3d", (8.0, 8.0, 2.0), (256, 256, 64), None),
    ("coulomb3d", (2.0, 2.0, 8.0), (64, 64, 256), None),
]


# the paper's timing workload (Table 3): 192^3 on [-12,12]^3, eps = 0.4
SHAPES_TABLE3 = [
    ("coulomb3d", (12.0, 12.0, 12.0), (192, 192, 192), None),
]


# large single 2D grids (2D Yukawa, quasi-2D dipole-dipole, log kernel)
SHAPES_2D_EXTRA = [
    ("yukawa2d", (12.0, 12.0), (2048, 2048), 2.0),
    ("yukawa2d", (12.0, 12.0), (1024, 1024), 2.0),
]


def arch_name():
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


def tune_batch(reps):
    """The batched launches of the 256-density 2D log-kernel batch (FP32)."""
    probs = synth.log2d_batch(256)
    plans = [F.Plan(p.kernel, p.L, p.N, "f32").build() for p in probs]
    rhos = [torch.from_numpy(synth.eval_gaussians(p.gaussians, p.L, p.N, dtype=np.float32)).cuda()
            for p in probs]
    F.autotune_batched(plans, rhos, reps=reps)
    groups = {}
    for p in probs:
        N0, N1 = p.N
        for key, lines in ((("r2c", N1), N0), (("conv", 2 * N0), N1 + 1), (("c2r", N1), N0)):
            groups[key] = groups.get(key, 0) + lines
    print("batch", {f"{a}_{b}": F.tune_get("f32", "batched_" + a, b, lines)
                    for (a, b), lines in groups.items()}, flush=True)
    for p in plans:
        p.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--out", default=None)
    ap.add_argument("--add", action="store_true",
                    help="tune only the extra 2D shapes into the shipped table")
    ap.add_argument("--batch", action="store_true",
                    help="tune only the batched launches into the shipped table")
    ap.add_argument("--table3", action="store_true",
                    help="tune only the 192^3 grid of Table 3 into the shipped table")
    args = ap.parse_args()
    table3 = [(k, L, N, lam, prec) for k, L, N, lam in SHAPES_TABLE3 for prec in ("f32", "f64")]
    extra = [(k, L, N, lam, prec) for k, L, N, lam in SHAPES_2D_EXTRA for prec in ("f32", "f64")]
    extra += [("log2d", (8.0, 8.0), N, None, "f64") for N in synth.LOG2D_SHAPES]
    if args.add or args.batch or args.table3:
        F.tune_load(os.path.join(HERE, f"{arch_name()}.json"))
        jobs = table3 if args.table3 else [] if args.batch else extra
    else:
        F.tune_reset()
        jobs = [(k, L, N, lam, prec) for k, L, N, lam in SHAPES_3D for prec in ("f32", "f64")]
        jobs += table3
        jobs += [("log2d", (8.0, 8.0), N, None, "f32") for N in synth.LOG2D_SHAPES]
        jobs += extra
    for kind, L, N, lam, prec in jobs:
        plan = F.Plan(kind, L, N, prec, lam=lam).build()
        rho = torch.rand(N, dtype=F.DTYPES[prec], device="cuda")
        table = plan.autotune(rho, reps=args.reps)
        print(kind, N, prec, {f"{a}_{b}": v for (a, b), v in table.items()}, flush=True)
        plan.close()
    if not (args.add or args.table3):
        tune_batch(args.reps)
    out = args.out or os.path.join(HERE, f"{arch_name()}.json")
    F.tune_save(out)
    print("wrote", out)


if __name__ == "__main__":
    main()
