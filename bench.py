#!/usr/bin/env python3
"""Throughput of the FSA convolution hot path on one MI355X.

One step = one evaluation of the potential (Execution in the paper's terms,
Sec. 5.1 Example 2): the 5 fused FFT-convolution passes over a 256^3 grid,
with the kernel tensor built once beforehand (Precomp, timed separately).

Workload: 3D Yukawa kernel e^{-lam r}/(4 pi r), lam = 1, eps = 2, on
[-8,8]^3 at 256^3, density = 8 seeded Gaussians (widths U[0.5,1.5]).
The FP64 path (the paper's precision, Table 3) gives `value`; the FP32 FFT
path (FP64-built tensor) is reported beside it with its own roofline.  The
step time is the median of per-evaluation hipEvent pairs.  Inputs are
resident in HBM before the timed region.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import ctypes
import hashlib
import json
import math
import os
import platform
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid pts/s per conv (FP64 vs FP32) at 256^3; %HBM peak; p50/p99 served latency"
HBM_PEAK_BPS = 8.0e12
PASS_NAMES_3D = ["A_r2c", "B_fwd_t", "C_conv", "D_inv_t", "E_c2r"]
PASS_NAMES_2D = ["A_r2c", "C_conv", "E_c2r"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def model_bytes(N, prec):
    """Algorithmic HBM bytes of each pass (every array read and written once):
    r = bytes per real, c = 2r, H = N_last + 1, M = prod N_j."""
    r = 4 if prec == "f32" else 8
    c = 2 * r
    if len(N) == 3:
        N0, N1, N2 = N
        H = N2 + 1
        M = N0 * N1 * N2
        X1 = N0 * N1 * H * c         # [i0][p2][i1]
        X2 = N0 * 2 * N1 * H * c     # [p2][p1][i0]
        Tb = (N0 + 1) * (N1 + 1) * (N2 + 1) * r
        return {"A_r2c": M * r + X1, "B_fwd_t": X1 + X2, "C_conv": 2 * X2 + Tb,
                "D_inv_t": X2 + X1, "E_c2r": X1 + M * r}
    N0, N1 = N
    H = N1 + 1
    M = N0 * N1
    X = N0 * H * c
    Tb = (N0 + 1) * (N1 + 1) * r
    return {"A_r2c": M * r + X, "C_conv": 2 * X + Tb, "E_c2r": X + M * r}


def precomp_model(N, prec):
    """Algorithmic HBM bytes and nominal FLOPs of one tensor build (Precomp).

    Bytes: the octant (prod_j (N_j + 1) values) is written in FP64 by the
    first axis' DCT (which generates T(1) itself), read and written by each
    middle axis, read by the last axis, which writes the tensor in the plan
    precision.  FLOPs: 5 P log2 P per complex FFT of length P = 2 N_j, one
    FFT per pair of lines of each axis (the special functions of T(1) and W
    are not counted)."""
    D = [n + 1 for n in N]
    octant = 1
    for x in D:
        octant *= x
    r = 4 if prec == "f32" else 8
    nbytes = (8 + 16 * (len(N) - 2) + 8 + r) * octant
    flops = 0.0
    for j, n in enumerate(N):
        P = 2 * n
        flops += (octant / D[j]) / 2 * 5 * P * math.log2(P)
    return nbytes, flops


class Hip:
    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so")
        P = ctypes.c_void_p
        self.lib.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(P), ctypes.c_uint]
        self.lib.hipEventRecord.argtypes = [P, P]
        self.lib.hipEventSynchronize.argtypes = [P]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), P, P]
        self.lib.hipEventDestroy.argtypes = [P]

    # hipEventDisableSystemFence: a timing event that does not write back and
    # invalidate the caches when it is recorded (a default event does, which
    # leaves the next kernel a cold L2 and a ~10 us gap, and so changes the
    # time it measures)
    TIMING_FLAGS = 0x20000000

    def event(self):
        e = ctypes.c_void_p()
        rc = self.lib.hipEventCreateWithFlags(ctypes.byref(e), self.TIMING_FLAGS)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
        return e

    def record(self, e, stream):
        rc = self.lib.hipEventRecord(e, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def ms(self, a, b):
        self.lib.hipEventSynchronize(b)
        f = ctypes.c_float()
        rc = self.lib.hipEventElapsedTime(ctypes.byref(f), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(f.value)

    def destroy(self, e):
        self.lib.hipEventDestroy(e)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fsa_fft.hpp", "fsa_walk.hpp", "fsa_passes.hpp", "fsa_launch.hpp"):
        with open(os.path.join(ROOT, "paper_2504_19410_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key, prec, slabs):
    """HBM bytes per launch of one kernel instance (key: pass_prec_len_vVAR)
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources with the same slab schedule; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_hash") != kernel_source_hash():
            return None
        if d.get("slabs", {}).get(prec, 1) != slabs:
            return None
        ent = d["kernels"][key]
        return int(ent["fetch_bytes"] + ent["write_bytes"])
    except Exception:
        return None


SETTLE_S = 0.3


def timed_evals(run, torch, hip, steps, warmup, settle_s=SETTLE_S):
    """Times `steps` calls of `run` (one evaluation each) with a hipEvent pair
    around every call on the current stream; returns the median (the step
    time reported), the mean, the first, and the wall time of the span.

    Before the `warmup` untimed calls, evaluations run back to back for at
    least `settle_s` seconds of wall time: the GPU leaves its idle clocks
    within tens of milliseconds of sustained work, and the host-side
    preparation before a timed leg (density synthesis, uploads, plan builds)
    leaves it idle long enough to drop them, so a few warm-up calls alone
    time the ramp."""
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    settle = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < settle_s or settle < 20:
        for _ in range(10):
            run()
        settle += 10
        torch.cuda.synchronize()
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    evs = [hip.event() for _ in range(steps + 1)]
    t0 = time.perf_counter()
    hip.record(evs[0], stream)
    for k in range(steps):
        run()
        hip.record(evs[k + 1], stream)
    total = hip.ms(evs[0], evs[steps])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    per = [hip.ms(evs[k], evs[k + 1]) for k in range(steps)]
    for e in evs:
        hip.destroy(e)
    return {"median_ms": float(np.median(per)), "mean_ms": total / steps, "first_ms": per[0],
            "wall_ms": wall, "per_ms": per, "settle_evals": settle}


def bench_precision(F, torch, hip, prob, rho64, prec, steps, warmup, tune=True):
    dtype = F.DTYPES[prec]
    stream = torch.cuda.current_stream()
    plan = F.Plan(prob.kernel, prob.L, prob.N, prec, eps=prob.eps, lam=prob.lam)
    # Precomp: tensor generation, timed with events on the same stream (the
    # first build also allocates the tensor and twiddles; median of 9 builds)
    e0, e1 = hip.event(), hip.event()
    plan.build()
    precomp_ms = timed_evals(lambda: plan.build(), torch, hip, 9, 2, settle_s=0.1)["median_ms"]
    rho = torch.from_numpy(rho64).to(dtype).cuda()
    out = torch.empty_like(rho)
    ws = plan.workspace()
    # launch choices per pass from the autotuner (untimed, before warm-up)
    if tune:
        tuned = plan.autotune(rho, reps=5)
    else:   # report the table in force (defaults, or a loaded one)
        tuned = plan.tuned()
        if plan.d == 3:
            tuned[("slabs", 0)] = F.tune_get_slabs(prec, plan.N)
    timing = timed_evals(lambda: plan.apply(rho, out, ws), torch, hip, steps, warmup)
    # per-pass durations: for each pass, K more evaluations with a start and
    # an end event recorded around that pass's launches only (the 3D middle
    # passes launch once per slab of the schedule); the pass's time is the
    # median over the evaluations of the sum over its launches.  Events
    # around every launch of one evaluation would put two event packets
    # between consecutive kernels and stretch each interval by a few us.
    launches = plan.launches()
    names = PASS_NAMES_3D if plan.d == 3 else PASS_NAMES_2D
    by_short = {n.split("_", 1)[1]: n for n in names}
    pass_ms = {n: 0.0 for n in names}
    pass_launches = {n: 0 for n in names}
    for i, ln in enumerate(launches):
        pass_launches[by_short[ln]] += 1
    for name in names:
        idx = [i for i, ln in enumerate(launches) if by_short[ln] == name]
        per = []
        for k in range(steps):
            evs = [None] * (2 * len(launches))
            for i in idx:
                evs[2 * i], evs[2 * i + 1] = hip.event(), hip.event()
            plan.apply_events(rho, out, evs, ws)
            torch.cuda.synchronize()
            per.append(sum(hip.ms(evs[2 * i], evs[2 * i + 1]) for i in idx))
            for i in idx:
                hip.destroy(evs[2 * i])
                hip.destroy(evs[2 * i + 1])
        pass_ms[name] = float(np.median(per))
    hip.destroy(e0)
    hip.destroy(e1)
    phi = out.double().cpu().numpy()
    plan.close()
    ms = timing["median_ms"]
    pts = 1
    for n in prob.N:
        pts *= n
    mb = model_bytes(prob.N, prec)
    dom = max(pass_ms, key=pass_ms.get)
    # per launch: the pass's bytes and time split over its launches
    nl = pass_launches[dom]
    achieved = mb[dom] / (pass_ms[dom] * 1e-3)
    dom_pass, dom_len = plan.passes()[names.index(dom)]
    dom_var = F.tune_get(prec, dom_pass, dom_len, plan.pass_lines()[names.index(dom)] // nl)[0]
    dom_key = f"{dom_pass}_{prec}_{dom_len}_v{dom_var}"
    slabs = F.tune_get_slabs(prec, plan.N)[0] if plan.d == 3 else 1
    traffic = measured_traffic(dom_key, prec, slabs)
    pb, pf = precomp_model(prob.N, prec)
    return {
        "value": pts / (ms * 1e-3),
        "ms_per_step": ms,
        "precomp": {"ms": precomp_ms, "model_bytes": pb, "nominal_fft_flops": pf,
                    "achieved_GBps": pb / (precomp_ms * 1e-3) / 1e9,
                    "hbm_frac": pb / (precomp_ms * 1e-3) / HBM_PEAK_BPS,
                    "fp64_frac": pf / (precomp_ms * 1e-3) / 78.6e12},
        "mean_ms_per_step": timing["mean_ms"],
        "first_ms": timing["first_ms"],
        "wall_ms_per_step": timing["wall_ms"] / steps,
        "settle_evals": timing["settle_evals"],
        "precomp_ms": precomp_ms,
        "pass_ms": {k: round(v, 5) for k, v in pass_ms.items()},
        "tuned": {(f"{name}_{n}" if name != "slabs" else "slabs"):
                  ({"variant": t[0], "occupancy": t[1], "us": round(t[2], 2)} if name != "slabs"
                   else {"slabs": t[0], "us": round(t[1], 2)})
                  for (name, n), t in tuned.items()},
        "launches_per_step": len(launches),
        "model_bytes_per_step": sum(mb.values()),
        "model_hbm_frac": sum(mb.values()) / (ms * 1e-3) / HBM_PEAK_BPS,
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved / 1e9,
            "peak": HBM_PEAK_BPS / 1e9,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_BPS,
            "traffic": traffic,
            "instance": dom_key,
            "launches_per_step": nl,
            "algorithmic_bytes": mb[dom] / nl,
            "avg_launch_ms": pass_ms[dom] / nl,
        },
    }, phi


def bench_conv_variants(F, torch, hip, prob, rho64, tune_file, steps=40):
    """Pass C of the bench workload in every compiled variant of its kernel
    at full occupancy, the other passes as the table has them: event pairs
    around the pass-C launches only, median per launch over `steps`
    evaluations after a settle phase.  Variant 3 exchanges the operands
    between the last two stages of each 512-point transform across lanes
    (DPP and lane swaps) instead of through the LDS."""
    out = {}
    for prec in ("f32", "f64"):
        plan = F.Plan(prob.kernel, prob.L, prob.N, prec, eps=prob.eps, lam=prob.lam).build()
        rho = torch.from_numpy(rho64).to(F.DTYPES[prec]).cuda()
        phi = torch.empty_like(rho)
        ws = plan.workspace()
        name, length = plan.passes()[2]
        launches = plan.launches()
        ci = [i for i, ln in enumerate(launches) if ln == name]
        lines = plan.pass_lines()[2] // len(ci)
        keep = F.tune_get(prec, name, length, lines)
        bytes_launch = model_bytes(prob.N, prec)["C_conv"] / len(ci)
        res = {}
        for var in F.tune_variants(prec, name, length):
            F.tune_set(prec, name, length, var, 0, lines)
            timed_evals(lambda: plan.apply(rho, phi, ws), torch, hip, 5, 5, settle_s=0.1)
            per = []
            for _ in range(steps):
                evs = [None] * (2 * len(launches))
                for i in ci:
                    evs[2 * i], evs[2 * i + 1] = hip.event(), hip.event()
                plan.apply_events(rho, phi, evs, ws)
                torch.cuda.synchronize()
                for i in ci:
                    per.append(hip.ms(evs[2 * i], evs[2 * i + 1]))
                    hip.destroy(evs[2 * i])
                    hip.destroy(evs[2 * i + 1])
            us = float(np.median(per)) * 1e3
            res[f"v{var}"] = {"us_per_launch": round(us, 2),
                              "GBps": round(bytes_launch / (us * 1e-6) / 1e9, 1),
                              "frac": round(bytes_launch / (us * 1e-6) / HBM_PEAK_BPS, 4)}
        if tune_file:
            F.tune_load(tune_file)
        else:
            F.tune_set(prec, name, length, keep[0], keep[1], lines)
        plan.close()
        out[prec] = {"launches_per_step": len(ci), "variants": res}
    out["variants"] = {"v0": "default plan and workgroup", "v1": "alternate radix family",
                       "v2": "half-size workgroups",
                       "v3": "default plan, last exchange of each transform across lanes "
                             "(DPP row rotation + v_permlane16/32_swap) instead of LDS",
                       "v4": "default plan, first forward stage as FP32 16x16x4 MFMA "
                             "products (operands loaded in the MFMA layout)"}
    return out


def precomp_sweep(F, torch, hip, n=256, gammas=(1, 2, 4, 8, 16), reps=5):
    """Tensor generation (Precomp) time against anisotropy: 3D Coulomb on
    [-8,8]^2 x [-8/g, 8/g] at n^3 (h_z = h/g), eps = R0/8; the paper reports
    FSA's precomputation as independent of the anisotropy (Sec. 5.1)."""
    out = {}
    for g in gammas:
        plan = F.Plan("coulomb3d", (8.0, 8.0, 8.0 / g), (n, n, n), "f32")
        out[str(g)] = round(_time_build(plan, torch, hip, reps), 3)
        plan.close()
    return {"grid": [n, n, n], "kernel": "coulomb3d", "ms_by_anisotropy": out}


def bench_ddi(F, torch, hip, synth, n=256, steps=50, warmup=10):
    """3D dipole-dipole evaluation at n^3 (FP32 and FP64): the derivative
    launches plus the Coulomb passes, with the paper's dipole orientations
    (Sec. 5.3) on the Yukawa workload's density."""
    prob = synth.yukawa_problem(1.0, n, "f32")
    rho64 = synth.eval_gaussians(prob.gaussians, prob.L, prob.N)
    out = {}
    for prec in ("f32", "f64"):
        plan = F.Plan("ddi3d", prob.L, prob.N, prec, eps=prob.eps,
                      n=(0.82778, 0.41505, -0.37751), m=(0.3118, 0.9378, -0.15214)).build()
        rho = torch.from_numpy(rho64).to(F.DTYPES[prec]).cuda()
        ms = _time_apply(plan, rho, torch, hip, steps=steps, warmup=warmup)
        plan.close()
        out[prec] = {"ms_per_step": ms, "value": prob.points / (ms * 1e-3)}
    return {"workload": f"3D dipole-dipole on the {n}^3 Yukawa-workload density, paper's n and m",
            "unit": "grid pts/s", **out}


def _time_build(plan, torch, hip, reps=5):
    """Median event-timed tensor build (see timed_evals)."""
    plan.build()
    return timed_evals(lambda: plan.build(), torch, hip, reps, 1, settle_s=0.05)["median_ms"]


def _time_apply(plan, rho, torch, hip, steps=20, warmup=5, settle_s=0.05):
    """Median event-timed evaluation (see timed_evals)."""
    o = torch.empty_like(rho)
    ws = plan.workspace()
    return timed_evals(lambda: plan.apply(rho, o, ws), torch, hip, steps, warmup,
                       settle_s=settle_s)["median_ms"]


def bench_aniso(F, torch, hip, synth, steps=20):
    """The anisotropic cigar and pancake densities (Sec. 1, Fig. 1): 3D
    Coulomb at h = 1/16 on every axis, pancake 256x256x64 on [-8,8]^2 x [-2,2]
    (rho = exp(-(x^2 + y^2) - gamma^2 z^2)) and cigar 64x64x256 on
    [-2,2]^2 x [-8,8] (rho = exp(-gamma^2 (x^2 + y^2) - z^2)), eps = R0/8 =
    0.5, gamma in {4, 16}.  FP32 and FP64 evaluation times (they do not depend
    on gamma) and the outputs, for the error check against the exact potential
    in the oracle leg."""
    out, phis = {}, {}
    for orient in ("pancake", "cigar"):
        row = {}
        for prec in ("f32", "f64"):
            p4 = synth.anisotropic_coulomb(orient, 4.0, prec)
            plan = F.Plan(p4.kernel, p4.L, p4.N, prec).build()
            for gamma in (4.0, 16.0):
                p = synth.anisotropic_coulomb(orient, gamma, prec)
                rho = torch.from_numpy(synth.eval_gaussians(p.gaussians, p.L, p.N)).to(
                    F.DTYPES[prec]).cuda()
                if gamma == 4.0:
                    ms = _time_apply(plan, rho, torch, hip, steps=steps)
                    pts = p.N[0] * p.N[1] * p.N[2]
                    mb = sum(model_bytes(p.N, prec).values())
                    row[prec] = {"ms_per_step": round(ms, 4), "value": pts / (ms * 1e-3),
                                 "model_hbm_frac": mb / (ms * 1e-3) / 8e12}
                phis[(orient, gamma, prec)] = (p, plan.apply(rho).double().cpu().numpy())
            plan.close()
        out[orient] = {"grid": list(p4.N), "box": list(p4.L), **row}
    return out, phis


def bench_yukawa_lambda(F, torch, hip, synth, steps=20):
    """The Yukawa workload over its screening lengths: lambda in {0.5, 1, 4}
    on [-8,8]^3 at 128^3 and 256^3, eps = 2, 8 seeded Gaussians, FP32 and FP64
    (tensors built in FP64 on the GPU).  The evaluation time does not depend
    on lambda (timed at 128^3; 256^3 is the headline line); the outputs go to
    the oracle leg for the error against the exact potential."""
    out, phis = {}, {}
    for n in (128, 256):
        for prec in ("f32", "f64"):
            for lam in (0.5, 1.0, 4.0):
                p = synth.yukawa_problem(lam, n, prec)
                plan = F.Plan(p.kernel, p.L, p.N, prec, eps=p.eps, lam=p.lam).build()
                rho = torch.from_numpy(synth.eval_gaussians(p.gaussians, p.L, p.N)).to(
                    F.DTYPES[prec]).cuda()
                if n == 128 and lam == 1.0:
                    ms = _time_apply(plan, rho, torch, hip, steps=steps)
                    out[f"{n}_{prec}"] = {"ms_per_step": round(ms, 4),
                                          "value": n ** 3 / (ms * 1e-3)}
                phis[(n, lam, prec)] = (p, plan.apply(rho).double().cpu().numpy())
                plan.close()
    return out, phis


def bench_table3(F, torch, hip, synth):
    """The paper's timing workload (Table 3, Sec. 5.1 Example 2): 3D Coulomb
    on [-12,12]^3 at h = 1/8 (192^3), eps = 0.4, the Case II density
    rho = -Laplace(Phi0) with Phi0 = exp(-|x|^2/0.8) + exp(-|x - x0|^2/0.8),
    x0 = (1, 1, 0), whose potential is Phi0 itself.  Tensor build
    (Precomp) and one evaluation (Execution) in FP64 and FP32, and the
    relative max error against Phi0 (the paper's measure)."""
    L, N, sigma, x0 = (12.0,) * 3, (192,) * 3, math.sqrt(0.8), (1.0, 1.0, 0.0)
    rho64 = synth.case2_density(L, N, sigma, (1.0, 1.0, 1.0), x0=x0)
    X = np.meshgrid(*synth.grid_axes(L, N), indexing="ij")
    phi0 = (np.exp(-(X[0] ** 2 + X[1] ** 2 + X[2] ** 2) / sigma ** 2) +
            np.exp(-((X[0] - x0[0]) ** 2 + (X[1] - x0[1]) ** 2 + (X[2] - x0[2]) ** 2) /
                   sigma ** 2))
    del X
    out = {"workload": "3D Coulomb, Case II density (Laplacian of a Gaussian pair, sigma^2 = "
                       "0.8, x0 = (1,1,0)) on [-12,12]^3, 192^3 grid (h = 1/8), eps = 0.4",
           "paper": "Precomp 2.84 s, Execution 2.24 s, error 3.3394e-16 (FP64, FORTRAN on one "
                    "Xeon Gold 6248R; other hardware, context only)"}
    for prec in ("f64", "f32"):
        plan = F.Plan("coulomb3d", L, N, prec, eps=0.4)
        precomp = _time_build(plan, torch, hip)
        rho = torch.from_numpy(rho64).to(F.DTYPES[prec]).cuda()
        ms = _time_apply(plan, rho, torch, hip)
        phi = plan.apply(rho).double().cpu().numpy()
        plan.close()
        err = float(np.abs(phi - phi0).max() / np.abs(phi0).max())
        out[prec] = {"precomp_ms": round(precomp, 3), "execution_ms": round(ms, 4),
                     "rel_max_err_vs_exact": err}
    return out


def bench_general(F, torch, hip, n=256, n2=2048):
    """The general construction (window + quadrature W, Sec. 4): tensor
    generation of 3D Yukawa at n^3 against the closed-form split, 2D Yukawa
    and the quasi-2D DDI at n2^2 (Table 5's L = 12, lambda = 2, eta =
    1/sqrt(32)); evaluation times of the two 2D kernels."""
    out = {}
    for general in (False, True):
        plan = F.Plan("yukawa3d", (8.0,) * 3, (n,) * 3, "f32", eps=1.0, lam=2.0,
                      general=general)
        out["yukawa3d_%d_precomp_ms_%s" % (n, "general" if general else "closed")] = round(
            _time_build(plan, torch, hip), 3)
        plan.close()
    axes = [(-12.0 + np.arange(n2) * (24.0 / n2)) for _ in range(2)]
    X = np.meshgrid(*axes, indexing="ij")
    rho64 = np.exp(-(X[0] ** 2 + X[1] ** 2) / 1.2)
    for kind, kw in (("yukawa2d", {"lam": 2.0}),
                     ("quasi2d_ddi", {"eta": 1 / np.sqrt(32), "n": (0.0, 0.0, 1.0)})):
        for prec in ("f32", "f64"):
            plan = F.Plan(kind, (12.0, 12.0), (n2, n2), prec, eps=1.0, **kw)
            if prec == "f32":
                out["%s_%d_precomp_ms" % (kind, n2)] = round(_time_build(plan, torch, hip), 3)
            else:
                plan.build()
            rho = torch.from_numpy(rho64).to(F.DTYPES[prec]).cuda()
            ms = _time_apply(plan, rho, torch, hip)
            out["%s_%d_%s_ms" % (kind, n2, prec)] = round(ms, 4)
            plan.close()
    return out


def bench_dd(F, torch, hip, synth, n=128):
    """The extended-precision (double-double) mode: Table 2's 3D Coulomb
    problem (L = 8, sigma^2 = 0.8, eps = 1) at n^3 = 128^3 (h = 1/8); tensor
    build and evaluation times."""
    L, N = (8.0,) * 3, (n,) * 3
    plan = F.Plan("coulomb3d", L, N, "dd", eps=1.0)
    pre = _time_build(plan, torch, hip)
    rho = torch.from_numpy(synth.gaussian_dd(L, N, 0.8)).cuda()
    ms = _time_apply(plan, rho, torch, hip, steps=5, warmup=2)
    plan.close()
    return {"workload": f"3D Coulomb {n}^3, double-double (Table 2's quad problem)",
            "precomp_ms": round(pre, 3), "ms_per_step": round(ms, 3),
            "value": n ** 3 / (ms * 1e-3), "unit": "grid pts/s"}


def stream_copy(torch, hip, nbytes=1 << 30, reps=10):
    """Device-to-device copy of nbytes (torch copy_ kernel): the practical
    bandwidth of the box, read + write bytes over time."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = hip.event(), hip.event()
    hip.record(e0, stream)
    for _ in range(reps):
        y.copy_(x)
    hip.record(e1, stream)
    ms = hip.ms(e0, e1) / reps
    hip.destroy(e0)
    hip.destroy(e1)
    del x, y
    return 2.0 * nbytes / (ms * 1e-3)


def bench_batch(F, torch, hip, synth, steps, warmup, count=256, tune=True):
    """The batched 2D log workload: `count` seeded densities on grids drawn
    from {256^2, 512^2, 1024x256, 2048x512, 1024^2}, boxes L_j in U[4,16],
    FP32 FFT with FP64-built tensors, one captured graph of persistent
    launches; compared with the same problems issued one fsa_apply at a time."""
    probs = synth.log2d_batch(count)
    t0 = time.perf_counter()
    plans = [F.Plan(p.kernel, p.L, p.N, "f32") for p in probs]
    stream = torch.cuda.current_stream()
    e0, e1 = hip.event(), hip.event()
    hip.record(e0, stream)
    for pl in plans:
        pl.build()
    hip.record(e1, stream)
    build_ms = hip.ms(e0, e1)
    rhos = [torch.from_numpy(synth.eval_gaussians(p.gaussians, p.L, p.N, dtype=np.float32)).cuda()
            for p in probs]
    outs = [torch.empty_like(r) for r in rhos]
    ws = torch.empty(F.batch_workspace_bytes(plans) + 256, dtype=torch.uint8, device="cuda")
    # autotune one plan per grid shape for the per-call path, then the batch's
    # own launches (their size classes are the batch's, not a problem's)
    t_tune = time.perf_counter()
    if tune:
        seen = set()
        for pl, r in zip(plans, rhos):
            if pl.N not in seen:
                seen.add(pl.N)
                pl.autotune(r, reps=5)
        F.autotune_batched(plans, rhos, outs, ws, reps=5)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t_tune
    log(f"  batch setup {time.perf_counter() - t0:.1f} s (tensor builds {build_ms:.1f} ms, "
        f"autotune {tune_s:.1f} s)")
    t1 = time.perf_counter()
    F.apply_batched(plans, rhos, outs, ws)  # captures the graph
    torch.cuda.synchronize()
    capture_ms = (time.perf_counter() - t1) * 1e3
    launches = F.batch_launches(plans, rhos, outs, ws)
    for _ in range(warmup):
        F.apply_batched(plans, rhos, outs, ws)
    torch.cuda.synchronize()
    hip.record(e0, stream)
    for _ in range(steps):
        F.apply_batched(plans, rhos, outs, ws)
    hip.record(e1, stream)
    batch_ms = hip.ms(e0, e1) / steps
    # the same problems, one fsa_apply each (3 launches per problem)
    big = max(pl.workspace_bytes for pl in plans)
    ws1 = torch.empty(big + 256, dtype=torch.uint8, device="cuda")
    outs2 = [torch.empty_like(r) for r in rhos]
    for pl, r, o in zip(plans, rhos, outs2):
        pl.apply(r, o, ws1)
    torch.cuda.synchronize()
    hip.record(e0, stream)
    for _ in range(steps):
        for pl, r, o in zip(plans, rhos, outs2):
            pl.apply(r, o, ws1)
    hip.record(e1, stream)
    percall_ms = hip.ms(e0, e1) / steps
    # With its tuned choices a batch group may run another launch variant than
    # a problem's own plan (the group's size class differs), so the timed
    # results agree to rounding; under the same choices (all defaults) they
    # are bitwise equal.
    tuned_diff = max(float((a.double() - b.double()).norm() / b.double().norm())
                     for a, b in zip(outs, outs2))
    with tempfile.TemporaryDirectory() as td:
        saved = os.path.join(td, "table.json")
        F.tune_save(saved)
        F.tune_reset()
        F.apply_batched(plans, rhos, outs, ws)  # re-captured under the reset table
        for pl, r, o in zip(plans, rhos, outs2):
            pl.apply(r, o, ws1)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(outs, outs2))
        F.tune_load(saved)
    hip.destroy(e0)
    hip.destroy(e1)
    pts = sum(p.points for p in probs)
    mbytes = sum(sum(model_bytes(p.N, "f32").values()) for p in probs)
    for pl in plans:
        pl.close()
    return {
        "workload": f"{count} 2D log-kernel densities, grids from "
                    "{256^2, 512^2, 1024x256, 2048x512, 1024^2}, L_j in U[4,16], FP32",
        "grid_points": pts,
        "value": pts / (batch_ms * 1e-3),
        "unit": "grid pts/s",
        "ms_per_batch": batch_ms,
        "launches_in_graph": launches,
        "graph_capture_ms": capture_ms,
        "model_hbm_frac": mbytes / (batch_ms * 1e-3) / HBM_PEAK_BPS,
        "per_call_ms": percall_ms,
        "per_call_value": pts / (percall_ms * 1e-3),
        "tensor_build_ms_total": build_ms,
        "autotune_s": tune_s,
        "bitwise_equal_to_per_call_same_choices": same,
        "tuned_max_rel_l2_vs_per_call": tuned_diff,
    }


def bench_serve(F, torch, hip, synth, duration=3.0, rate=2000.0, budget=200 << 30,
                inflight=16, streams=4, per_call=True, fp64_fraction=0.05):
    """Served workload: seeded Poisson arrivals (mean `rate` req/s) of 3D
    Coulomb / Yukawa requests on {64^3, 128^3, 256^3, 512x64x64, 64x64x512}
    grids with 1-8 Gaussian densities, 5% FP64, tensors cached under an HBM
    budget (200 GiB by default).  Every latency is completion - scheduled
    arrival (time.monotonic, the server's clock), so any wait before a
    request is submitted counts.  The same arrival stream is replayed through
    the plain per-call path (one synchronous fsa_apply at a time, tensors
    cached): in FP64, in FP32, and in each request's own precision."""
    reqs = synth.serve_stream(seed=5000, rate=rate, duration=duration,
                              fp64_fraction=fp64_fraction)
    kinds = {}
    for _, p in reqs:
        kinds.setdefault((p.N, p.L, p.precision), p)
    dens = {}
    outs = {}
    for key, p in kinds.items():
        dt = F.DTYPES[p.precision]
        dens[key] = torch.from_numpy(synth.eval_gaussians(p.gaussians, p.L, p.N)).to(dt).cuda()
        pool = inflight + 8 if p.points <= 128 ** 3 else 12
        outs[key] = [[torch.empty_like(dens[key]), None] for _ in range(pool)]
    clock_offset_us = (F.Server.clock() - time.monotonic()) * 1e6
    srv = F.Server(budget, max_inflight=inflight, n_streams=streams)
    # warm the tensor cache: one request per distinct tensor key, untimed
    seen = set()
    for _, p in reqs:
        k = (p.kernel, p.lam, p.N, p.L, p.precision)
        if k in seen:
            continue
        seen.add(k)
        key = (p.N, p.L, p.precision)
        t = srv.submit(p.kernel, p.L, p.N, dens[key], outs[key][0][0], precision=p.precision,
                       lam=p.lam or None)
        srv.wait(t)
    srv.reset_stats()

    def take(key):
        # an output buffer no pending request writes (the wait counts in the
        # latency, which runs from the scheduled arrival)
        pool = outs[key]
        while True:
            for slot in pool:
                if slot[1] is None or srv.poll(slot[1])[0]:
                    return slot
            time.sleep(20e-6)

    t0 = time.monotonic()
    tickets = []
    late = 0
    for t_arr, p in reqs:
        while time.monotonic() - t0 < t_arr:
            pass
        if time.monotonic() - t0 > t_arr + 1e-3:
            late += 1
        key = (p.N, p.L, p.precision)
        slot = take(key)
        slot[1] = srv.submit(p.kernel, p.L, p.N, dens[key], slot[0], precision=p.precision,
                             lam=p.lam or None, arrival=t0 + t_arr)
        tickets.append(slot[1])
    bad = sum(srv.wait(t) != "FSA_OK" for t in tickets)
    st = srv.stats()
    srv.close()

    def per_call_path(prec_override):
        plans = {}
        ws = {}
        lat = []
        for _, p in reqs:  # build plans and time nothing yet
            prec = prec_override or p.precision
            k = (p.kernel, p.lam, p.N, p.L, prec)
            if k not in plans:
                plans[k] = F.Plan(p.kernel, p.L, p.N, prec, lam=p.lam or None).build()
                ws[k] = plans[k].workspace()
        inputs = {}
        for key, d in dens.items():
            for prec in ("f32", "f64"):
                inputs[(key[0], key[1], prec)] = d.to(F.DTYPES[prec])
        torch.cuda.synchronize()
        out_cache = {}
        t0 = time.monotonic()
        for t_arr, p in reqs:
            while time.monotonic() - t0 < t_arr:
                pass
            prec = prec_override or p.precision
            k = (p.kernel, p.lam, p.N, p.L, prec)
            x = inputs[(p.N, p.L, prec)]
            o = out_cache.setdefault((p.N, p.L, prec), torch.empty_like(x))
            plans[k].apply(x, o, ws[k])
            torch.cuda.synchronize()
            lat.append((time.monotonic() - t0 - t_arr) * 1e3)
        span = time.monotonic() - t0
        for pl in plans.values():
            pl.close()
        n = len(lat)
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "throughput_rps": n / span, "requests": n}

    fp64 = per_call_path("f64") if per_call else None
    fp32 = per_call_path("f32") if per_call else None
    mixed = per_call_path(None) if per_call else None
    pts = sum(p.points for _, p in reqs)
    return {
        "workload": f"Poisson arrivals at {rate:.0f} req/s for {duration:.1f} s (seed 5000): "
                    "3D Coulomb (1/2) / Yukawa lam in {0.5,1,4}; grids 64^3, 128^3, 256^3, "
                    f"512x64x64, 64x64x512; {100 * fp64_fraction:.0f}% FP64; "
                    f"HBM budget {budget / 2**30:.0f} GiB",
        "latency": "completion - scheduled arrival, every path",
        "requests": len(reqs),
        "grid_points": pts,
        "server": {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                   "throughput_rps": st["throughput_rps"], "gpts_per_s": st["gpts_per_s"],
                   "failed": bad, "late_submissions": late, "cache_hits": st["cache_hits"],
                   "cache_misses": st["cache_misses"], "hbm_peak_GB": st["hbm_peak"] / 1e9,
                   "max_inflight": inflight, "streams": streams,
                   "clock_offset_us": clock_offset_us},
        "per_call_fp64": fp64,
        "per_call_fp32": fp32,
        "per_call_requested_precision": mixed,
    }


def cpu_baseline(synth, prob, rho64, phis, aniso_phis):
    """The FP64 oracle on the host cores, on the whole timed workload: one
    evaluation of the 256^3 Yukawa problem (tensor build, then the FFT
    convolution; value = grid points / convolution time).  Its output is
    also the reference for the timed GPU outputs (`phis`, per precision)
    over every grid point, with a second oracle convolution of the density
    as the FP32 path received it (rounded to FP32); and the cigar / pancake
    and Yukawa outputs are checked against the exact potential (1-D integral
    or closed form) at 40 seeded points and the maximum."""
    from oracle import oracle as O
    from oracle import reference as Rf
    cores = O.set_threads(0)
    t0 = time.perf_counter()
    T = O.build_tensor(prob.kernel, prob.L, prob.N, prob.eps, lam=prob.lam)
    t1 = time.perf_counter()
    ref64 = O.conv_fft(T, rho64)
    t2 = time.perf_counter()
    pts = 1
    for n in prob.N:
        pts *= n
    out = {
        "value": pts / (t2 - t1),
        "unit": "grid pts/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"one FP64 oracle evaluation of the whole {prob.N[0]}^3 Yukawa workload; "
                  "value = grid points / FFT-convolution time; "
                  f"tensor build {t1 - t0:.2f} s, convolution {t2 - t1:.2f} s",
        "precomp_s": t1 - t0,
        "execution_s": t2 - t1,
        "cpu": platform.processor() or platform.machine(),
    }
    # thread scaling on a bounded sample (the 128^3 grid of the same workload
    # recipe): one evaluation on every host thread, then on one
    small = synth.yukawa_problem(prob.lam, 128, "f64")
    rho_s = synth.eval_gaussians(small.gaussians, small.L, small.N)
    by_threads = {}
    for nth in (cores, 1):
        O.set_threads(nth)
        ta = time.perf_counter()
        Ts = O.build_tensor(small.kernel, small.L, small.N, small.eps, lam=small.lam)
        tb = time.perf_counter()
        O.conv_fft(Ts, rho_s)
        tc = time.perf_counter()
        by_threads[str(nth)] = {"precomp_s": round(tb - ta, 3), "execution_s": round(tc - tb, 3),
                                "value": 128 ** 3 / (tc - tb)}
        del Ts
    O.set_threads(cores)
    out["threads"] = {"sample": "one FP64 oracle evaluation of the 128^3 grid of the same "
                                "Yukawa recipe (lam = 1, eps = 2, 8 Gaussians), on all host "
                                "threads and on one",
                      "unit": "grid pts/s", "by_threads": by_threads}
    parity = {"points": pts, "kind": "oracle convolution, every grid point"}
    for prec, phi in phis.items():
        ref = ref64 if prec == "f64" else O.conv_fft(T, rho64.astype(np.float32).astype(np.float64))
        d = phi - ref
        parity[prec] = {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                        "rel_max": float(np.abs(d).max() / np.abs(ref).max())}
        del ref, d
    del T, ref64
    parity["aniso"] = {}
    for key, (p, phi) in (aniso_phis or {}).items():
        rng = np.random.default_rng(1)
        idx = np.unique(np.append(rng.choice(phi.size, 40, replace=False),
                                  int(np.argmax(np.abs(phi)))))
        gs = [(g.amp, g.center, g.width) for g in p.gaussians]
        ex = Rf.gaussian_sum_potential(p.kernel, gs, p.L, p.N, lam=p.lam, points=idx)
        parity["aniso"][key] = float(np.abs(phi.ravel()[idx] - ex).max() / np.abs(ex).max())
    return out, parity


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--n", type=int, default=256, help="grid points per axis")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 2D workload")
    ap.add_argument("--batch-only", action="store_true", help="only the batched 2D workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the served workload")
    ap.add_argument("--no-ddi", action="store_true", help="skip the dipole-dipole timing")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the general-construction timings")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the cigar/pancake, Yukawa-over-lambda and Table 3 workloads")
    ap.add_argument("--serve-only", action="store_true", help="only the served workload")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (every pass at its default launch variant)")
    ap.add_argument("--tune-file", default=None,
                    help="load this saved tuning table instead of autotuning")
    ap.add_argument("--retune", action="store_true",
                    help="autotune in this run instead of loading the shipped table")
    ap.add_argument("--save-tune", default=None,
                    help="save the tuning table to this path at the end")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: this library runs on exactly one GPU (asked for {args.gpus}); "
              "sharding the path over several GPUs is a design, not implemented", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2504_19410_amd import fsa as F
    from paper_2504_19410_amd import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    # launch choices: the table fsa_autotune wrote for this GPU type and ships
    # with the package (paper_2504_19410_amd/tune/<arch>.json), unless asked
    # to retune here, to load another table, or to run untuned
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    shipped = os.path.join(ROOT, "paper_2504_19410_amd", "tune", f"{arch}.json")
    if args.tune_file is None and not args.retune and not args.no_tune and os.path.exists(shipped):
        args.tune_file = shipped
    if args.tune_file:
        F.tune_load(args.tune_file)
        args.no_tune = True
        tuning = f"table loaded from {os.path.relpath(args.tune_file, ROOT)} (written by fsa_autotune)"
    elif args.no_tune:
        tuning = "untuned: every pass at variant 0, full occupancy"
    else:
        tuning = "fsa_autotune in this run (untimed, before warm-up)"
    hip = Hip()
    copy_bps = stream_copy(torch, hip)
    log(f"stream copy (1 GiB): {copy_bps / 1e9:.0f} GB/s")
    if args.copy_only:
        return
    if args.serve_only:
        sv = bench_serve(F, torch, hip, synth, duration=args.serve_seconds)
        sv["server_one_stream"] = bench_serve(F, torch, hip, synth, duration=args.serve_seconds,
                                              inflight=4, streams=1, per_call=False)["server"]
        # the same arrivals with every request in FP32: the server beside
        # per_call_fp32, which runs exactly these requests
        sv["server_all_fp32"] = bench_serve(F, torch, hip, synth, duration=args.serve_seconds,
                                            per_call=False, fp64_fraction=0.0)["server"]
        log(f"  serve: {json.dumps(sv)}")
        burst = bench_serve(F, torch, hip, synth, duration=1.0, rate=6000.0, budget=2 << 30)
        log(f"  burst: {json.dumps(burst)}")
        print(json.dumps({"serve": sv, "serve_burst": burst}), flush=True)
        return
    if args.batch_only:
        b = bench_batch(F, torch, hip, synth, max(3, args.steps // 2), 2, tune=not args.no_tune)
        log(f"  batch: {b['ms_per_batch']:.3f} ms ({b['value'] / 1e9:.2f} Gpts/s) in "
            f"{b['launches_in_graph']} launches; per-call {b['per_call_ms']:.3f} ms")
        print(json.dumps({"batch": b}), flush=True)
        return
    prob = synth.yukawa_problem(1.0, args.n, "f32")
    log(f"density: {len(prob.gaussians)} Gaussians on {prob.N} ...")
    rho64 = synth.eval_gaussians(prob.gaussians, prob.L, prob.N)
    res = {}
    phis = {}
    for prec in ("f32", "f64"):
        log(f"bench {prec}: {args.warmup} warmup + {args.steps} timed evaluations")
        res[prec], phis[prec] = bench_precision(F, torch, hip, prob, rho64, prec, args.steps,
                                                args.warmup, tune=not args.no_tune)
        log(f"  {prec}: {res[prec]['ms_per_step']:.4f} ms/eval, "
            f"{res[prec]['value'] / 1e9:.2f} Gpts/s, passes {res[prec]['pass_ms']}")
    diff = float(np.linalg.norm(phis["f32"] - phis["f64"]) / np.linalg.norm(phis["f64"]))
    if args.no_cpu:
        del phis
    sweep = precomp_sweep(F, torch, hip, n=args.n)
    log(f"  precomp vs anisotropy (ms): {sweep['ms_by_anisotropy']}")
    conv_vars = bench_conv_variants(F, torch, hip, prob, rho64, args.tune_file)
    log(f"  pass C by variant: {json.dumps(conv_vars)}")
    ddi = None
    if not args.no_ddi:
        ddi = bench_ddi(F, torch, hip, synth, n=args.n)
        log(f"  dipole-dipole: FP32 {ddi['f32']['ms_per_step']:.4f} ms, "
            f"FP64 {ddi['f64']['ms_per_step']:.4f} ms")
    table3 = aniso = yuk = aniso_phis = None
    if not args.no_extra:
        table3 = bench_table3(F, torch, hip, synth)
        log(f"  Table 3 workload (192^3): {table3}")
        aniso, aniso_phis = bench_aniso(F, torch, hip, synth)
        log(f"  cigar / pancake: {aniso}")
        yuk, yuk_phis = bench_yukawa_lambda(F, torch, hip, synth)
        log(f"  Yukawa over lambda: {yuk}")
        aniso_phis.update({("yukawa",) + k: v for k, v in yuk_phis.items()})
        del yuk_phis
        if args.no_cpu:
            aniso_phis = None  # only the oracle leg reads them
    general = None
    if not args.no_general:
        general = bench_general(F, torch, hip, n=args.n)
        log(f"  general construction: {general}")
    dd = None
    if not args.no_general:
        dd = bench_dd(F, torch, hip, synth)
        log(f"  double-double 128^3: build {dd['precomp_ms']} ms, {dd['ms_per_step']} ms/eval")
    batch = None
    if not args.no_batch:
        log("batched 2D log workload (256 densities) ...")
        batch = bench_batch(F, torch, hip, synth, max(3, args.steps // 2), 2,
                            tune=not args.no_tune)
        log(f"  batch: {batch['ms_per_batch']:.3f} ms ({batch['value'] / 1e9:.2f} Gpts/s) in "
            f"{batch['launches_in_graph']} launches; per-call {batch['per_call_ms']:.3f} ms")
    serve = serve_burst = None
    if not args.no_serve:
        log("served workload (Poisson arrivals) ...")
        serve = bench_serve(F, torch, hip, synth, duration=args.serve_seconds)
        serve["server_one_stream"] = bench_serve(F, torch, hip, synth,
                                                 duration=args.serve_seconds, inflight=4,
                                                 streams=1, per_call=False)["server"]
        # the same arrivals with every request in FP32: the server beside
        # per_call_fp32, which runs exactly these requests
        serve["server_all_fp32"] = bench_serve(F, torch, hip, synth,
                                               duration=args.serve_seconds,
                                               per_call=False, fp64_fraction=0.0)["server"]
        log(f"  server p50/p99 {serve['server']['p50_ms']:.3f}/{serve['server']['p99_ms']:.3f} ms, "
            f"per-call FP64 p50/p99 {serve['per_call_fp64']['p50_ms']:.3f}/"
            f"{serve['per_call_fp64']['p99_ms']:.3f} ms")
        log("burst: 6000 req/s for 1 s under a 2 GB HBM budget ...")
        serve_burst = bench_serve(F, torch, hip, synth, duration=1.0, rate=6000.0,
                                  budget=2 << 30)
        log(f"  burst server p50/p99 {serve_burst['server']['p50_ms']:.3f}/"
            f"{serve_burst['server']['p99_ms']:.3f} ms")
    cpu = parity = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu, parity = cpu_baseline(synth, prob, rho64, phis, aniso_phis)
        for key, e in parity.pop("aniso").items():
            if key[0] == "yukawa":
                _, n, lam, prec = key
                yuk.setdefault("rel_max_err_vs_exact", {})[f"{n}_{prec}_lam{lam:g}"] = e
            else:
                orient, gamma, prec = key
                aniso[orient].setdefault("rel_max_err_vs_exact", {})[f"{prec}_gamma{gamma:g}"] = e
        del phis
        log(f"  oracle: {cpu['value'] / 1e6:.3f} Mpts/s on {cpu['cores']} threads")
        log(f"  timed outputs against the oracle: {parity}")
    r32, r64 = res["f32"], res["f64"]

    def leg(r):
        return {"value": r["value"], "ms_per_step": r["ms_per_step"],
                "mean_ms_per_step": r["mean_ms_per_step"], "first_ms": r["first_ms"],
                "wall_ms_per_step": r["wall_ms_per_step"], "roofline": r["roofline"],
                "pass_ms": r["pass_ms"], "model_bytes_per_step": r["model_bytes_per_step"],
                "model_hbm_frac": r["model_hbm_frac"],
                "model_copy_frac": r["model_bytes_per_step"] / (r["ms_per_step"] * 1e-3) / copy_bps,
                "precomp_ms": r["precomp_ms"], "precomp": r["precomp"], "tuned": r["tuned"]}

    line = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Yukawa lam=1 eps=2 on [-8,8]^3, {args.n}^3 grid, 8 seeded "
                        "Gaussians (widths U[0.5,1.5]); FP64 FFT convolution with an FP64 tensor "
                        "built on the GPU by the closed-form Gaussian-screened split",
            "grid": list(prob.N),
            "kernel": "yukawa3d",
            "construction": "closed-form Gaussian-screened split",
        },
        "timing": f"ms_per_step = median of {args.steps} evaluations, each between its own "
                  f"hipEvent pair, after >= {SETTLE_S:g} s of untimed evaluations and "
                  f"{args.warmup} warm-up evaluations; mean_ms_per_step = the events' span / "
                  "steps",
        "mean_ms_per_step": r64["mean_ms_per_step"],
        "first_ms": r64["first_ms"],
        "roofline": r64["roofline"],
        "cpu_baseline": cpu,
        "oracle_parity": parity,
        "fp32": leg(r32),
        "pass_ms": r64["pass_ms"],
        "tuned": r64["tuned"],
        "tuning": tuning,
        "model_bytes_per_step": r64["model_bytes_per_step"],
        "model_hbm_frac": r64["model_hbm_frac"],
        "precomp_ms": r64["precomp_ms"],
        "precomp": r64["precomp"],
        "precomp_vs_anisotropy": sweep,
        "pass_c_variants": conv_vars,
        "ddi": ddi,
        "general": general,
        "double_double": dd,
        "wall_ms_per_step": r64["wall_ms_per_step"],
        "f32_vs_f64_rel_l2": diff,
        "batch": batch,
        "serve": serve,
        "serve_burst": serve_burst,
        "stream_copy_GBps": copy_bps / 1e9,
        "model_copy_frac": r64["model_bytes_per_step"] / (r64["ms_per_step"] * 1e-3) / copy_bps,
        "kernel_source_hash": kernel_source_hash(),
        "paper_context": "FSA Execution 2.24 s / Precomp 2.84 s at 192^3 in FP64, FORTRAN on one "
                         "Xeon Gold 6248R 3.0 GHz (Table 3); other hardware, context only",
        "table3_workload": table3,
        "cigar_pancake": aniso,
        "yukawa_lambda": yuk,
    }
    if args.save_tune:
        F.tune_save(args.save_tune)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
