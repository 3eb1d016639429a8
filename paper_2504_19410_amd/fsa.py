"""Python binding of the C ABI in ``include/fsa.h`` (argument marshalling only).

Every step of an evaluation runs in the HIP kernels of ``libfsa.so``; PyTorch
only provides device memory and the current stream.  Importing this module
fails loudly if the library has not been built.

    plan = Plan("coulomb3d", L=(8, 8, 8), N=(32, 32, 32), precision="f64").build()
    phi = plan.apply(rho)          # rho: contiguous cuda tensor of shape N
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfsa.so")

KINDS = {
    "coulomb3d": 1,
    "yukawa3d": 2,
    "log2d": 3,
    "coulomb2d": 4,
    "biharmonic3d": 5,
    "biharmonic2d": 6,
    "ddi3d": 7,
    "yukawa2d": 8,
    "quasi2d_ddi": 9,
}
KIND_DIM = {"coulomb3d": 3, "yukawa3d": 3, "biharmonic3d": 3,
            "log2d": 2, "coulomb2d": 2, "biharmonic2d": 2, "ddi3d": 3,
            "yukawa2d": 2, "quasi2d_ddi": 2}
# "dd": double-double, each real an interleaved (hi, lo) pair of float64, so
# rho / phi tensors have shape N + (2,)
PRECISIONS = {"f32": 0, "f64": 1, "dd": 2}
# compiled launch variants of the pass kernels (fsa_tune_variants bit mask)
NUM_VARIANTS = 5
DTYPES = {"f32": torch.float32, "f64": torch.float64, "dd": torch.float64}

# FSA_NOALLOC_SCRATCH_BYTES: the workspace capacity of fsa_apply_noalloc
NOALLOC_SCRATCH_BYTES = 128 << 20

STATUS = {
    0: "FSA_OK", 1: "FSA_EINVAL", 2: "FSA_EUNSUPPORTED", 3: "FSA_ENOMEM",
    4: "FSA_EDEVICE", 5: "FSA_ESTATE", 6: "FSA_EBUDGET", 7: "FSA_ECANCELLED",
    8: "FSA_ETIMEDOUT",
}

EXPORTS = (
    "fsa_plan_create", "fsa_plan_query", "fsa_build_tensor", "fsa_apply", "fsa_apply_events",
    "fsa_apply_noalloc",
    "fsa_batch_workspace_bytes", "fsa_apply_batched", "fsa_batch_launches",
    "fsa_autotune_batched", "fsa_plan_destroy",
    "fsa_plan_tensor",
    "fsa_server_create", "fsa_server_submit", "fsa_server_submit_at", "fsa_server_clock",
    "fsa_server_poll", "fsa_server_wait", "fsa_server_wait_for",
    "fsa_server_cancel", "fsa_server_set_queue_timeout", "fsa_server_stats",
    "fsa_server_reset_stats", "fsa_server_destroy",
    "fsa_plan_launches",
    "fsa_autotune", "fsa_tune_set", "fsa_tune_get", "fsa_tune_variants", "fsa_tune_save",
    "fsa_tune_load", "fsa_tune_reset", "fsa_tune_set_slabs", "fsa_tune_get_slabs",
    "fsa_last_error",
)

# fsa_pass: the passes of one evaluation, in execution order for 3D
PASSES = {"r2c": 0, "fwd_t": 1, "conv": 2, "inv_t": 3, "c2r": 4}
LAUNCH_KINDS = dict(PASSES, spectral=5)


class FsaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("lambda_", ctypes.c_double), ("eps", ctypes.c_double),
                ("n", ctypes.c_double * 3), ("m", ctypes.c_double * 3),
                ("eta", ctypes.c_double), ("general", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("throughput_rps", ctypes.c_double), ("gpts_per_s", ctypes.c_double),
                ("done", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("cache_hits", ctypes.c_uint64),
                ("cache_misses", ctypes.c_uint64), ("hbm_in_use", ctypes.c_size_t),
                ("hbm_peak", ctypes.c_size_t), ("timed_out", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} is not built; run `python -m paper_2504_19410_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    S = ctypes.c_size_t
    sigs = {
        "fsa_plan_create": [ctypes.POINTER(_Kernel), I, P, P, I, ctypes.POINTER(P)],
        "fsa_plan_query": [P, P, P, P, P],
        "fsa_build_tensor": [P, P],
        "fsa_apply": [P, P, P, P, P],
        "fsa_apply_events": [P, P, P, P, P, P, I],
        "fsa_apply_noalloc": [P, P, P, P],
        "fsa_batch_workspace_bytes": [I, P, P],
        "fsa_apply_batched": [I, P, P, P, P, S, P],
        "fsa_batch_launches": [I, P, P, P, P, P],
        "fsa_plan_destroy": [P],
        "fsa_plan_tensor": [P, P, P],
        "fsa_server_create": [S, I, I, ctypes.POINTER(P)],
        "fsa_server_submit": [P, ctypes.POINTER(_Kernel), I, P, P, I, P, P, P],
        "fsa_server_submit_at": [P, ctypes.POINTER(_Kernel), I, P, P, I, P, P, ctypes.c_double,
                                 P],
        "fsa_server_clock": [P],
        "fsa_server_poll": [P, ctypes.c_uint64, P, P],
        "fsa_server_wait": [P, ctypes.c_uint64, P],
        "fsa_server_wait_for": [P, ctypes.c_uint64, ctypes.c_double, P, P],
        "fsa_server_cancel": [P, ctypes.c_uint64],
        "fsa_server_set_queue_timeout": [P, ctypes.c_double],
        "fsa_server_stats": [P, ctypes.POINTER(Stats)],
        "fsa_server_reset_stats": [P],
        "fsa_server_destroy": [P],
        "fsa_autotune": [P, P, P, P, P, I],
        "fsa_autotune_batched": [I, P, P, P, P, S, P, I],
        "fsa_tune_set": [I, I, I, ctypes.c_int64, I, I],
        "fsa_tune_get": [I, I, I, ctypes.c_int64, P, P, P],
        "fsa_tune_variants": [I, I, I, P],
        "fsa_tune_save": [ctypes.c_char_p],
        "fsa_tune_load": [ctypes.c_char_p],
        "fsa_tune_reset": [],
        "fsa_tune_set_slabs": [I, P, I],
        "fsa_tune_get_slabs": [I, P, P, P],
        "fsa_plan_launches": [P, P, P, I],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.fsa_last_error.argtypes = []
    lib.fsa_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status: int):
    if status != 0:
        raise FsaError(status, _lib.fsa_last_error().decode(errors="replace"))


def _stream_ptr(stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _kernel(kind: str, eps: Optional[float], lam: Optional[float], n=None, m=None,
            eta: Optional[float] = None, general: bool = False) -> _Kernel:
    if kind not in KINDS:
        raise ValueError(f"unknown kernel {kind!r}; choose from {sorted(KINDS)}")
    k = _Kernel(KINDS[kind], float(lam or 0.0), float(eps) if eps else 0.0)
    for j, v in enumerate(n if n is not None else (0.0, 0.0, 0.0)):
        k.n[j] = float(v)
    for j, v in enumerate(m if m is not None else (0.0, 0.0, 0.0)):
        k.m[j] = float(v)
    k.eta = float(eta or 0.0)
    k.general = 1 if general else 0
    return k


class Plan:
    """A plan for one kernel, box and grid (``fsa_plan_create``)."""

    def __init__(self, kernel: str, L: Sequence[float], N: Sequence[int], precision: str = "f32",
                 eps: Optional[float] = None, lam: Optional[float] = None,
                 n: Optional[Sequence[float]] = None, m: Optional[Sequence[float]] = None,
                 eta: Optional[float] = None, general: bool = False):
        """n, m: dipole orientations of the "ddi3d" kernel, n of "quasi2d_ddi"
        (ignored otherwise); eta: confinement width of "quasi2d_ddi";
        general: the general construction (window + quadrature W) for the
        kernels that also have a closed-form one ("yukawa2d" and
        "quasi2d_ddi" always use it)."""
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        self.kernel, self.precision = kernel, precision
        self.L = tuple(float(x) for x in L)
        self.N = tuple(int(n) for n in N)
        self.lam = lam
        self.d = len(self.N)
        if len(self.L) != self.d:
            raise ValueError("L and N must have the same length")
        k = _kernel(kernel, eps, lam, n, m, eta, general)
        self.general = bool(general) or kernel in ("yukawa2d", "quasi2d_ddi")
        Ls = (ctypes.c_double * self.d)(*self.L)
        Ns = (ctypes.c_int64 * self.d)(*self.N)
        h = ctypes.c_void_p()
        _check(_lib.fsa_plan_create(ctypes.byref(k), self.d, Ls, Ns, PRECISIONS[precision],
                                    ctypes.byref(h)))
        self._h = h
        e = ctypes.c_double()
        hs = (ctypes.c_double * self.d)()
        tb = ctypes.c_size_t()
        wb = ctypes.c_size_t()
        _check(_lib.fsa_plan_query(h, ctypes.byref(e), hs, ctypes.byref(tb), ctypes.byref(wb)))
        self.eps = e.value
        self.h = tuple(hs)
        self.tensor_bytes = tb.value
        self.workspace_bytes = wb.value
        self.dtype = DTYPES[precision]
        self._ws = None
        self.device = None

    @property
    def handle(self):
        return self._h

    def build(self, stream: Optional[torch.cuda.Stream] = None) -> "Plan":
        _check(_lib.fsa_build_tensor(self._h, _stream_ptr(stream)))
        self.device = torch.cuda.current_device()
        return self

    def workspace(self) -> torch.Tensor:
        """A workspace owned by this Python object (allocated once)."""
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                   device=f"cuda:{torch.cuda.current_device()}")
        return self._ws

    def _ws_ptr(self, ws: torch.Tensor) -> int:
        p = ws.data_ptr()
        return (p + 255) & ~255

    @property
    def shape(self):
        """Shape of rho and phi: N, or N + (2,) for double-double pairs."""
        return self.N + ((2,) if self.precision == "dd" else ())

    def check_input(self, rho: torch.Tensor):
        if not rho.is_cuda:
            raise ValueError("rho must be a device tensor")
        if tuple(rho.shape) != self.shape:
            raise ValueError(f"rho shape {tuple(rho.shape)} != plan grid {self.shape}")
        if rho.dtype != self.dtype:
            raise ValueError(f"rho dtype {rho.dtype} != plan precision {self.dtype}")
        if not rho.is_contiguous():
            raise ValueError("rho must be contiguous")

    def apply(self, rho: torch.Tensor, out: Optional[torch.Tensor] = None,
              workspace: Optional[torch.Tensor] = None,
              stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """phi = U * rho on the grid (``fsa_apply``); out may alias rho."""
        self.check_input(rho)
        if out is None:
            out = torch.empty_like(rho)
        else:
            self.check_input(out)
        ws = workspace if workspace is not None else self.workspace()
        if ws.numel() < self.workspace_bytes + 256:
            raise ValueError("workspace too small")
        _check(_lib.fsa_apply(self._h, ctypes.c_void_p(rho.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(self._ws_ptr(ws)),
                              _stream_ptr(stream)))
        return out

    def apply_noalloc(self, rho: torch.Tensor, out: Optional[torch.Tensor] = None,
                      stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """``fsa_apply_noalloc``: as apply, with the library's static device
        scratch as the workspace (no allocation when ``out`` is given)."""
        self.check_input(rho)
        if out is None:
            out = torch.empty_like(rho)
        else:
            self.check_input(out)
        _check(_lib.fsa_apply_noalloc(self._h, ctypes.c_void_p(rho.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    @property
    def n_passes(self) -> int:
        return 5 if self.d == 3 else 3

    def launches(self):
        """Pass name of every kernel launch of one evaluation, in order (the
        3D middle passes repeat once per slab of the tuned schedule)."""
        n = ctypes.c_int()
        _check(_lib.fsa_plan_launches(self._h, ctypes.byref(n), None, 0))
        arr = (ctypes.c_int * n.value)()
        _check(_lib.fsa_plan_launches(self._h, ctypes.byref(n), arr, n.value))
        names = {v: k for k, v in LAUNCH_KINDS.items()}
        return [names[a] for a in arr]

    def passes(self):
        """(pass name, transform length) of each pass, in execution order."""
        N = self.N
        if self.d == 3:
            return [("r2c", N[2]), ("fwd_t", 2 * N[1]), ("conv", 2 * N[0]),
                    ("inv_t", 2 * N[1]), ("c2r", N[2])]
        return [("r2c", N[1]), ("conv", 2 * N[0]), ("c2r", N[1])]

    def pass_lines(self):
        """Transforms one whole-grid launch of each pass runs (the size the
        tuning table is keyed by), in execution order."""
        N = self.N
        if self.d == 3:
            H = N[2] + 1
            return [N[0] * N[1], N[0] * H, H * 2 * N[1], N[0] * H, N[0] * N[1]]
        return [N[0], N[1] + 1, N[0]]

    def tuned(self):
        """{(pass, length): (variant, occupancy, us)} in force for this plan."""
        return {(name, n): tune_get(self.precision, name, n, lines)
                for (name, n), lines in zip(self.passes(), self.pass_lines())}

    def autotune(self, rho: Optional[torch.Tensor] = None, reps: int = 10,
                 stream: Optional[torch.cuda.Stream] = None) -> dict:
        """Times every launch variant of every pass (``fsa_autotune``) and
        returns the chosen {(pass, length): (variant, occupancy, us)}."""
        if rho is None:
            rho = torch.rand(self.shape, dtype=self.dtype, device="cuda")
        self.check_input(rho)
        out = torch.empty_like(rho)
        ws = self.workspace()
        _check(_lib.fsa_autotune(self._h, ctypes.c_void_p(rho.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(self._ws_ptr(ws)), _stream_ptr(stream),
                                 int(reps)))
        out = self.tuned()
        if self.d == 3:
            out[("slabs", 0)] = tune_get_slabs(self.precision, self.N)
        return out

    def apply_events(self, rho: torch.Tensor, out: torch.Tensor, events,
                     workspace: Optional[torch.Tensor] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """fsa_apply with caller-created hipEvent_t handles, two per launch,
        recorded right before and right after each launch (None, None: that
        launch untimed)."""
        self.check_input(rho)
        self.check_input(out)
        ws = workspace if workspace is not None else self.workspace()
        arr = (ctypes.c_void_p * len(events))(*events)
        _check(_lib.fsa_apply_events(self._h, ctypes.c_void_p(rho.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(self._ws_ptr(ws)), _stream_ptr(stream), arr,
                                     len(events)))
        return out

    def tensor(self) -> torch.Tensor:
        """Copy of the built spectral octant, shape (N_{d-1}+1, ..., N_0+1)."""
        ptr = ctypes.c_void_p()
        dims = (ctypes.c_int64 * self.d)()
        _check(_lib.fsa_plan_tensor(self._h, ctypes.byref(ptr), dims))
        shape = tuple(dims) + ((2,) if self.precision == "dd" else ())
        n = 1
        for s in shape:
            n *= s
        out = torch.empty(shape, dtype=self.dtype)
        torch.cuda.synchronize()
        hip = _hip()
        rc = hip.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ptr,
                           ctypes.c_size_t(n * out.element_size()), 2)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_int]
        _hip_lib.hipMemcpy.restype = ctypes.c_int
    return _hip_lib


PASS_BATCHED = 16  # FSA_PASS_BATCHED


def _tune_pass(pass_name: str) -> int:
    """fsa_pass of a pass name; "batched_<pass>" names the entries of the
    batched launches (FSA_PASS_BATCHED)."""
    if pass_name.startswith("batched_"):
        return PASSES[pass_name[len("batched_"):]] | PASS_BATCHED
    return PASSES[pass_name]


def tune_get(precision: str, pass_name: str, length: int, lines: int = 1):
    """(variant, occupancy, us) a launch of `lines` transforms would use."""
    v, o, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(_lib.fsa_tune_get(PRECISIONS[precision], _tune_pass(pass_name), int(length),
                             int(lines), ctypes.byref(v), ctypes.byref(o), ctypes.byref(us)))
    return v.value, o.value, us.value


def tune_set(precision: str, pass_name: str, length: int, variant: int, occupancy: int = 0,
             lines: int = 1):
    _check(_lib.fsa_tune_set(PRECISIONS[precision], _tune_pass(pass_name), int(length),
                             int(lines), int(variant), int(occupancy)))


def tune_variants(precision: str, pass_name: str, length: int):
    """Variants compiled (distinct) at this pass and length."""
    m = ctypes.c_int()
    _check(_lib.fsa_tune_variants(PRECISIONS[precision], _tune_pass(pass_name), int(length),
                                  ctypes.byref(m)))
    return [v for v in range(NUM_VARIANTS) if m.value >> v & 1]


def tune_set_slabs(precision: str, N, slabs: int):
    arr = (ctypes.c_int64 * 3)(*N)
    _check(_lib.fsa_tune_set_slabs(PRECISIONS[precision], arr, int(slabs)))


def tune_get_slabs(precision: str, N):
    """(slabs, us) of the schedule of a 3D grid."""
    arr = (ctypes.c_int64 * 3)(*N)
    sl, us = ctypes.c_int(), ctypes.c_double()
    _check(_lib.fsa_tune_get_slabs(PRECISIONS[precision], arr, ctypes.byref(sl), ctypes.byref(us)))
    return sl.value, us.value


def tune_save(path: str):
    _check(_lib.fsa_tune_save(os.fsencode(path)))


def tune_load(path: str):
    _check(_lib.fsa_tune_load(os.fsencode(path)))


def tune_reset():
    _check(_lib.fsa_tune_reset())


def batch_workspace_bytes(plans: Sequence[Plan]) -> int:
    arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    b = ctypes.c_size_t()
    _check(_lib.fsa_batch_workspace_bytes(len(plans), arr, ctypes.byref(b)))
    return b.value


def apply_batched(plans: Sequence[Plan], rhos: Sequence[torch.Tensor],
                  outs: Optional[Sequence[torch.Tensor]] = None,
                  workspace: Optional[torch.Tensor] = None,
                  stream: Optional[torch.cuda.Stream] = None):
    """Evaluates every (plan, rho) pair in one batched call (``fsa_apply_batched``)."""
    n, outs, workspace = _batch_args(plans, rhos, outs, workspace)
    base = (workspace.data_ptr() + 255) & ~255
    arr = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(_lib.fsa_apply_batched(n, arr, rp, op, ctypes.c_void_p(base),
                                  ctypes.c_size_t(workspace.numel() - (base - workspace.data_ptr())),
                                  _stream_ptr(stream)))
    return outs


def _batch_args(plans, rhos, outs, workspace):
    """Host-side checks of a batch's buffers (the C ABI cannot size-check
    device pointers): one density and one output per plan, each of the plan's
    shape, dtype and layout on the device; outputs allocated if not given; a
    workspace of at least fsa_batch_workspace_bytes after 256-byte alignment."""
    n = len(plans)
    if len(rhos) != n:
        raise ValueError("one density per plan")
    if outs is not None and len(outs) != n:
        raise ValueError("one output per plan")
    for p, r in zip(plans, rhos):
        p.check_input(r)
    if outs is None:
        outs = [torch.empty_like(r) for r in rhos]
    else:
        for p, o in zip(plans, outs):
            p.check_input(o)
    need = batch_workspace_bytes(plans)
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=rhos[0].device)
    elif not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("the workspace must be a contiguous device tensor")
    return n, outs, workspace


def autotune_batched(plans: Sequence[Plan], rhos: Sequence[torch.Tensor],
                     outs: Optional[Sequence[torch.Tensor]] = None,
                     workspace: Optional[torch.Tensor] = None, reps: int = 5,
                     stream: Optional[torch.cuda.Stream] = None):
    """Tunes the persistent launches of this batch at their own size classes
    (``fsa_autotune_batched``); returns the outputs, which hold a valid
    evaluation under the tuned choices."""
    n, outs, workspace = _batch_args(plans, rhos, outs, workspace)
    base = (workspace.data_ptr() + 255) & ~255
    arr = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(_lib.fsa_autotune_batched(
        n, arr, rp, op, ctypes.c_void_p(base),
        ctypes.c_size_t(workspace.numel() - (base - workspace.data_ptr())), _stream_ptr(stream),
        int(reps)))
    return outs


def batch_launches(plans: Sequence[Plan], rhos, outs, workspace: torch.Tensor) -> int:
    """Persistent launches in the graph captured for this batch (fsa_batch_launches)."""
    n, outs, workspace = _batch_args(plans, rhos, outs, workspace)
    base = (workspace.data_ptr() + 255) & ~255
    arr = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    k = ctypes.c_int()
    _check(_lib.fsa_batch_launches(n, arr, rp, op, ctypes.c_void_p(base), ctypes.byref(k)))
    return k.value


class Server:
    """Continuous-batching convolution server on the current device
    (``fsa_server_*``): requests are admitted as slots and HBM budget free up
    and run concurrently; kernel tensors are cached per (kernel, box, grid,
    precision)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 16, n_streams: int = 4):
        h = ctypes.c_void_p()
        _check(_lib.fsa_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), int(max_inflight),
                                      int(n_streams), ctypes.byref(h)))
        self._h = h

    def submit(self, kernel: str, L: Sequence[float], N: Sequence[int], rho: torch.Tensor,
               phi: torch.Tensor, precision: str = "f32", eps: Optional[float] = None,
               lam: Optional[float] = None, general: bool = False,
               arrival: Optional[float] = None) -> int:
        """Queues phi = U * rho; returns a ticket.  rho and phi must stay alive
        (and phi untouched) until the ticket completes.  arrival: when the
        request arose, in seconds of time.monotonic() (fsa_server_clock);
        latency is counted from it (default: now)."""
        d = len(N)
        if tuple(rho.shape) != tuple(N) or tuple(phi.shape) != tuple(N):
            raise ValueError("rho/phi shape must equal N")
        if rho.dtype != DTYPES[precision] or phi.dtype != DTYPES[precision]:
            raise ValueError("rho/phi dtype must match the precision")
        if not (rho.is_cuda and phi.is_cuda and rho.is_contiguous() and phi.is_contiguous()):
            raise ValueError("rho/phi must be contiguous device tensors")
        k = _kernel(kernel, eps, lam, general=general)
        Ls = (ctypes.c_double * d)(*[float(x) for x in L])
        Ns = (ctypes.c_int64 * d)(*[int(n) for n in N])
        t = ctypes.c_uint64()
        _check(_lib.fsa_server_submit_at(self._h, ctypes.byref(k), d, Ls, Ns,
                                         PRECISIONS[precision], ctypes.c_void_p(rho.data_ptr()),
                                         ctypes.c_void_p(phi.data_ptr()),
                                         -1.0 if arrival is None else float(arrival),
                                         ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int()
        st = ctypes.c_int()
        _check(_lib.fsa_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done),
                                    ctypes.byref(st)))
        return bool(done.value), (STATUS[st.value] if done.value else None)

    def wait(self, ticket: int, timeout_ms: Optional[float] = None) -> Optional[str]:
        """Status name once the request finished; None if timeout_ms ran out."""
        st = ctypes.c_int()
        if timeout_ms is None:
            _check(_lib.fsa_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(st)))
            return STATUS[st.value]
        done = ctypes.c_int()
        _check(_lib.fsa_server_wait_for(self._h, ctypes.c_uint64(ticket), float(timeout_ms),
                                        ctypes.byref(done), ctypes.byref(st)))
        return STATUS[st.value] if done.value else None

    @staticmethod
    def clock() -> float:
        """The server clock (seconds; the clock of time.monotonic)."""
        t = ctypes.c_double()
        _check(_lib.fsa_server_clock(ctypes.byref(t)))
        return t.value

    def cancel(self, ticket: int):
        _check(_lib.fsa_server_cancel(self._h, ctypes.c_uint64(ticket)))

    def set_queue_timeout(self, timeout_ms: float):
        """Queued requests older than timeout_ms (from arrival) finish with
        FSA_ETIMEDOUT instead of launching; 0 turns the limit off."""
        _check(_lib.fsa_server_set_queue_timeout(self._h, float(timeout_ms)))

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.fsa_server_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        _check(_lib.fsa_server_reset_stats(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsa_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
