"""ctypes binding of the FP64 CPU oracle (``fsa_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is shared with the GPU
library; arrays come in and go out as numpy float64.

The oracle computes the paper's discretisation step by step (Liu & Zhang,
arXiv 2504.19410):

* ``build_tensor``: T = T(1) + T(2), Sec. 2.1 eq. Tensor1 / TensorAnis,
  Sec. 2.2 eqs. FouTran and Tensor2, on the full periodic grid prod_j 2N_j;
* ``conv_direct`` / ``conv_fft`` / ``conv_direct_points``: eq. DiscConv;
* ``ueps`` / ``what`` / ``u``: Table 1 and eqs. KerAppr, lnrAppr;
* ``ueps_general`` / ``what_general``: the general construction of Sec. 4
  (eq. GeneralApprox1, W by quadrature of eq. Fourier-Symmetric), with its
  own K0 (``k0``, ``k0e``) and J0 (``j0``);
* ``solve_ddi`` / ``solve_q2d``: the 3D and quasi-2D dipole-dipole
  potentials of Sec. 5.3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC_Q = os.path.join(_HERE, "fsa_oracle_q.c")
_LIB_Q = os.path.join(_HERE, "liboracle_q.so")

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
# kinds that only exist in the general construction (window + quadrature W)
GENERAL_ONLY = ("yukawa2d", "quasi2d_ddi")

BUILD_CMD = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
             _SRC, "-o", _LIB, "-lm"]
# quad-precision oracle of the extended-precision mode (libquadmath)
BUILD_CMD_Q = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11",
               _SRC_Q, "-o", _LIB_Q, "-lquadmath", "-lm"]

_lock = threading.Lock()
_lib = None
_lib_q = None


def build() -> str:
    """Compile the oracle libraries (FP64 and quad) in place; returns the FP64 one's path."""
    subprocess.run(BUILD_CMD, check=True)
    subprocess.run(BUILD_CMD_Q, check=True)
    return _LIB


def _load_q():
    global _lib_q
    with _lock:
        if _lib_q is not None:
            return _lib_q
        if (not os.path.exists(_LIB_Q)
                or os.path.getmtime(_LIB_Q) < os.path.getmtime(_SRC_Q)):
            subprocess.run(BUILD_CMD_Q, check=True)
        lib = ctypes.CDLL(_LIB_Q)
        P = ctypes.c_void_p
        lib.orcq_solve.restype = ctypes.c_int
        lib.orcq_solve.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, P, P, P, P]
        lib.orcq_fft1d.restype = ctypes.c_int
        lib.orcq_fft1d.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
        _lib_q = lib
        return lib


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.c_double
        I = ctypes.c_int
        L = ctypes.c_long
        P = ctypes.c_void_p
        sig = {
            "orc_set_threads": (I, [I]),
            "orc_ein": (D, [D]),
            "orc_e1": (D, [D]),
            "orc_u": (D, [I, D, D]),
            "orc_ueps": (D, [I, D, D, D]),
            "orc_what": (D, [I, D, D, D]),
            "orc_kernel_dim": (I, [I]),
            "orc_fft1d": (I, [I, P, P, I]),
            "orc_fftnd": (I, [I, P, P, I]),
            "orc_build_tensor": (I, [I, D, D, I, P, P, P, P, P, P]),
            "orc_build_tensor_g": (I, [I, D, D, I, I, P, P, P, P, P, P]),
            "orc_solve_g": (I, [I, D, D, I, I, P, P, P, P]),
            "orc_solve_ddi_g": (I, [D, I, P, P, P, P, P, P]),
            "orc_solve_q2d": (I, [D, D, P, P, P, P, P]),
            "orc_windowed": (I, [I]),
            "orc_k0": (D, [D]),
            "orc_k0e": (D, [D]),
            "orc_j0": (D, [D]),
            "orc_k0_vec": (None, [L, P, P]),
            "orc_k0e_vec": (None, [L, P, P]),
            "orc_j0_vec": (None, [L, P, P]),
            "orc_u_any_vec": (None, [I, D, L, P, P]),
            "orc_ueps_general_vec": (None, [I, D, D, L, P, P]),
            "orc_what_general_vec": (None, [I, D, D, L, P, P]),
            "orc_conv_direct": (I, [I, P, P, P, P]),
            "orc_conv_direct_points": (I, [I, P, P, P, L, P, P]),
            "orc_conv_fft": (I, [I, P, P, P, P]),
            "orc_solve": (I, [I, D, D, I, P, P, P, P]),
            "orc_solve_ddi": (I, [D, P, P, P, P, P, P]),
            "orc_ueps_vec": (None, [I, D, D, L, P, P]),
            "orc_what_vec": (None, [I, D, D, L, P, P]),
            "orc_u_vec": (None, [I, D, L, P, P]),
            "orc_e1_vec": (None, [L, P, P]),
            "orc_ein_vec": (None, [L, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def set_threads(n: int) -> int:
    """Set the OpenMP thread count (n <= 0 keeps it); returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def _kind(kind) -> int:
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def _vec(fn, kind, x, *params):
    x = _f64(x)
    out = np.empty_like(x)
    fn(_kind(kind), *params, x.size, _p(x), _p(out))
    return out


def ueps(kind, r, eps, lam=0.0) -> np.ndarray:
    """Far-field smooth kernel U^eps(r) (Table 1; eqs. KerAppr, lnrAppr)."""
    r = _f64(r)
    out = np.empty_like(r)
    _load().orc_ueps_vec(_kind(kind), float(lam), float(eps), r.size, _p(r), _p(out))
    return out


def what(kind, k, eps, lam=0.0) -> np.ndarray:
    """Whole-space transform of U - U^eps at radial wavenumber k (Table 1)."""
    k = _f64(k)
    out = np.empty_like(k)
    _load().orc_what_vec(_kind(kind), float(lam), float(eps), k.size, _p(k), _p(out))
    return out


def u(kind, r, lam=0.0) -> np.ndarray:
    r = _f64(r)
    out = np.empty_like(r)
    _load().orc_u_vec(_kind(kind), float(lam), r.size, _p(r), _p(out))
    return out


def e1(x) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_e1_vec(x.size, _p(x), _p(out))
    return out


def ein(x) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_ein_vec(x.size, _p(x), _p(out))
    return out


def fft1d(x, sign: int = -1) -> np.ndarray:
    """The oracle's own unnormalised mixed-radix FFT of one complex vector."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    out = np.empty_like(x)
    rc = _load().orc_fft1d(x.size, _p(x), _p(out), int(sign))
    if rc:
        raise RuntimeError(f"orc_fft1d failed ({rc})")
    return out


def fftnd(a, sign: int = -1) -> np.ndarray:
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    shape = _i64(a.shape)
    rc = _load().orc_fftnd(a.ndim, _p(shape), _p(a), int(sign))
    if rc:
        raise RuntimeError(f"orc_fftnd failed ({rc})")
    return a


def _par(kind, lam, eta):
    """The kernel parameter the C oracle takes: eta for the quasi-2D DDI, else lambda."""
    if kind == "quasi2d_ddi" or kind == KINDS["quasi2d_ddi"]:
        return float(eta)
    return float(lam)


def k0(x) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_k0_vec(x.size, _p(x), _p(out))
    return out


def k0e(x) -> np.ndarray:
    """e^x K0(x)."""
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_k0e_vec(x.size, _p(x), _p(out))
    return out


def j0(x) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_j0_vec(x.size, _p(x), _p(out))
    return out


def windowed(kind) -> bool:
    """Whether the general construction needs the window xi for this kind."""
    return bool(_load().orc_windowed(_kind(kind)))


def u_any(kind, r, lam=0.0, eta=None) -> np.ndarray:
    r = _f64(r)
    out = np.empty_like(r)
    _load().orc_u_any_vec(_kind(kind), _par(kind, lam, eta), r.size, _p(r), _p(out))
    return out


def ueps_general(kind, r, eps, lam=0.0, eta=None) -> np.ndarray:
    """U^eps = U erf(r/eps) (1 - xi(r)) of the general construction (eq. GeneralApprox1)."""
    r = _f64(r)
    out = np.empty_like(r)
    _load().orc_ueps_general_vec(_kind(kind), _par(kind, lam, eta), float(eps), r.size,
                                 _p(r), _p(out))
    return out


def what_general(kind, k, eps, lam=0.0, eta=None) -> np.ndarray:
    """W(k) by quadrature of the radial transform (eq. Fourier-Symmetric)."""
    k = _f64(k)
    out = np.empty_like(k)
    _load().orc_what_general_vec(_kind(kind), _par(kind, lam, eta), float(eps), k.size,
                                 _p(k), _p(out))
    return out


def build_tensor(kind, L, N, eps, lam=0.0, parts=False, general=False, eta=None):
    """T on the periodic grid prod_j 2N_j (C order, n_j stored at n_j mod 2N_j).

    ``general`` selects the general construction (window + quadrature W);
    the yukawa2d and quasi2d_ddi kinds always use it.  With ``parts=True``
    returns (T, T1, T2, max|Im T2|).
    """
    L = _f64(L)
    N = _i64(N)
    d = L.size
    shape = tuple(int(2 * n) for n in N)
    T = np.empty(shape, dtype=np.float64)
    T1 = np.empty(shape, dtype=np.float64) if parts else None
    T2 = np.empty(shape, dtype=np.float64) if parts else None
    imax = ctypes.c_double(0.0)
    rc = _load().orc_build_tensor_g(
        _kind(kind), _par(kind, lam, eta), float(eps), int(bool(general)), d, _p(L), _p(N),
        _p(T),
        _p(T1) if parts else None, _p(T2) if parts else None,
        ctypes.cast(ctypes.pointer(imax), ctypes.c_void_p))
    if rc:
        raise ValueError(f"orc_build_tensor rejected the arguments ({rc})")
    if parts:
        return T, T1, T2, imax.value
    return T


def conv_direct(T, rho) -> np.ndarray:
    rho = _f64(rho)
    T = _f64(T)
    N = _i64(rho.shape)
    phi = np.empty_like(rho)
    rc = _load().orc_conv_direct(rho.ndim, _p(N), _p(T), _p(rho), _p(phi))
    if rc:
        raise ValueError(f"orc_conv_direct failed ({rc})")
    return phi


def conv_direct_points(T, rho, flat_idx) -> np.ndarray:
    rho = _f64(rho)
    T = _f64(T)
    idx = _i64(flat_idx)
    N = _i64(rho.shape)
    out = np.empty(idx.size, dtype=np.float64)
    rc = _load().orc_conv_direct_points(rho.ndim, _p(N), _p(T), _p(rho), idx.size,
                                         _p(idx), _p(out))
    if rc:
        raise ValueError(f"orc_conv_direct_points failed ({rc})")
    return out


def conv_fft(T, rho) -> np.ndarray:
    rho = _f64(rho)
    T = _f64(T)
    N = _i64(rho.shape)
    phi = np.empty_like(rho)
    rc = _load().orc_conv_fft(rho.ndim, _p(N), _p(T), _p(rho), _p(phi))
    if rc:
        raise ValueError(f"orc_conv_fft failed ({rc})")
    return phi


def solve_ddi(L, N, rho, eps, n, m, general=False) -> np.ndarray:
    """3D dipole-dipole potential -(m.n) rho - 3 Coulomb(d_nm rho) (Sec. 5.3),
    d_nm rho by the periodic spectral derivative on the grid."""
    L = _f64(L)
    N = _i64(N)
    rho = _f64(rho)
    n = _f64(n)
    m = _f64(m)
    phi = np.empty_like(rho)
    rc = _load().orc_solve_ddi_g(float(eps), int(bool(general)), _p(L), _p(N), _p(n), _p(m),
                                 _p(rho), _p(phi))
    if rc:
        raise ValueError(f"orc_solve_ddi rejected the arguments ({rc})")
    return phi


def solve_q2d(L, N, rho, eps, eta, n) -> np.ndarray:
    """Quasi-2D dipole-dipole potential U~ conv [-(3/2)(d_{n_perp n_perp} -
    n_3^2 Lap_perp) rho] (Sec. 5.3), the derivative spectral on the grid."""
    L = _f64(L)
    N = _i64(N)
    rho = _f64(rho)
    n = _f64(n)
    phi = np.empty_like(rho)
    rc = _load().orc_solve_q2d(float(eps), float(eta), _p(L), _p(N), _p(n), _p(rho), _p(phi))
    if rc:
        raise ValueError(f"orc_solve_q2d rejected the arguments ({rc})")
    return phi


def solve(kind, L, N, rho, eps, lam=0.0, general=False, eta=None) -> np.ndarray:
    """Phi on the grid: build T, then the FFT route of eq. DiscConv."""
    L = _f64(L)
    N = _i64(N)
    rho = _f64(rho)
    phi = np.empty_like(rho)
    rc = _load().orc_solve_g(_kind(kind), _par(kind, lam, eta), float(eps),
                             int(bool(general)), L.size, _p(L), _p(N), _p(rho), _p(phi))
    if rc:
        raise ValueError(f"orc_solve rejected the arguments ({rc})")
    return phi


def grid_axes(L, N):
    """Grid coordinates x_j = -L_j + i h_j, i in [0, N_j) (eq. UniformMesh)."""
    return [(-float(l) + np.arange(int(n)) * (2.0 * float(l) / int(n))) for l, n in zip(L, N)]


# --------------------------------------------------------------------------- #
# Quad precision (Coulomb kernels), double-double pairs in and out            #
# --------------------------------------------------------------------------- #

def solve_quad(kind, L, N, rho_dd, eps) -> np.ndarray:
    """Phi in quadruple precision (fsa_oracle_q.c) for the 3D / 2D Coulomb
    kernels; ``rho_dd`` has shape N + (2,) (hi, lo pairs), so has the result."""
    L = _f64(L)
    N = _i64(N)
    rho = _f64(rho_dd)
    if rho.shape != tuple(int(n) for n in N) + (2,):
        raise ValueError("rho_dd must have shape N + (2,)")
    phi = np.empty_like(rho)
    rc = _load_q().orcq_solve(_kind(kind), float(eps), L.size, _p(L), _p(N), _p(rho), _p(phi))
    if rc:
        raise ValueError(f"orcq_solve rejected the arguments ({rc})")
    return phi


def fft1d_quad(x_dd, sign: int = -1) -> np.ndarray:
    """The quad oracle's own FFT of one complex vector given as (re_hi, re_lo,
    im_hi, im_lo) rows."""
    x = _f64(x_dd)
    out = np.empty_like(x)
    rc = _load_q().orcq_fft1d(x.shape[0], _p(x), _p(out), int(sign))
    if rc:
        raise RuntimeError(f"orcq_fft1d failed ({rc})")
    return out
