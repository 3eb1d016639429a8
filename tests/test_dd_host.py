"""The double-double arithmetic of the extended-precision mode
(`csrc/fsa_dd.hpp`), compiled for the host with g++ and checked against mpmath
at 50 digits (no GPU).  The device code includes the same header."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dd_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("dd") / "dd_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(ROOT, "tests", "host", "dd_check.cpp"),
                    "-o", exe], check=True)
    return exe


def _split(v):
    import mpmath as mp
    hi = float(v)
    return hi, float(v - mp.mpf(hi))


def _run(exe, op, xs, ys=None):
    import mpmath as mp
    lines, ins = [], []
    for i, x in enumerate(xs):
        xh, xl = _split(x)
        yh, yl = _split(ys[i]) if ys is not None else (0.0, 0.0)
        lines.append(f"{op} {xh.hex()} {xl.hex()} {yh.hex()} {yl.hex()}")
        ins.append((mp.mpf(xh) + mp.mpf(xl), mp.mpf(yh) + mp.mpf(yl)))
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    res = [[float.fromhex(t) for t in l.split()] for l in out if l.strip()]
    return ins, res


def _worst(ins, res, f, two=False):
    import mpmath as mp
    worst = 0.0
    for (x, y), r in zip(ins, res):
        ref = f(x, y)
        if two:
            for (h, l), rr in zip(((r[0], r[1]), (r[2], r[3])), ref):
                worst = max(worst, float(abs(mp.mpf(h) + mp.mpf(l) - rr)))
        else:
            worst = max(worst, float(abs(mp.mpf(r[0]) + mp.mpf(r[1]) - ref) / abs(ref)))
    return worst


@pytest.mark.parametrize("op,f,lo,hi,bound", [
    ("add", lambda x, y: x + y, 0.1, 5, 4e-32),
    ("mul", lambda x, y: x * y, 0.1, 5, 4e-32),
    ("div", lambda x, y: x / y, 0.1, 5, 4e-32),
    ("sqrt", lambda x, y: __import__("mpmath").sqrt(x), 0.1, 50, 4e-32),
    ("exp", lambda x, y: __import__("mpmath").exp(x), -90, 90, 4e-32),
    ("expm1", lambda x, y: __import__("mpmath").expm1(x), -0.45, 0.45, 1e-31),
    ("erf", lambda x, y: __import__("mpmath").erf(x), 0.001, 9.4, 5e-31),
])
def test_dd_functions(dd_exe, op, f, lo, hi, bound):
    import mpmath as mp
    mp.mp.dps = 50
    rng = np.random.default_rng(abs(hash(op)) % 1000)
    xs = [mp.mpf(float(v)) / 3 for v in rng.uniform(3 * lo, 3 * hi, 60)]
    ys = [mp.mpf(float(v)) / 7 for v in rng.uniform(0.7, 35, 60)]
    ins, res = _run(dd_exe, op, xs, ys)
    assert _worst(ins, res, f) <= bound


def test_dd_sincos_turns(dd_exe):
    """cos and sin of 2 pi m / 4096 (the twiddles and the DCT table) in every
    octant, to 5e-32 absolute."""
    import mpmath as mp
    mp.mp.dps = 50
    fs = [mp.mpf(m) / 4096 for m in list(range(0, 4096, 37)) + [512, 1024, 2048, 4095]]
    ins, res = _run(dd_exe, "sincos", fs)
    worst = _worst(ins, res, lambda f, _: (mp.sin(2 * mp.pi * f), mp.cos(2 * mp.pi * f)),
                   two=True)
    assert worst <= 5e-32
