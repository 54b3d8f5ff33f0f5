"""The solver kernels' exp and erf polynomials (paper_2406_07441_amd/csrc/
lskum_math_coef.h): the header holds what its generator writes, and the
polynomials, evaluated step by step as the kernels do (each fused
multiply-add rounded once), stay within two units in the last place of mpmath's 50-digit exp and erf over the reduced
range and beyond."""
import math
import os
from fractions import Fraction
import re
import subprocess
import sys

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
mp.mp.dps = 50

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2406_07441_amd", "csrc")


def coef():
    text = open(os.path.join(CSRC, "lskum_math_coef.h")).read()
    out = {}
    for name, body in re.findall(r"constexpr double (\w+)\[\d+\] = \{([^}]*)\}", text):
        out[name] = [float.fromhex(v.strip()) for v in body.split(",")]
    for name, v in re.findall(r"constexpr double (\w+) = ([^;]+);", text):
        out[name] = float.fromhex(v.strip())
    return out


def test_header_is_generated():
    text = open(os.path.join(CSRC, "lskum_math_coef.h")).read()
    gen = subprocess.run([sys.executable, os.path.join(CSRC, "gen_lskum_math.py")],
                         capture_output=True, text=True, check=True).stdout
    assert gen == text


def ulp(x):
    return math.ulp(abs(x)) if x != 0 else math.ulp(0.0)


def fma(a, b, c):
    """a * b + c rounded once, as the kernels' fused multiply-add."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp_poly(x, c):
    # the kernels' steps: k = rint(x log2 e), r by two fused steps, Horner by
    # fused steps, 1 + fma(r^2, q, r), scaled by 2^k
    k = float(np.rint(x * c["kLog2e"]))
    r = fma(-k, c["kLn2Hi"], x)
    r = fma(-k, c["kLn2Lo"], r)
    q = c["kExpQ"][0]
    for a in c["kExpQ"][1:]:
        q = fma(q, r, a)
    return math.ldexp(1.0 + fma(r * r, q, r), int(k))


def erf_poly(x, c):
    t = x * x
    p = c["kErfP"][0]
    for a in c["kErfP"][1:]:
        p = fma(p, t, a)
    return x * p


def test_exp_polynomial():
    c = coef()
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-0.35, 0.35, 4000), rng.uniform(-40, 5, 4000),
                         rng.uniform(-700, 700, 2000), [0.0, -1e-300, 1e-12, -0.3465, 0.3465]])
    worst = 0.0
    for x in xs:
        ref = float(mp.exp(mp.mpf(float(x))))
        got = exp_poly(float(x), c)
        worst = max(worst, abs(got - ref) / ulp(ref))
    assert worst <= 2.0, worst


def test_erf_polynomial():
    c = coef()
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-1, 1, 8000), [0.0, 1e-200, -1e-8, 0.5, -0.999999]])
    worst = 0.0
    for x in xs:
        ref = float(mp.erf(mp.mpf(float(x))))
        got = erf_poly(float(x), c)
        worst = max(worst, abs(got - ref) / ulp(ref))
    assert worst <= 2.0, worst
