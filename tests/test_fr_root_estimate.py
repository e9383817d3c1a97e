"""The f(R) sweeps' root of the cubic (Sect. 3.11, n = 1) on the GPU: the closed form of
each case is evaluated in FP32 and polished by two FP64 Newton steps (fr.hip, root3 and
newton3). These CPU checks pin the two numerical facts that scheme rests on, with the
coefficients read from the kernel source so that the test follows the code:

* the trigonometric case takes g(s) = cos(arccos(s) / 3) on [0, 1] from a degree-5
  polynomial; its relative error stays below 1e-6;
* from an estimate with a relative error of 2e-6 (the polynomial plus FP32 rounding),
  two Newton steps on u^3 + p u + q land within a few FP64 ulp of the largest root for
  q < 0 in every case (p > 0, p < 0 with one real root, three real roots).
"""
import os
import re

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_2410_20501_amd", "csrc", "fr.hip")


def _poly_coeffs():
    text = open(SRC).read()
    start = text.index("float g = ")
    block = text[start:text.index("return newton3", start)]
    lead = float(re.search(r"float g = (-?[0-9.]+)f;", block).group(1))
    rest = [float(x) for x in re.findall(r"g = fmaf\(g, sf, (-?[0-9.]+)f\);", block)]
    return [lead] + rest  # highest degree first


def _largest_root(p, q):
    """Largest real root by numpy's companion-matrix solver (FP64), one case at a time."""
    out = np.empty_like(p)
    for i in range(len(p)):
        r = np.roots([1.0, 0.0, p[i], q[i]])
        out[i] = r[np.abs(r.imag) < 1e-9 * max(1.0, abs(r).max())].real.max()
    return out


def test_polynomial_for_the_trigonometric_root():
    c = _poly_coeffs()
    assert len(c) == 6
    s = np.linspace(0.0, 1.0, 200001)
    g = np.cos(np.arccos(s) / 3.0)
    err = np.abs(np.polyval(c, s) / g - 1.0).max()
    assert err < 1e-6, err


@pytest.mark.parametrize("case", ["p_pos", "one_real", "three_real"])
def test_two_newton_steps_reach_fp64(case):
    rng = np.random.Generator(np.random.PCG64(11))
    m = 4000
    ap = 10.0 ** rng.uniform(-6, 6, m)
    qmax = 2.0 * (ap / 3.0) ** 1.5        # |q| bound of three real roots when p < 0
    if case == "p_pos":
        p, q = ap, -10.0 ** rng.uniform(-12, 9, m)
    elif case == "one_real":
        p, q = -ap, -qmax * (1.0 + 10.0 ** rng.uniform(-3, 3, m))
    else:
        p, q = -ap, -qmax * rng.uniform(1e-6, 1.0, m)
    r = _largest_root(p, q)
    # an estimate off by up to 2e-6 either way, then the kernel's two steps
    u = r * (1.0 + rng.uniform(-2e-6, 2e-6, m))
    for _ in range(2):
        f = (u * u + p) * u + q
        u = u - f / (3.0 * u * u + p)
    rel = np.abs(u / r - 1.0)
    assert rel.max() < 2e-14, rel.max()
