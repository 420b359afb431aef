"""The kernels' complementary error function (half-range Maxwellian moments,
Sec. 2.1) against a 40-digit evaluation, on the CPU.

The FP64 and FP32 kernels form erfc(z) = exp(-z^2) p(t) / (1 + 2|z|) with
t = (|z| - K) / (|z| + K) and erfc(-a) = 2 - erfc(a); K and the coefficients
of p are read from the kernel header.  The formula is evaluated here in the
kernel's type with products and sums rounded separately (the kernels fuse
them), and compared with mpmath's erfc.
"""
import os
import re

import mpmath as mp
import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1901_00261_amd", "csrc", "gks_math.h")


def header_table(name):
    src = open(HDR).read()
    body = re.search(name + r"\[\d+\] = \{([^}]*)\}", src).group(1)
    return [float(x.strip().rstrip("f")) for x in body.split(",") if x.strip()]


def header_const(name):
    return float(re.search(name + r" = ([0-9.]+)f?;", open(HDR).read()).group(1))


def kernel_erfc(z, c, K, ft, q=None):
    """erfc(z) as the kernel forms it, in type ft; q = exp(-z^2) (40 digits
    when not given, so that only p and the mapping are tested)."""
    z = ft(z)
    a = abs(z)
    if q is None:
        q = ft(float(mp.exp(-mp.mpf(float(a)) ** 2)))
    one, two, k = ft(1), ft(2), ft(K)
    b = two * a + one
    r = one / ((a + k) * b)
    t = (a - k) * b * r
    w = (a + k) * r
    t2 = t * t
    ev = ft(c[(len(c) - 1) // 2 * 2])
    for j in range((len(c) - 1) // 2 * 2 - 2, -1, -2):
        ev = ft(ev * t2 + ft(c[j]))
    jo = (len(c) - 2) // 2 * 2 + 1
    od = ft(c[jo])
    for j in range(jo - 2, 0, -2):
        od = ft(od * t2 + ft(c[j]))
    v = q * ((od * t + ev) * w)
    return two - v if z < 0 else v


mp.mp.dps = 40


@pytest.mark.parametrize("ft,tab,kname,bar", [(np.float64, "kErfcP64", "kErfcK64", 4.0),
                                            (np.float32, "kErfcP32", "kErfcK32", 4.0)])
def test_erfc_against_40_digits(ft, tab, kname, bar):
    c, K = header_table(tab), header_const(kname)
    eps, tiny = float(np.finfo(ft).eps), float(np.finfo(ft).tiny)
    zs = np.concatenate([np.linspace(-6, 27, 1651), -np.geomspace(1e-9, 6, 200), np.geomspace(1e-9, 27, 400), [0.0]])
    worst_pos = worst_neg = 0.0
    for z in zs.astype(ft):
        got = float(kernel_erfc(z, c, K, ft))
        want = mp.erfc(mp.mpf(float(z)))
        if z >= 0 and want < 2 * tiny:
            # exp(-z^2) and erfc(z) below the normal range (z > 9.3 in FP32,
            # 26.6 in FP64): no relative precision to keep
            assert abs(got - want) <= 2 * tiny
        elif z >= 0:
            # relative to erfc itself: the scaled function's error carries over
            worst_pos = max(worst_pos, float(abs(got - want) / want) / eps)
        else:
            # erfc(z) in (1, 2): 2 - v rounds once more
            worst_neg = max(worst_neg, float(abs(got - want) / want) / eps)
    print(f"{ft.__name__}: worst {worst_pos:.2f} ulp (z >= 0), {worst_neg:.2f} ulp (z < 0)")
    assert worst_pos <= bar and worst_neg <= bar


def test_erfc_limits_and_symmetry():
    """erfc(0) = 1, erfc(z) + erfc(-z) = 2, and exp(a^2) erfc(a) -> 1/(a sqrt(pi))."""
    c, K = header_table("kErfcP64"), header_const("kErfcK64")
    assert abs(kernel_erfc(0.0, c, K, np.float64) - 1.0) <= 2e-16
    for a in (1e-6, 0.3, 1.7, 4.0, 9.5):
        s = kernel_erfc(a, c, K, np.float64) + kernel_erfc(-a, c, K, np.float64)
        assert abs(s - 2.0) <= 4e-16
    a = 1e6  # far outside the fitted range: the mapping's limit t -> 1 still holds
    scaled = kernel_erfc(a, c, K, np.float64, q=np.float64(1.0))
    assert abs(scaled * a * np.sqrt(np.pi) - 1.0) <= 1e-6
