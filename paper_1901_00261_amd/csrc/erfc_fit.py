"""Coefficients of the complementary error function used by the half-range
Maxwellian moments (Sec. 2.1) in the FP64 and FP32 kernels.

For a >= 0 the kernels evaluate erfc(a) = exp(-a^2) p(t) / (1 + 2a) with
t = (a - K) / (a + K), which maps [0, inf) onto [-1, 1): the scaled function
g(a) = (1 + 2a) exp(a^2) erfc(a) runs from 1 at a = 0 to 2/sqrt(pi) as
a -> inf and is analytic in t on [-1, 1], so a polynomial in t converges
geometrically (the mapping of J. L. Schonfelder, "Chebyshev expansions for
the error and related functions", Math. Comp. 32 (1978)).  p interpolates g
at the Chebyshev points of [-1, 1] in 50-digit arithmetic (mpmath); its
monomial coefficients are rounded to the kernel's type.  The script then
evaluates the kernel's formula in that type (even and odd parts in t^2,
combined at the end) over a in [0, 30] and prints the worst relative error
against the 50-digit erfc.

Usage: python erfc_fit.py    (prints both tables and their errors)
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 50

# (type, K, degree): the lowest degrees within 3 ulp over [0, 30]
FITS = ((np.float64, 3, 24), (np.float32, 2, 10))


def scaled(t, K):
    t = mp.mpf(t)
    if t == 1:
        return 2 / mp.sqrt(mp.pi)
    a = K * (1 + t) / (1 - t)
    return (1 + 2 * a) * mp.erfc(a) * mp.exp(a * a)


def fit(K, deg):
    n = deg + 1
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]
    A = mp.matrix([[x ** j for j in range(n)] for x in nodes])
    c = mp.lu_solve(A, mp.matrix([scaled(x, K) for x in nodes]))
    return [c[j] for j in range(n)]


def kernel_scaled(a, c, K, ft):
    """exp(a^2) erfc(a) as the kernels form it for a >= 0, in type ft: the
    even and odd parts of p as Horner chains in t^2, p = even + t odd, times
    1 / (1 + 2a).  Products and sums round separately here (the kernels fuse
    them, one rounding fewer), so the printed error is an upper estimate."""
    one, two, k = ft(1), ft(2), ft(K)
    b = one + two * a
    r = one / ((a + k) * b)
    t = (a - k) * b * r
    w = (a + k) * r
    t2 = t * t
    ev_idx, od_idx = list(range(0, len(c), 2)), list(range(1, len(c), 2))
    ev, od = c[ev_idx[-1]], c[od_idx[-1]]
    for j in reversed(ev_idx[:-1]):
        ev = ft(ev * t2 + c[j])
    for j in reversed(od_idx[:-1]):
        od = ft(od * t2 + c[j])
    return ft((od * t + ev) * w)


def main():
    for ft, K, deg in FITS:
        c = [ft(float(x)) for x in fit(mp.mpf(K), deg)]
        worst = 0.0
        grid = np.concatenate([np.linspace(0, 30, 6001), np.geomspace(1e-8, 30, 2000)])
        for a in grid.astype(ft):
            sx = kernel_scaled(a, c, K, ft)
            am = mp.mpf(float(a))
            exact = mp.erfc(am) * mp.exp(am * am)
            worst = max(worst, abs(float((mp.mpf(float(sx)) - exact) / exact)))
        name = "double" if ft is np.float64 else "float"
        print(f"// {name}: K = {K}, degree {deg}; worst relative error of exp(a^2) erfc(a) "
              f"{worst / np.finfo(ft).eps:.2f} ulp over [0, 30]")
        print("{" + ", ".join(repr(float(x)) + ("" if ft is np.float64 else "f") for x in c) + "}")


if __name__ == "__main__":
    main()
