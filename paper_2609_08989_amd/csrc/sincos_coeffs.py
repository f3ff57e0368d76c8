"""Derives the polynomial coefficients of sincos64 (fastmath.hpp) and of the
angle shift from a step's start (kShift64).

sin(r)/r and cos(r) are series in z = r^2.  On |r| <= pi/4 (z <= 0.61686) the
Taylor series are truncated far beyond double precision, re-expanded in
Chebyshev polynomials of the interval in exact rational arithmetic, and the
Chebyshev series is cut at degree 6 (sin) and 7 (cos) in z ("economization",
Lanczos).  The printed bound is the sum of the dropped Chebyshev coefficients,
a bound on the absolute truncation error of the economized polynomial.

    python sincos_coeffs.py
"""
import math
from fractions import Fraction as F

ZMAX = F(61686, 100000)          # >= (pi/4)^2 = 0.616850...


def taylor(first_odd, nterms):
    # first_odd: sin(r)/r = sum (-1)^k z^k/(2k+1)!; else cos(r) = sum (-1)^k z^k/(2k)!
    return [F((-1) ** k, math.factorial(2 * k + (1 if first_odd else 0))) for k in range(nterms)]


def economize(c, deg, zmax=ZMAX):
    n = len(c)
    # z = zmax (t + 1) / 2: coefficients in t
    pt = [F(0)] * n
    for k, ck in enumerate(c):
        s = (zmax / 2) ** k
        for j in range(k + 1):
            pt[j] += ck * s * math.comb(k, j)
    # t^j -> Chebyshev T_m
    ch = [F(0)] * n
    for j, a in enumerate(pt):
        for i in range(j + 1):
            ch[abs(j - 2 * i)] += a * F(math.comb(j, i), 2 ** j)
    bound = sum(abs(x) for x in ch[deg + 1:])
    # back to monomials in t, then in z
    T = [[F(1)], [F(0), F(1)]]
    for m in range(2, deg + 1):
        nxt = [F(0)] * (m + 1)
        for i, v in enumerate(T[m - 1]):
            nxt[i + 1] += 2 * v
        for i, v in enumerate(T[m - 2]):
            nxt[i] -= v
        T.append(nxt)
    mt = [F(0)] * (deg + 1)
    for m in range(deg + 1):
        for i, v in enumerate(T[m]):
            mt[i] += ch[m] * v
    mz = [F(0)] * (deg + 1)
    for i, a in enumerate(mt):
        for j in range(i + 1):
            mz[j] += a * math.comb(i, j) * (F(2) / zmax) ** j * (-1) ** (i - j)
    return mz, bound


# The angle shift (sincos_shift in kerr.hpp) evaluates sin(d)/d and cos(d) on
# |d| <= 1/16 (z <= 1/256), degrees 3 and 4 in z; their z^0 and z^1
# coefficients round to 1 and -1/2 exactly, and the code takes them so.
ZMAX_SHIFT = F(1, 256)

if __name__ == "__main__":
    for name, odd, deg, zmax in (("sin(r)/r", True, 6, ZMAX), ("cos(r)", False, 7, ZMAX),
                                 ("sin(d)/d (shift)", True, 3, ZMAX_SHIFT), ("cos(d) (shift)", False, 4, ZMAX_SHIFT)):
        mz, bound = economize(taylor(odd, 14), deg, zmax)
        print(f"{name}: degree {deg} in z, truncation bound {float(bound):.2e}")
        for k, v in enumerate(mz):
            print(f"  z^{k}: {float(v):.17g}")
