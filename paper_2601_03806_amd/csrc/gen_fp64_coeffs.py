#!/usr/bin/env python3
"""Print the double-precision constants of gmf_math.hpp from their definitions.

The logarithm and the sine/cosine of 2 pi r behind the FP64 Box-Muller
transform are evaluated as polynomials on reduced arguments:
* ln m = s P(s^2),  s = (m - 1)/(m + 1),  |s| <= 3 - 2 sqrt 2, where
  P(z) ~ 2 artanh(sqrt z) / sqrt z = sum_k 2 z^k / (2k + 1);
* sin(2 pi r) = r S(r^2),  S(z) ~ sin(2 pi sqrt z) / sqrt z,
  cos(2 pi r) = C(r^2),    C(z) ~ cos(2 pi sqrt z),  |r| <= 1/8, z <= 1/64.
Each polynomial is the minimax approximation of least relative error of its
degree (the Remez exchange algorithm: E. Ya. Remez, 1934), with the degree the
smallest whose relative error is at most 2^-53, one unit of a double's
relative precision.  The target functions are summed from their Taylor series
with 60-digit decimal arithmetic (pi from Machin's formula); every constant is
rounded to a double once.  ln 2 is split into a high part with 32 significant
bits (e * LN2_HI is exact for |e| < 2^21) and the remainder.
"""
from decimal import Decimal, getcontext
from fractions import Fraction
import math

getcontext().prec = 60
TARGET = Decimal(2) ** -53
GRID = 1000       # points of the error scan on the interval
ITERATIONS = 10   # exchange steps


def pi_decimal():
    # Machin: pi = 16 atan(1/5) - 4 atan(1/239)
    def atan_inv(n):
        x = Decimal(1) / n
        x2 = x * x
        s, term, k = Decimal(0), x, 0
        while abs(term) > Decimal(10) ** -58:
            s += term / (2 * k + 1) * (-1 if k % 2 else 1)
            term *= x2
            k += 1
        return s
    return 16 * atan_inv(5) - 4 * atan_inv(239)


TWOPI = 2 * pi_decimal()


def series(coef, z):
    """sum_k coef(k) z^k for 0 <= z < 1 with terms decreasing past the third"""
    s, zk, k = Decimal(0), Decimal(1), 0
    while True:
        t = coef(k) * zk
        s += t
        if k > 2 and abs(t) < Decimal(10) ** -55:
            return s
        zk *= z
        k += 1


def factorial(n):
    r = Decimal(1)
    for i in range(2, n + 1):
        r *= i
    return r


def f_log(z):   # 2 artanh(sqrt z) / sqrt z
    return series(lambda k: Decimal(2) / (2 * k + 1), z)


def f_sin(z):   # sin(2 pi sqrt z) / sqrt z
    return series(lambda k: (-1) ** k * TWOPI ** (2 * k + 1) / factorial(2 * k + 1), z)


def f_cos(z):   # cos(2 pi sqrt z)
    return series(lambda k: (-1) ** k * TWOPI ** (2 * k) / factorial(2 * k), z)


def solve(A, b):
    """Gaussian elimination with partial pivoting"""
    n = len(b)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        p = max(range(c, n), key=lambda r: abs(M[r][c]))
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c:
                f = M[r][c] / M[c][c]
                for k in range(c, n + 1):
                    M[r][k] -= f * M[c][k]
    return [M[i][n] / M[i][i] for i in range(n)]


def horner(c, z):
    s = Decimal(0)
    for a in reversed(c):
        s = s * z + a
    return s


def remez(f, a, b, n):
    """Coefficients of the degree-n polynomial of least maximum relative error
    to f on [a, b], and that error (measured on the scan grid)."""
    # start from the Chebyshev extrema; each step solves
    # P(z_i) - f(z_i) = (-1)^i E f(z_i) on the reference and moves the
    # reference to the alternating extrema of the relative error
    ref = [a + (b - a) * (1 - Decimal(math.cos(math.pi * i / (n + 1)))) / 2 for i in range(n + 2)]
    zs = [a + (b - a) * Decimal(i) / GRID for i in range(GRID + 1)]
    fz = [f(z) for z in zs]
    c, worst = None, None
    for _ in range(ITERATIONS):
        A, rhs = [], []
        for i, z in enumerate(ref):
            v = f(z)
            A.append([Decimal(1) if j == 0 else z ** j for j in range(n + 1)] + [Decimal((-1) ** i) * v])
            rhs.append(v)
        c = solve(A, rhs)[:-1]
        err = [(horner(c, z) - v) / v for z, v in zip(zs, fz)]
        worst = max(abs(e) for e in err)
        ext = []
        for i, e in enumerate(err):
            left = abs(err[i - 1]) if i > 0 else Decimal(-1)
            right = abs(err[i + 1]) if i < GRID else Decimal(-1)
            if abs(e) >= left and abs(e) >= right:
                if ext and (ext[-1][1] > 0) == (e > 0):
                    if abs(e) > abs(ext[-1][1]):
                        ext[-1] = (zs[i], e)
                else:
                    ext.append((zs[i], e))
        while len(ext) > n + 2:
            ext.pop(0 if abs(ext[0][1]) < abs(ext[-1][1]) else -1)
        if len(ext) < n + 2:
            break
        ref = [z for z, _ in ext]
    return c, worst


def minimax(f, a, b, start):
    """the lowest degree from start up whose relative error is within TARGET"""
    n = start
    while True:
        c, e = remez(f, a, b, n)
        if e <= TARGET:
            return c
        n += 1


def hexd(x):
    return float(x).hex()


def main():
    ln2 = Decimal(2).ln()
    smax = Decimal(3) - 2 * Decimal(2).sqrt()
    logc = minimax(f_log, Decimal(0), smax * smax, 5)
    sinc = minimax(f_sin, Decimal(0), Decimal(1) / 64, 5)
    cosc = minimax(f_cos, Decimal(0), Decimal(1) / 64, 5)
    ln2_hi = float(Fraction(int(float(ln2) * 2 ** 32), 2 ** 32))   # 32 significant bits
    ln2_lo = float(ln2 - Decimal(ln2_hi))
    print("// generated by gen_fp64_coeffs.py")
    print(f"constexpr double kLn2Hi = {hexd(ln2_hi)};")
    print(f"constexpr double kLn2Lo = {hexd(ln2_lo)};")
    print(f"constexpr int kLogTerms = {len(logc)};")
    print("constexpr double kLogC[kLogTerms] = {" + ", ".join(hexd(c) for c in logc) + "};")
    print(f"constexpr int kSinTerms = {len(sinc)};")
    print("constexpr double kSinC[kSinTerms] = {" + ", ".join(hexd(c) for c in sinc) + "};")
    print(f"constexpr int kCosTerms = {len(cosc)};")
    print("constexpr double kCosC[kCosTerms] = {" + ", ".join(hexd(c) for c in cosc) + "};")


if __name__ == "__main__":
    main()
