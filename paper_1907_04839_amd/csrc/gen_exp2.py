"""Coefficients of the FP64 2^f polynomial used by the pair kernels.

2^f on [-1/2, 1/2] is interpolated at the 12 Chebyshev points of the first
kind (degree 11); the interpolant is converted to monomial form by solving
the Vandermonde system in 60-digit decimal arithmetic and rounded to FP64.
The interpolation error bound max|d^12/df^12 2^f| / (2^11 12!) (1/2)^12 is
below 5e-18, far under one FP64 ulp.  Run as a script to print the C++
table that shoot_kernels.hip holds; tests check that the two agree.
"""
from __future__ import annotations

from decimal import Decimal, getcontext

DEGREE = 11


def coefficients(degree: int = DEGREE) -> list[float]:
    getcontext().prec = 60
    pi = Decimal("3.14159265358979323846264338327950288419716939937510582097494")
    ln2 = Decimal(2).ln()

    def cos(x: Decimal) -> Decimal:           # Taylor series, |x| <= pi
        s, term, k = Decimal(1), Decimal(1), 0
        while True:
            k += 2
            term = -term * x * x / (k * (k - 1))
            if abs(term) < Decimal(10) ** -58:
                return s + term
            s += term

    n = degree + 1
    xs = [Decimal("0.5") * cos(pi * (Decimal(k) + Decimal("0.5")) / n) for k in range(n)]
    ys = [(x * ln2).exp() for x in xs]
    # Vandermonde system V c = y, Gaussian elimination with partial pivoting
    A = [[x ** j for j in range(n)] + [y] for x, y in zip(xs, ys)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(A[r][col]))
        A[col], A[piv] = A[piv], A[col]
        for r in range(col + 1, n):
            f = A[r][col] / A[col][col]
            for c in range(col, n + 1):
                A[r][c] -= f * A[col][c]
    c = [Decimal(0)] * n
    for r in range(n - 1, -1, -1):
        c[r] = (A[r][n] - sum(A[r][k] * c[k] for k in range(r + 1, n))) / A[r][r]
    return [float(v) for v in c]


def cpp_table(coef: list[float]) -> str:
    body = ",\n".join(f"    {v!r}" for v in coef)
    return ("constexpr double kExp2Poly[" + str(len(coef)) + "] = {\n" + body + "};\n")


if __name__ == "__main__":
    print(cpp_table(coefficients()), end="")
