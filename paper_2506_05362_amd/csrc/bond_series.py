"""Coefficients of the bond-law polynomial used by the step kernels.

The bond force of Sec. 3.1 needs g(x) = 1 - (1 + x)^(-1/2) with
x = (|y|^2 - |xi|^2) / |xi|^2.  For |x| <= 0.02 the kernels evaluate
g = x * q(x) with q a degree-8 polynomial: the interpolant of
q(x) = (1 - (1 + x)^(-1/2)) / x at the nine Chebyshev nodes of [-0.02, 0.02],
computed here in 80-digit decimal arithmetic.  Its constant term is exactly
1/2; with the other eight coefficients rounded to double its relative error
on the interval is about 1e-18 (the ten-term Taylor series: 3.5e-18).

    python paper_2506_05362_amd/csrc/bond_series.py
prints the coefficients (highest degree first, as C hex literals) and the
error of the rounded polynomial on a 801-point grid.
"""
from decimal import Decimal as D, getcontext

getcontext().prec = 80
R = D("0.02")
N = 9
PI = D("3.14159265358979323846264338327950288419716939937510582097494459230781640628620899")


def q(x):
    if abs(x) < D(10) ** -20:
        return D("0.5") - D(3) * x / 8
    return (1 - 1 / (1 + x).sqrt()) / x


def cos(t):
    s, term, k = D(0), D(1), 0
    while abs(term) > D(10) ** -75:
        s += term
        term = -term * t * t / ((2 * k + 1) * (2 * k + 2))
        k += 1
    return s


def solve(A, b):
    n = len(b)
    for c in range(n):
        p = max(range(c, n), key=lambda i: abs(A[i][c]))
        A[c], A[p], b[c], b[p] = A[p], A[c], b[p], b[c]
        for i in range(c + 1, n):
            f = A[i][c] / A[c][c]
            for j in range(c, n):
                A[i][j] -= f * A[c][j]
            b[i] -= f * b[c]
    x = [D(0)] * n
    for i in reversed(range(n)):
        x[i] = (b[i] - sum(A[i][j] * x[j] for j in range(i + 1, n))) / A[i][i]
    return x


def coefficients():
    xs = [R * cos((2 * k + 1) * PI / (2 * N)) for k in range(N)]
    return solve([[x ** j for j in range(N)] for x in xs], [q(x) for x in xs])


def max_rel_error(cs):
    worst = D(0)
    for k in range(-400, 401):
        x = R * k / 400
        p = D(0)
        for c in reversed(cs):
            p = p * x + c
        worst = max(worst, abs(p - q(x)) / q(x))
    return worst


if __name__ == "__main__":
    co = coefficients()
    rounded = [D(float(c)) for c in co]
    print("constant term:", float(co[0]))
    print("c8..c1:", ", ".join(float(c).hex() for c in reversed(co[1:])))
    print("max relative error, rounded coefficients: %.3e" % max_rel_error(rounded))
