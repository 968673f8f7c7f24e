"""Exact rational brute force for tiny inputs (test helper).

Every float32/float64 input is a dyadic rational, so ``Fraction(x)`` is exact
and the sums below are the mathematically exact value of each definition.
These restate textbook definitions directly (Bernstein sum, Cox-de Boor
basis recursion, tensor triple sum); they are independent of the oracle's
algorithms (de Casteljau, peeling, de Boor, separable contraction).
"""
from fractions import Fraction
from math import comb


def F(x):
    return Fraction(float(x))


def bernstein(d, i, t):
    return comb(d, i) * (1 - t) ** (d - i) * t ** i


def bezier(b, t):
    """Exact Bezier value sum_i C(d,i) (1-t)^(d-i) t^i b_i."""
    d = len(b) - 1
    return sum(bernstein(d, i, t) * b[i] for i in range(d + 1))


def rational(b, w, t):
    d = len(b) - 1
    num = sum(bernstein(d, i, t) * w[i] * b[i] for i in range(d + 1))
    den = sum(bernstein(d, i, t) * w[i] for i in range(d + 1))
    return num / den


def bspline_basis(U, i, p, u):
    """Cox-de Boor recursion N_{i,p}(u) with the 0/0 = 0 convention and
    half-open spans [U_i, U_{i+1})."""
    if p == 0:
        return Fraction(1) if U[i] <= u < U[i + 1] else Fraction(0)
    a = Fraction(0)
    if U[i + p] != U[i]:
        a = (u - U[i]) / (U[i + p] - U[i]) * bspline_basis(U, i, p - 1, u)
    b = Fraction(0)
    if U[i + p + 1] != U[i + 1]:
        b = (U[i + p + 1] - u) / (U[i + p + 1] - U[i + 1]) * bspline_basis(U, i + 1, p - 1, u)
    return a + b


def nurbs(P, w, U, p, u):
    """Exact NURBS point sum N_i w_i P_i / sum N_i w_i (u strictly inside)."""
    n = len(w)
    N = [bspline_basis(U, i, p, u) for i in range(n)]
    den = sum(N[i] * w[i] for i in range(n))
    return [sum(N[i] * w[i] * P[k][i] for i in range(n)) / den for k in range(len(P))]


def tensor(P, du, dv, dw, u, v, w):
    """Exact triple sum over the tensor-product Bernstein basis; P is a flat
    list indexed (i*(dv+1)+j)*(dw+1)+k."""
    acc = Fraction(0)
    for i in range(du + 1):
        for j in range(dv + 1):
            for k in range(dw + 1):
                acc += bernstein(du, i, u) * bernstein(dv, j, v) * bernstein(dw, k, w) * \
                    P[(i * (dv + 1) + j) * (dw + 1) + k]
    return acc
