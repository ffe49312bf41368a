"""Exact rational-arithmetic brute force for tiny inputs (test pins only).

Every quantity is a fractions.Fraction, so results are exact: no rounding,
no library routine.  Used to pin the float64 oracle:

* the Kronecker product by its entry definition
  (A (x) B)[(a, b), (i, j)] = A[a, i] B[b, j] with row-major multi-indices;
* Gaussian elimination for A x = b;
* conjugate gradients in exact arithmetic, which for an SPD n x n matrix
  reaches the exact solution after at most n steps (finite termination).
"""
from fractions import Fraction
from itertools import product


def frac_matrix(m):
    return [[Fraction(v) for v in row] for row in m]


def kron(a, b):
    ra, ca, rb, cb = len(a), len(a[0]), len(b), len(b[0])
    out = [[Fraction(0)] * (ca * cb) for _ in range(ra * rb)]
    for i, j, k, l in product(range(ra), range(ca), range(rb), range(cb)):
        out[i * rb + k][j * cb + l] = a[i][j] * b[k][l]
    return out


def add(a, b):
    return [[x + y for x, y in zip(ra, rb)] for ra, rb in zip(a, b)]


def add_diag(a, d):
    out = [list(r) for r in a]
    for i in range(len(out)):
        out[i][i] += d[i]
    return out


def matvec(a, x):
    return [sum((aij * xj for aij, xj in zip(row, x)), Fraction(0)) for row in a]


def dot(x, y):
    return sum((a * b for a, b in zip(x, y)), Fraction(0))


def solve(a, b):
    n = len(a)
    m = [list(a[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if m[r][c] != 0)
        m[c], m[piv] = m[piv], m[c]
        for r in range(n):
            if r != c and m[r][c] != 0:
                f = m[r][c] / m[c][c]
                m[r] = [x - f * y for x, y in zip(m[r], m[c])]
    return [m[i][n] / m[i][i] for i in range(n)]


def cg(a, b, steps):
    """Exact CG iterates x_0 = 0, x_1, ..., stopping early at r = 0."""
    n = len(b)
    x = [Fraction(0)] * n
    r = list(b)
    p = list(r)
    rho = dot(r, r)
    xs = [list(x)]
    for _ in range(steps):
        if rho == 0:
            break
        q = matvec(a, p)
        alpha = rho / dot(p, q)
        x = [xi + alpha * pi for xi, pi in zip(x, p)]
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        rho_new = dot(r, r)
        beta = rho_new / rho
        p = [ri + beta * pi for ri, pi in zip(r, p)]
        rho = rho_new
        xs.append(list(x))
    return xs
