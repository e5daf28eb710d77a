"""Derive, in exact arithmetic, the reconstruction constants hard-coded in gks_stencils.h.

Cells have unit width; cell o spans [o - 1/2, o + 1/2]. For a stencil of cells, the polynomial whose
cell averages match the data is evaluated (or differentiated) at a point xi of the centre cell.
Gauss points are xi = s sqrt(3)/6 (s = -1, +1), so every weight has the form e + s sqrt(3) o with
rational e and o. Run: python derive_stencils.py  (prints the constants; nothing imports it).
"""
from fractions import Fraction as Fr


def avg_monomial(o, p):
    return (Fr(2 * o + 1, 2) ** (p + 1) - Fr(2 * o - 1, 2) ** (p + 1)) / (p + 1)


def solve(M, b):
    n = len(b)
    A = [row[:] + [b[i]] for i, row in enumerate(M)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[i][n] / A[i][i] for i in range(n)]


def weights(offsets, vec):
    """w with sum_r w_r qbar_r = sum_p a_p vec_p where a solves the cell-average system."""
    deg = len(offsets) - 1
    At = [[avg_monomial(o, p) for o in offsets] for p in range(deg + 1)]  # A^T
    return solve(At, vec)


def point_vec(deg, xi_pows, deriv):
    """vec_p = d^deriv/dxi^deriv xi^p at the point, given xi^k for k = 0..deg."""
    v = []
    for p in range(deg + 1):
        if p < deriv:
            v.append(Fr(0))
        else:
            coef = 1
            for q in range(deriv):
                coef *= (p - q)
            v.append(coef * xi_pows[p - deriv])
    return v


def gauss_split(offsets, deriv):
    """Weights at xi = s sqrt(3)/6 as (even part e, odd part o): w = e + s sqrt(3) o."""
    deg = len(offsets) - 1
    # xi^k = (sqrt3/6)^k s^k: even k rational 1/12^(k/2); odd k = s sqrt3 * (1/6) (1/12)^((k-1)/2)
    even = [Fr(1, 12) ** (k // 2) if k % 2 == 0 else Fr(0) for k in range(deg + 1)]
    odd = [Fr(0) if k % 2 == 0 else Fr(1, 6) * Fr(1, 12) ** ((k - 1) // 2) for k in range(deg + 1)]
    e = weights(offsets, point_vec(deg, even, deriv))
    o = weights(offsets, point_vec(deg, odd, deriv))
    return e, o


def main():
    sub = [(-2, -1, 0), (-1, 0, 1), (0, 1, 2)]
    half = [Fr(1) / 2 ** k for k in range(5)]
    print("face xi=+1/2 substencils:", [[str(w) for w in weights(s, point_vec(2, half, 0))] for s in sub])
    mh = [Fr(-1, 2) ** k for k in range(5)]
    print("face xi=-1/2 substencils:", [[str(w) for w in weights(s, point_vec(2, mh, 0))] for s in sub])
    print("normal derivative (cells -1..2 at xi=1/2):",
          [str(w) for w in weights((-1, 0, 1, 2), point_vec(3, half, 1))])
    for s in sub:
        e, o = gauss_split(s, 0)
        print("gauss substencil", s, "even", [str(x) for x in e], "odd", [str(x) for x in o])
    e, o = gauss_split((-2, -1, 0, 1, 2), 0)
    print("gauss quartic value even", [str(x) for x in e], "odd", [str(x) for x in o])
    e, o = gauss_split((-2, -1, 0, 1, 2), 1)
    print("gauss quartic derivative even", [str(x) for x in e], "odd", [str(x) for x in o])


if __name__ == "__main__":
    main()
