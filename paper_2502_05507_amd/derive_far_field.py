"""Derive the far-field (large |n|) expansion of the sigma = 0 lattice Green's function.

Run:  python -m paper_2502_05507_amd.derive_far_field      (needs sympy; about 30 s)

The LGF of Sec. 2.2 is the inverse Fourier transform of 1/sigma(theta),
sigma(theta) = 6 - 2 sum cos(theta_i) = |theta|^2 - A4 + A6 - A8 + ...,
A4 = sum theta_i^4 / 12, A6 = sum theta_i^6 / 360, A8 = sum theta_i^8 / 20160.
Expanding 1/sigma = 1/|theta|^2 (1 - e)^-1, e = (A4 - A6 + A8)/|theta|^2, and collecting terms
of equal homogeneity gives P(theta)/|theta|^(2k) pieces; theta^alpha -> (-i d)^alpha and
|theta|^(-2k) -> f_k with -Lap f_k = f_(k-1), f_1 = 1/(4 pi r):
  f_2 = -r/(8 pi), f_3 = r^3/(96 pi), f_4 = -r^5/(2880 pi).
The script checks that the first two corrections are the paper's q = 2 and q = 3 terms (the
latter with -228, see the reading of the printed -288) and prints the q = 4 term used by the
LGF-sum kernel, as a polynomial in p1 = |n|^2, e2 = j^2k^2 + k^2l^2 + l^2j^2, e3 = j^2k^2l^2.
"""
import sympy as sp


def main():
    x, y, z = sp.symbols("x y z", real=True)
    r = sp.sqrt(x * x + y * y + z * z)
    pi = sp.pi
    f2, f3, f4 = -r / (8 * pi), r ** 3 / (96 * pi), -r ** 5 / (2880 * pi)

    def S(f, p):
        return sum(sp.diff(f, v, p) for v in (x, y, z))

    X, Y, Z = x * x, y * y, z * z
    p1, e2, e3 = X + Y + Z, X * Y + Y * Z + Z * X, X * Y * Z
    q2 = sp.Rational(1, 12) * S(f2, 4)
    P4 = p1 ** 2 - 5 * e2
    assert sp.simplify(q2 - P4 / (16 * pi * r ** 7)) == 0
    q3 = sp.Rational(1, 360) * S(f2, 6) + sp.Rational(1, 144) * S(S(f3, 4), 4)
    P8 = 23 * p1 ** 4 - 336 * p1 ** 2 * e2 + 1155 * e2 ** 2 - 1134 * p1 * e3
    assert sp.simplify(q3 - P8 / (128 * pi * r ** 13)) == 0
    q4 = (sp.Rational(1, 20160) * S(f2, 8) + sp.Rational(2, 4320) * S(S(f3, 4), 6)
          + sp.Rational(1, 1728) * S(S(S(f4, 4), 4), 4))
    P12 = sp.expand(sp.simplify(q4 * 512 * pi * r ** 19))
    a = sp.symbols("a0:7")
    cand = (a[0] * p1 ** 6 + a[1] * p1 ** 4 * e2 + a[2] * p1 ** 2 * e2 ** 2 + a[3] * e2 ** 3
            + a[4] * p1 ** 3 * e3 + a[5] * p1 * e2 * e3 + a[6] * e3 ** 2)
    sol = sp.solve(sp.Poly(sp.expand(cand - P12), x, y, z).coeffs(), a)
    print("q = 4 term: P12 / (512 pi |n|^19) with P12 =",
          " + ".join(f"({sol[a[i]]})*{m}" for i, m in enumerate(
              ["p1^6", "p1^4 e2", "p1^2 e2^2", "e2^3", "p1^3 e3", "p1 e2 e3", "e3^2"])))


if __name__ == "__main__":
    main()
